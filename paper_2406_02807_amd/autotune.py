"""Autotuner for the collision kernels' launch shape.

Searches `capt_tuning` (wavefronts per workgroup, persistent workgroups per
CU, configurations per queue pop, tree levels in LDS, set-scan steps in
flight) by coordinate descent on the caller's own workload, timing each
candidate with HIP events on the current stream.  Every candidate's answers
must equal the first candidate's bit for bit (the launch shape never changes
an answer); a mismatch raises.  The winner is applied with `capt_set_tuning`
and can be cached in a JSON file keyed by a workload signature.

`autotune_step` tunes the same knobs for a caller-defined step instead of a
lone query launch (for example double-buffered frames, where the query shares
the chip with the next frame's filter and build and the best shape leaves
room for them), timed by wall clock with the device synchronised.
"""
from __future__ import annotations

import json
import os
import time

from . import capt_collides, capt_get_tuning, capt_set_tuning

SPACE = {
    "waves_per_group": [4, 8, 12, 16],
    "groups_per_cu": [1, 2, 3, 4, 6],
    "tile_cfgs": [16, 64, 256],
    "lds_levels": [12, 13, 14, 15],
    "scan_unroll": [1, 2, 4],
}


def _time_once(fn, reps):
    import torch
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def signature(forest, spheres, group, query_off) -> str:
    infos = [forest.info(c) for c in range(forest.ncloud)]
    return json.dumps({"clouds": forest.ncloud,
                       "D": sorted({i["D"] for i in infos}),
                       "entries": sum(i["set_total"] for i in infos),
                       "spheres": int(spheres.shape[0]), "group": int(group),
                       "batched": forest.ncloud > 1}, sort_keys=True)


def autotune(forest, spheres, group, query_off=None, flags=0, space=None, reps=3, rounds=2,
             cache=None, verbose=False):
    """Tune for this workload; returns (best tuning dict, list of (tuning, ms))."""
    import torch
    cache = cache or os.environ.get("CAPT_TUNE_CACHE")
    key = signature(forest, spheres, group, query_off)
    if cache and os.path.exists(cache):
        try:
            stored = json.load(open(cache)).get(key)
        except (OSError, ValueError):
            stored = None
        if stored:
            capt_set_tuning(**stored)
            return stored, []
    space = dict(SPACE if space is None else space)
    if forest.ncloud == 1:
        space.pop("tile_cfgs", None)      # single clouds do not use the tile queue shape
    out = torch.empty(spheres.shape[0] // group, dtype=torch.uint8, device=spheres.device)
    ref = None
    best = capt_get_tuning()
    history = []

    def run(t):
        capt_set_tuning(**t)

        def fn():
            capt_collides(forest, spheres, group, query_off=query_off, flags=flags, out=out)
        fn()                                   # warm-up (and graph capture for forests)
        torch.cuda.synchronize()
        ms = _time_once(fn, reps)
        return ms

    best_ms = run(best)
    ref = out.clone()
    history.append((dict(best), best_ms))
    for _ in range(rounds):
        improved = False
        for name, values in space.items():
            for v in values:
                if best[name] == v:
                    continue
                cand = dict(best)
                cand[name] = v
                t0 = time.perf_counter()
                ms = run(cand)
                if not torch.equal(out, ref):
                    capt_set_tuning(**best)
                    raise RuntimeError(f"launch shape {cand} changed an answer")
                history.append((cand, ms))
                if verbose:
                    print(f"  {cand} {ms:.3f} ms ({time.perf_counter() - t0:.2f} s)", flush=True)
                if ms < best_ms * 0.99:
                    best, best_ms, improved = cand, ms, True
        if not improved:
            break
    capt_set_tuning(**best)
    if cache:
        try:
            data = json.load(open(cache)) if os.path.exists(cache) else {}
        except (OSError, ValueError):
            data = {}
        data[key] = best
        with open(cache, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    return best, history


STEP_SPACE = {
    "waves_per_group": [8, 12, 14, 16],
    "groups_per_cu": [1, 2, 3, 4],
    "lds_levels": [12, 13, 14],
    "scan_unroll": [1, 2, 4],
}


def autotune_step(step, answers, space=None, reps=5, rounds=2, verbose=False):
    """Coordinate descent over the launch shape for `step()` (any host code
    that runs the workload and returns when it is queued); `answers()` returns
    the tensor of results, which must not change with the shape.  Each
    candidate's cost is the median wall time of `reps` synchronised runs; at
    the end the winner and the starting shape are timed again with twice the
    repetitions and the faster one is kept, so one noisy median cannot move
    the choice.  Returns (best tuning dict, list of (tuning, ms))."""
    import torch
    space = dict(STEP_SPACE if space is None else space)

    def run(t):
        capt_set_tuning(**t)
        step()                                  # warm-up
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            step()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        ts.sort()
        return ts[len(ts) // 2]

    best = capt_get_tuning()
    best_ms = run(best)
    ref = answers().clone()
    history = [(dict(best), best_ms)]
    for _ in range(rounds):
        improved = False
        for name, values in space.items():
            for v in values:
                if best[name] == v:
                    continue
                cand = dict(best)
                cand[name] = v
                ms = run(cand)
                if not torch.equal(answers(), ref):
                    capt_set_tuning(**best)
                    raise RuntimeError(f"launch shape {cand} changed an answer")
                history.append((cand, ms))
                if verbose:
                    print(f"  {cand} {ms:.3f} ms", flush=True)
                if ms < best_ms * 0.99:
                    best, best_ms, improved = cand, ms, True
        if not improved:
            break
    start = history[0][0]
    if best != start:
        reps *= 2
        t_best, t_start = run(best), run(start)
        history.append((dict(best), t_best))
        history.append((dict(start), t_start))
        if t_start <= t_best:
            best = start
    capt_set_tuning(**best)
    return best, history
