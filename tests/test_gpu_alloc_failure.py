"""Allocation failures: with allocator hooks that fail the k-th request, every
entry point that allocates returns CAPT_ENOMEM (never a wrong answer or a
crash) and gives back everything it allocated before the failure, for every
k up to the number of requests a successful run makes."""
import ctypes as C
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def capt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_02807_amd as capt
    capt.load_library()
    return capt


class FailingAt:
    """hipMalloc / hipFree behind the library's allocator hooks; request number
    `fail_at` (1-based) returns NULL.  Tracks the live blocks."""
    ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
    RELEASE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

    def __init__(self, lib, fail_at=None):
        self.lib, self.fail_at = lib, fail_at
        self.hip = C.CDLL("libamdhip64.so")
        self.calls, self.live = 0, {}

        def alloc(nbytes, stream, ctx):
            self.calls += 1
            if self.fail_at is not None and self.calls == self.fail_at:
                return None
            p = C.c_void_p()
            if self.hip.hipMalloc(C.byref(p), C.c_size_t(max(nbytes, 1))) != 0:
                return None
            self.live[p.value] = nbytes
            return p.value

        def release(ptr, stream, ctx):
            # the library hands a block back once its last use is queued on
            # `stream`: wait for that work, then free
            self.hip.hipStreamSynchronize(C.c_void_p(stream))
            self.hip.hipFree(C.c_void_p(ptr))
            self.live.pop(ptr)

        self._a, self._r = self.ALLOC(alloc), self.RELEASE(release)

    def __enter__(self):
        assert self.lib.capt_set_allocator(C.cast(self._a, C.c_void_p), C.cast(self._r, C.c_void_p), None) == 0
        return self

    def __exit__(self, *exc):
        assert self.lib.capt_set_allocator(None, None, None) == 0


def _run(capt, torch, pts, sph, cloud_off, query_off, group):
    """filter of the first cloud, build of all, one query, destroy."""
    f = None
    try:
        capt.capt_filter(pts[:cloud_off[1]], 0.01)
        f = capt.capt_build(pts, 0.015, 0.08, cloud_off=cloud_off)
        out = capt.capt_collides(f, sph, group, query_off=query_off)
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        if f is not None:
            f.close()
        torch.cuda.synchronize()


@pytest.mark.parametrize("nclouds", [1, 3])
def test_every_allocation_failure_is_enomem_and_leaks_nothing(capt, orc, nclouds):
    import torch
    clouds = [synth.tabletop_cloud(3000 + 500 * c, 951 + c) for c in range(nclouds)]
    cloud_off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])])
    tpl = synth.chain_template(2003)
    sph = [synth.posed_spheres(tpl, 40 + 10 * c, synth.WORKSPACE, 961 + c) for c in range(nclouds)]
    query_off = np.concatenate([[0], np.cumsum([len(s) for s in sph])])
    pts = torch.from_numpy(np.concatenate(clouds)).cuda()
    spheres = torch.from_numpy(np.concatenate(sph)).cuda()
    want = np.concatenate([orc.brute_f32(clouds[c], sph[c], 60) for c in range(nclouds)])
    lib = capt.load_library()
    _say(f"case: allocation failures, {nclouds} cloud(s), counting run")
    with FailingAt(lib) as hooks:
        got = _run(capt, torch, pts, spheres, cloud_off, query_off, 60)
    assert np.array_equal(got, want)
    assert hooks.live == {}
    total = hooks.calls
    assert total >= 4
    for k in range(1, total + 1):
        _say(f"case: allocation failures, {nclouds} cloud(s), request {k} of {total} fails")
        with FailingAt(lib, fail_at=k) as hooks:
            with pytest.raises(capt.CaptError) as e:
                _run(capt, torch, pts, spheres, cloud_off, query_off, 60)
        assert e.value.status == capt.CAPT_ENOMEM, (k, str(e.value))
        assert hooks.live == {}, (k, hooks.live)
    # the library works normally afterwards, on its default pool
    assert np.array_equal(_run(capt, torch, pts, spheres, cloud_off, query_off, 60), want)
