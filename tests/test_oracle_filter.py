"""Pins for the oracle's Morton keys and Filter (Alg. 2, Sec. IV-C).

- Morton keys against hand-derived closed forms;
- the quantisation grid at its corners;
- a 1-D cloud, where every permutation orders points by x and Alg. 2 reduces
  to the textbook greedy cover of a sorted line (computed here with integers);
- r_filter above the diameter keeps exactly the first point of the first
  curve; r_filter = 0 drops only exact duplicates;
- the filter's guarantee (Sec. IV-C, Lemma 2's proof): every dropped point has
  a kept point within r_filter in its own pass, hence within 6 r_filter of the
  final cloud (chaining over the six passes).
"""
import numpy as np
import pytest

from conftest import golden


def test_morton_closed_forms(orc):
    for case in golden("morton_and_predicates.json")["morton"]:
        assert orc.morton_key(case["q"], case["perm"]) == case["key"], case


def test_morton_key_is_a_bijection_on_small_grid(orc):
    keys = {orc.morton_key([x, y, z], 2) for x in range(8) for y in range(8) for z in range(8)}
    assert keys == set(range(512))


def test_morton_grid_corners(orc):
    pts = np.array([[-1, 2, 0], [3, 2.5, 1], [1, 2.25, 0.5]], dtype=np.float32)
    lo, scale = orc.morton_grid(pts)
    assert lo.tolist() == [-1, 2, 0]
    assert scale == 2 ** 21 / 4.0
    assert orc.morton_cell(pts[0], lo, scale).tolist() == [0, 0, 0]
    # the top corner clamps to 2^21 - 1 on the longest axis
    assert orc.morton_cell(pts[1], lo, scale).tolist() == [2 ** 21 - 1, 2 ** 18, 2 ** 19]
    assert orc.morton_cell(pts[2], lo, scale).tolist() == [2 ** 20, 2 ** 17, 2 ** 18]
    # a degenerate cloud (zero extent) puts every point in cell 0
    same = np.ones((4, 3), np.float32)
    lo1, s1 = orc.morton_grid(same)
    assert s1 == 0.0 and orc.morton_cell(same[0], lo1, s1).tolist() == [0, 0, 0]


def _greedy_line(xs, rf2_int):
    kept = [0]
    for j in range(1, len(xs)):
        if (xs[j] - xs[kept[-1]]) ** 2 > rf2_int:
            kept.append(j)
    return kept


@pytest.mark.parametrize("rf", [0.5, 2.5, 7.0, 30.0])
def test_line_cloud_is_textbook_greedy_cover(orc, rf):
    rng = np.random.default_rng(int(rf * 10))
    xs = np.sort(rng.choice(5000, 700, replace=False))
    pts = np.stack([xs, np.zeros_like(xs), np.zeros_like(xs)], 1).astype(np.float32)
    perm = rng.permutation(len(pts))
    kept, counts = orc.filter(pts[perm], rf)
    got = sorted(perm[kept].tolist())
    # integers: (dx)^2 > rf^2 evaluated exactly; fl(rf*rf) is exact for these rf
    want = _greedy_line(xs.tolist(), rf * rf)
    assert got == want
    assert counts[0] == len(want) and (counts == len(want)).all()


def test_radius_above_diameter_keeps_first_point_of_first_curve(orc):
    rng = np.random.default_rng(2)
    pts = rng.random((500, 3)).astype(np.float32)
    kept, counts = orc.filter(pts, 10.0)
    lo, scale = orc.morton_grid(pts)
    keys = [orc.morton_key(orc.morton_cell(p, lo, scale), 0) for p in pts]
    first = min(range(len(pts)), key=lambda j: (keys[j], j))
    assert kept.tolist() == [first] and counts.tolist() == [1] * 6


def test_zero_radius_drops_only_duplicates(orc):
    rng = np.random.default_rng(4)
    base = (rng.choice(4096, size=(300, 3)) / 4096.0).astype(np.float32)
    base = np.unique(base, axis=0)
    pts = np.concatenate([base, base[:100], base[:50]])
    pts = pts[rng.permutation(len(pts))]
    kept, _ = orc.filter(pts, 0.0)
    assert len(kept) == len(base)
    assert len(np.unique(pts[kept], axis=0)) == len(base)


def test_empty_and_single(orc):
    assert orc.filter(np.zeros((0, 3), np.float32), 0.01)[0].tolist() == []
    assert orc.filter(np.ones((1, 3), np.float32), 0.01)[0].tolist() == [0]


def _cover_radius(src, dst):
    """max over src of the distance to the nearest dst point (float64)."""
    best = np.full(len(src), np.inf)
    for s in range(0, len(dst), 2048):
        d = np.sqrt(((src[:, None, :].astype(np.float64) - dst[None, s:s + 2048, :]) ** 2).sum(-1))
        best = np.minimum(best, d.min(1))
    return best.max() if len(src) else 0.0


@pytest.mark.parametrize("rf", [0.01, 0.03])
def test_per_pass_and_overall_cover(orc, rf):
    import synth
    pts = synth.tabletop_cloud(6000, 77)
    prev = np.arange(len(pts))
    for npass in range(1, 7):
        kept, _ = orc.filter(pts, rf, npass=npass)
        assert set(kept.tolist()) <= set(prev.tolist())
        dropped = np.setdiff1d(prev, kept)
        # every point dropped in this pass is within r_f of a point it kept
        # (slack for the float32 predicate)
        assert _cover_radius(pts[dropped], pts[kept]) <= rf * (1 + 1e-5)
        prev = kept
    assert _cover_radius(pts, pts[prev]) <= 6 * rf * (1 + 1e-5)
    # kept points are pairwise farther than r_f along the final curve
    d = np.sqrt(((pts[prev][1:].astype(np.float64) - pts[prev][:-1]) ** 2).sum(-1))
    assert (d > rf * (1 - 1e-5)).all()
    assert len(np.unique(prev)) == len(prev)


def test_presorted_passes_equal_iterated_sorts(orc):
    """Each pass's order is "key of the pass, then original index", whatever
    the earlier passes did: every permutation's key is a bijection of the grid
    cell, so a tie under one key is a tie under all of them and the stable
    sorts keep ties in index order.  The survivors of a pass in that order are
    the full sorted list with the dead points skipped.  Here the filter is
    recomputed that way (all six orders fixed up front, liveness flags) and
    must give the oracle's answer, order and per-pass counts included; the
    cloud holds exact duplicates and near-duplicates so that ties occur."""
    rng = np.random.default_rng(77)
    base = rng.random((600, 3)).astype(np.float32)
    pts = np.concatenate([base, base[:150], base[:40] + np.float32(1e-7), rng.random((400, 3)).astype(np.float32)])
    pts = pts[rng.permutation(len(pts))]
    lo, scale = orc.morton_grid(pts)
    cells = [orc.morton_cell(p, lo, scale) for p in pts]
    for rf in (0.0, 0.01, 0.05):
        rf2 = np.float32(rf) * np.float32(rf)
        live = np.ones(len(pts), bool)
        counts = []
        order = None
        for p in range(6):
            keys = [orc.morton_key(c.tolist(), p) for c in cells]
            order = sorted(range(len(pts)), key=lambda i: (keys[i], i))
            last = None
            nxt = np.zeros(len(pts), bool)
            for i in order:
                if not live[i]:
                    continue
                if last is None or orc.sqdist_f32(pts[last], pts[i]) > rf2:
                    nxt[i] = True
                    last = i
            live = nxt
            counts.append(int(live.sum()))
        mine = [i for i in order if live[i]]
        want, want_counts = orc.filter(pts, rf)
        assert mine == want.tolist(), rf
        assert counts == want_counts.tolist(), rf
