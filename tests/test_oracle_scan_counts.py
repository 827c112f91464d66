"""Pins for the parts of the oracle that the benchmark's byte counts and its
CPU baseline rest on:

- CollisionCheck's per-sphere scan count m_s (Alg. 3, Sec. IV-D) against
  counts worked by hand on the golden five-point tree (first, middle and last
  stored position of the first hit, a miss, an AABB rejection), against the
  position of the first hit found by testing the leaf's stored points one at
  a time with brute force, and on sets given in reversed order;
- the single-thread CollisionCheck with per-configuration early exit against
  brute force (a different function: the plain definition) on groups whose
  only colliding sphere is the first, a middle or the last one, or none;
- the r_min pruning threshold of Construct (Sec. IV-B) at its exact boundary
  r_min^2 (1 - 2^-18) and one float32 step either side.
"""
from fractions import Fraction

import numpy as np
import pytest

from conftest import golden


def test_scan_counts_hand_worked(orc):
    g = golden("tiny_tree.json")
    pts = np.array(g["points"], dtype=np.float32)
    t = orc.build_tree(pts, g["r_min"], g["r_max"], prune=False)
    sph = np.array([q["sphere"] for q in g["queries"]], dtype=np.float32)
    hit, leaf, rej, scanned = orc.query_tree(t, pts, sph)
    for i, q in enumerate(g["queries"]):
        assert leaf[i] == q["leaf"], q
        assert hit[i] == q["hit"], q
        assert rej[i] == q["rejected"], q
        assert scanned[i] == q["scanned"], q
    # the golden cases reach the first, a middle and the last stored position
    # of a hit, a full miss and a rejection
    got = {(int(h), int(s)) for h, s in zip(hit, scanned)}
    assert {(1, 1), (1, 2), (1, 3), (1, 4), (0, 4), (0, 0)} <= got


def _trees():
    rng = np.random.default_rng(31)
    yield "uniform-300", rng.random((300, 3)).astype(np.float32) * np.float32(0.3), 0.01, 0.05
    lat = np.stack(np.meshgrid(*[np.arange(5)] * 3, indexing="ij"), -1).reshape(-1, 3)
    yield "lattice-125", lat.astype(np.float32) * np.float32(0.02), 0.0, 0.03
    yield "dups-120", np.repeat(rng.random((30, 3)), 4, axis=0).astype(np.float32) * np.float32(0.2), 0.01, 0.04


@pytest.mark.parametrize("name,pts,r_min,r_max", list(_trees()), ids=[c[0] for c in _trees()])
def test_scan_count_is_position_of_first_hit(orc, name, pts, r_min, r_max):
    """Independent of the counter: the first hit found by brute force over the
    leaf's stored points, in stored order, sits at position m_s - 1; without
    a hit m_s is the set size; a rejected sphere scans nothing."""
    t = orc.build_tree(pts, r_min, r_max)
    rng = np.random.default_rng(7)
    lo, hi = pts.min(0) - r_max, pts.max(0) + r_max
    cen = lo + rng.random((3000, 3)) * (hi - lo)
    cen = np.concatenate([cen, pts[rng.integers(0, len(pts), 1000)]])
    rad = rng.uniform(max(r_min, 1e-3), r_max, len(cen))
    sph = np.concatenate([cen, rad[:, None]], 1).astype(np.float32)
    hit, leaf, rej, scanned = orc.query_tree(t, pts, sph)
    seen = set()
    for i, q in enumerate(sph):
        ids = t.set_of(leaf[i])
        if rej[i]:
            assert scanned[i] == 0
            continue
        # brute force over the stored points in stored order, one by one
        first = -1
        for k, j in enumerate(ids):
            if orc.brute_f32(pts[j:j + 1], q[None])[0]:
                first = k
                break
        if first < 0:
            assert hit[i] == 0 and scanned[i] == len(ids), i
        else:
            assert hit[i] == 1 and scanned[i] == first + 1, i
            seen.add(min(first, 2))
    assert 0 in seen and len(seen) >= 2    # hits at the first stored position and later ones


def test_scan_counts_on_a_stored_order_replay(orc):
    """orc.query on explicit arrays counts in the order the set is given, not
    in index order: reversing every set moves the first hit."""
    rng = np.random.default_rng(3)
    pts = rng.random((400, 3)).astype(np.float32) * np.float32(0.2)
    t = orc.build_tree(pts, 0.0, 0.04)
    sph = np.concatenate([pts[:200], np.full((200, 1), 0.01)], 1).astype(np.float32)
    hit, leaf, rej, sc = orc.query_tree(t, pts, sph)
    rev = np.concatenate([t.set_of(l)[::-1] for l in range(t.N)]).astype(np.int32)
    hit2, leaf2, rej2, sc2 = orc.query(t.N, t.D, t.T, t.aabb, t.off, pts[rev], sph)
    assert np.array_equal(hit, hit2) and np.array_equal(leaf, leaf2)
    for i in range(len(sph)):
        ids = t.set_of(leaf[i])
        if hit[i]:
            # the same first-hit rule from the other end of the set
            r = ids[::-1]
            k = next(k for k, j in enumerate(r) if orc.brute_f32(pts[j:j + 1], sph[i:i + 1])[0])
            assert sc2[i] == k + 1
    assert (sc != sc2).any()


def _grouped(pts, g, rng):
    """Configurations of g spheres: every sphere misses (radius small, centre
    far from the cloud) except at most one, placed first, in the middle, last,
    or nowhere."""
    far = pts.max(0) + 1.0
    cfgs, want = [], []
    for kind in ("first", "middle", "last", "none") * 25:
        c = np.tile(np.append(far, 0.01), (g, 1))
        c[:, 0] += np.arange(g) * 0.5
        pos = {"first": 0, "middle": g // 2, "last": g - 1, "none": None}[kind]
        if pos is not None:
            p = pts[rng.integers(0, len(pts))]
            c[pos, :3] = p
        cfgs.append(c)
        want.append(pos is not None)
    return np.concatenate(cfgs).astype(np.float32), np.array(want, np.uint8)


@pytest.mark.parametrize("g", [1, 7, 60])
def test_query_serial_early_exit(orc, g):
    rng = np.random.default_rng(g)
    pts = rng.random((2000, 3)).astype(np.float32)
    t = orc.build_tree(pts, 0.01, 0.05)
    sph, want = _grouped(pts, g, rng)
    out = orc.query_serial(t.N, t.D, t.T, t.aabb, t.off, pts[t.idx], sph, g)
    if g > 1:
        assert np.array_equal(out, want)
    assert np.array_equal(out, orc.brute_f32(pts, sph, g))
    # random grouped spheres, about half the configurations colliding
    cen = rng.random((600 * g, 3)) * 1.1 - 0.05
    r = rng.uniform(0.01, 0.05, (600 * g, 1)) * (0.3 if g > 1 else 1.0)
    sph = np.concatenate([cen, r], 1).astype(np.float32)
    out = orc.query_serial(t.N, t.D, t.T, t.aabb, t.off, pts[t.idx], sph, g)
    ref = orc.brute_f32(pts, sph, g)
    assert np.array_equal(out, ref)
    assert 0 < ref.sum() < len(ref)
    # and the per-sphere CollisionCheck, OR-ed per configuration
    assert np.array_equal(out, orc.query_tree(t, pts, sph)[0].reshape(-1, g).max(1))


def _boundary_cell():
    """A bounded cell [-u, 0] x [-v, 0] x [0, 0] with representative t at the
    origin and r_min = 1, so the farthest corner's float64 squared distance
    is fl(fl(u*u) + fl(v*v)) (the zero axis adds 0), searched so that it
    equals fl(1 * 1 * (1 - 2^-18)) exactly."""
    thr = 1.0 * (1.0 - 2.0 ** -18)            # IEEE double product, exact here
    u = np.float32(np.sqrt(thr))
    for _ in range(4000):
        u = np.nextafter(u, np.float32(0))     # below sqrt(thr): a positive remainder for v^2
        uu = float(u) * float(u)               # exact: 24-bit * 24-bit mantissas
        rem = thr - uu
        if rem <= 0:
            continue
        v = np.float32(np.sqrt(rem))
        for vv in (v, np.nextafter(v, np.float32(0)), np.nextafter(v, np.float32(1))):
            if uu + float(vv) * float(vv) == thr:
                return float(u), float(vv), thr
    raise AssertionError("no boundary case found")


def test_prune_threshold_boundary(orc):
    u, v, thr = _boundary_cell()
    # check the construction in exact arithmetic: the double sum rounds to thr
    exact = Fraction(u) ** 2 + Fraction(v) ** 2
    assert abs(exact - Fraction(thr)) <= Fraction(2) ** -53
    t = (0.0, 0.0, 0.0)
    cell = (-u, -v, 0.0, 0.0, 0.0, 0.0)
    assert orc.prunable(cell, t, 1.0), "equality is inside (<=)"
    # one float32 step farther on either axis: outside; nearer: inside
    uo = float(np.nextafter(np.float32(u), np.float32(2)))
    ui = float(np.nextafter(np.float32(u), np.float32(0)))
    vo = float(np.nextafter(np.float32(v), np.float32(2)))
    assert not orc.prunable((-uo, -v, 0.0, 0.0, 0.0, 0.0), t, 1.0)
    assert not orc.prunable((-u, -vo, 0.0, 0.0, 0.0, 0.0), t, 1.0)
    assert orc.prunable((-ui, -v, 0.0, 0.0, 0.0, 0.0), t, 1.0)
    # the farthest corner is per axis: the same extents on the other side
    assert orc.prunable((0.0, 0.0, 0.0, u, v, 0.0), t, 1.0)
    assert not orc.prunable((0.0, 0.0, 0.0, uo, v, 0.0), t, 1.0)
    # r_min one float32 step smaller moves the threshold below the corner,
    # one step larger keeps the corner inside
    assert not orc.prunable(cell, t, float(np.nextafter(np.float32(1), np.float32(0))))
    assert orc.prunable(cell, t, float(np.nextafter(np.float32(1), np.float32(2))))
    # the margin itself: without it (threshold exactly r_min^2) the one-step
    # farther cell would still be inside, so the test above pins 2^-18
    assert float(np.float32(uo)) ** 2 + v * v <= 1.0
    # an unbounded cell or r_min = 0 never prunes
    assert not orc.prunable((-u, -v, -np.inf, 0.0, 0.0, 0.0), t, 1.0)
    assert not orc.prunable((0.0, 0.0, 0.0, 0.0, 0.0, 0.0), t, 0.0)
