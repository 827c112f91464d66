"""Pins for the oracle's Construct (Alg. 1) and CollisionCheck (Alg. 3).

- a hand-worked 5-point tree (T, representatives, cells, sets, AABBs, queries);
- structural invariants of the k-d split (Sec. III, Sec. IV-A);
- every affordance set against the direct, non-recursive definition of
  Lemma 1, case 1, with exact rational arithmetic on small clouds;
- pruned leaves against the exact farthest-corner condition (Sec. IV-B);
- Lemma 1 itself: CollisionCheck equals brute force on random, grid and
  adversarial queries, with and without the AABB step.
"""
from fractions import Fraction

import numpy as np
import pytest

from conftest import fnum, golden


def _clouds():
    rng = np.random.default_rng(5)
    out = {
        "uniform-200": rng.random((200, 3)).astype(np.float32),
        "uniform-37": rng.random((37, 3)).astype(np.float32),
        "lattice-64": np.stack(np.meshgrid(*[np.arange(4)] * 3, indexing="ij"), -1)
                        .reshape(-1, 3).astype(np.float32) * np.float32(0.02),
        "dups-50": np.repeat(rng.random((10, 3)), 5, axis=0).astype(np.float32) * np.float32(0.2),
        "collinear-33": np.stack([np.linspace(0, 0.3, 33), np.zeros(33), np.zeros(33)], 1).astype(np.float32),
        "coplanar-48": np.concatenate([rng.random((48, 2)) * 0.3, np.zeros((48, 1))], 1).astype(np.float32),
        "single": np.array([[0.5, 0.25, 0.125]], dtype=np.float32),
        "pair": np.array([[0, 0, 0], [0.01, 0, 0]], dtype=np.float32),
        "three": rng.random((3, 3)).astype(np.float32),
        "five": rng.random((5, 3)).astype(np.float32) * np.float32(0.1),
        "pow2p1": rng.random((17, 3)).astype(np.float32) * np.float32(0.2),
    }
    return out


CLOUDS = _clouds()


def test_golden_tiny_tree(orc):
    g = golden("tiny_tree.json")
    pts = np.array(g["points"], dtype=np.float32)
    t = orc.build_tree(pts, g["r_min"], g["r_max"], prune=False)
    assert (t.N, t.D) == (g["N"], g["D"])
    assert t.T.tolist() == [fnum(v) for v in g["T"]]
    assert t.rep.tolist() == g["rep"]
    assert t.cell.tolist() == [[fnum(v) for v in c] for c in g["cells"]]
    assert [t.set_of(l).tolist() for l in range(t.N)] == g["sets"]
    assert t.aabb.tolist() == [[fnum(v) for v in a] for a in g["aabb"]]
    for q in g["queries"]:
        sph = np.array([q["sphere"]], dtype=np.float32)
        hit, leaf, rej, scanned = orc.query_tree(t, pts, sph)
        assert leaf[0] == q["leaf"], q
        assert hit[0] == q["hit"], q
        assert orc.brute_f32(pts, sph)[0] == q["hit"]


def _node_points(t, node):
    """Representatives in the subtree of Eytzinger node `node`."""
    lo, hi = node, node
    while lo < t.N - 1:
        lo, hi = 2 * lo + 1, 2 * hi + 2
    return t.rep[lo - (t.N - 1): hi - (t.N - 1) + 1]


@pytest.mark.parametrize("name", sorted(CLOUDS))
def test_structure_invariants(orc, name):
    pts = CLOUDS[name]
    n = len(pts)
    t = orc.build_tree(pts, 0.01, 0.05)
    assert t.N == 1 << t.D and t.N >= n and (t.N == 1 or t.N < 2 * n)
    # every point, real or padding, is the representative of exactly one leaf
    assert sorted(t.rep.tolist()) == list(range(t.N))
    padded = np.concatenate([pts, np.full((t.N - n, 3), np.inf, np.float32)])
    for i in range(t.N - 1):
        depth = int(np.floor(np.log2(i + 1)))
        ax = depth % 3
        left = _node_points(t, 2 * i + 1)
        right = _node_points(t, 2 * i + 2)
        assert len(left) == len(right)
        # lower median of the node under (coordinate, index)
        allp = np.concatenate([left, right])
        order = sorted(allp.tolist(), key=lambda j: (padded[j, ax], j))
        assert set(order[:len(left)]) == set(left.tolist())
        assert t.T[i] == padded[order[len(left) - 1], ax]
        assert (padded[left, ax] <= t.T[i]).all() and (padded[right, ax] >= t.T[i]).all()
    # each leaf's closed cell contains its representative
    for l in range(t.N):
        p = padded[t.rep[l]]
        c = t.cell[l]
        assert (c[:3] <= p).all() and (p <= c[3:]).all()


def _exact_cell_dist2(p, cell):
    d2 = Fraction(0)
    for a in range(3):
        lo, hi, v = float(cell[a]), float(cell[3 + a]), Fraction(float(p[a]))
        if lo == np.inf or hi == -np.inf:
            return None                      # a cell at infinity touches no point
        if np.isfinite(lo) and v < Fraction(lo):
            d2 += (Fraction(lo) - v) ** 2
        elif np.isfinite(hi) and v > Fraction(hi):
            d2 += (v - Fraction(hi)) ** 2
    return d2


@pytest.mark.parametrize("name", ["uniform-37", "lattice-64", "dups-50", "collinear-33",
                                  "coplanar-48", "five", "pow2p1", "three", "pair"])
@pytest.mark.parametrize("radii", [(0.0, 0.05), (0.02, 0.06), (0.05, 0.05)])
def test_sets_match_direct_definition_exactly(orc, name, radii):
    pts = CLOUDS[name]
    r_min, r_max = radii
    t = orc.build_tree(pts, r_min, r_max)
    rmax = Fraction(float(np.float32(r_max)))
    R = rmax * (1 + Fraction(1, 2 ** 20))
    rmin = Fraction(float(np.float32(r_min)))
    for l in range(t.N):
        cell = t.cell[l]
        s = set(t.set_of(l).tolist())
        rep = int(t.rep[l])
        if t.pruned[l]:
            # Sec. IV-B: every point of the (bounded) cell is within r_min of t
            assert rep < len(pts) and s == {rep}
            assert np.isfinite(cell).all()
            far2 = sum(max((Fraction(float(pts[rep, a])) - Fraction(float(cell[a]))) ** 2,
                           (Fraction(float(cell[3 + a])) - Fraction(float(pts[rep, a]))) ** 2)
                       for a in range(3))
            assert far2 <= rmin ** 2
            continue
        for j in range(len(pts)):
            d2 = _exact_cell_dist2(pts[j], cell)
            if d2 is not None and d2 <= rmax ** 2:
                assert j in s, (l, j)          # Lemma 1, case 1: nothing missing
            if j in s:
                assert d2 is not None and d2 <= R ** 2, (l, j)   # nothing beyond the slack
        if rep < len(pts):
            assert rep in s
        # AABB is the exact float32 box of the stored points
        if s:
            sp = pts[sorted(s)]
            assert (t.aabb[l, :3] == sp.min(0)).all() and (t.aabb[l, 3:] == sp.max(0)).all()
        else:
            assert (t.aabb[l, :3] == np.inf).all() and (t.aabb[l, 3:] == -np.inf).all()


def test_no_pruning_when_rmin_zero_or_disabled(orc):
    pts = CLOUDS["lattice-64"]
    assert orc.build_tree(pts, 0.0, 0.05).pruned.sum() == 0
    assert orc.build_tree(pts, 0.02, 0.05, prune=False).pruned.sum() == 0
    # a dense lattice with r_min above the cell diagonal prunes interior cells
    assert orc.build_tree(pts, 0.05, 0.06).pruned.sum() > 0


def test_rmax_above_diameter_gives_whole_cloud(orc):
    pts = CLOUDS["uniform-37"]
    t = orc.build_tree(pts, 0.0, 2.0)
    for l in range(t.N):
        at_inf = (t.cell[l, :3] == np.inf).any() or (t.cell[l, 3:] == -np.inf).any()
        want = [] if at_inf else list(range(len(pts)))
        assert t.set_of(l).tolist() == want
    assert sum(not ((t.cell[l, :3] == np.inf).any()) for l in range(t.N)) >= len(pts)


def test_single_and_empty(orc):
    t = orc.build_tree(CLOUDS["single"], 0.01, 0.05)
    assert (t.N, t.D) == (1, 0) and t.set_of(0).tolist() == [0] and t.pruned[0] == 0
    sph = np.array([[0.5, 0.25, 0.125, 0.01], [0.5, 0.25, 0.171875, 0.05], [0.5, 0.25, 0.3, 0.05]],
                   dtype=np.float32)
    assert orc.query_tree(t, CLOUDS["single"], sph)[0].tolist() == [1, 1, 0]
    e = orc.build_tree(np.zeros((0, 3), np.float32), 0.01, 0.05)
    assert (e.N, e.D, len(e.idx)) == (1, 0, 0)
    assert orc.query_tree(e, np.zeros((0, 3), np.float32), sph)[0].tolist() == [0, 0, 0]


def _adversarial_queries(t, pts, r_min, r_max, rng, m=3000):
    """Centres on split planes, cell corners and cloud points; radii at the
    ends of [r_min, r_max] and in between."""
    qs = []
    finite_cells = np.where(np.isfinite(t.cell), t.cell, 0.0)
    for l in rng.integers(0, t.N, m // 3):
        c = finite_cells[l]
        corner = np.where(rng.random(3) < 0.5, c[:3], c[3:])
        qs.append(corner)
    for j in rng.integers(0, len(pts), m // 3):
        qs.append(pts[j].astype(np.float64))
    for i in rng.integers(0, max(t.N - 1, 1), m // 3):
        if t.N == 1:
            break
        q = pts[rng.integers(0, len(pts))].astype(np.float64)
        depth = int(np.floor(np.log2(i + 1)))
        if np.isfinite(t.T[i]):
            q[depth % 3] = t.T[i]
        qs.append(q)
    qs = np.array(qs)
    radii = rng.choice([r_min, r_max, 0.5 * (r_min + r_max)], len(qs))
    radii = np.where(radii <= 0, r_max, radii)
    return np.concatenate([qs, radii[:, None]], 1).astype(np.float32)


@pytest.mark.parametrize("name", sorted(CLOUDS))
def test_lemma1_capt_equals_brute_force(orc, name):
    pts = CLOUDS[name]
    rng = np.random.default_rng(hash(name) % 2 ** 32)
    for r_min, r_max in [(0.01, 0.05), (0.0, 0.03), (0.02, 0.02)]:
        t = orc.build_tree(pts, r_min, r_max)
        lo = pts.min(0) - 0.1
        hi = pts.max(0) + 0.1
        cen = lo + rng.random((4000, 3)) * (hi - lo)
        rad = rng.uniform(max(r_min, 1e-3), r_max, 4000)
        sph = np.concatenate([cen, rad[:, None]], 1).astype(np.float32)
        sph = np.concatenate([sph, _adversarial_queries(t, pts, max(r_min, 1e-3), r_max, rng)])
        want = orc.brute_f32(pts, sph)
        hit, leaf, rej, scanned = orc.query_tree(t, pts, sph)
        assert (hit == want).all()
        sizes = np.diff(t.off)[leaf]
        assert (scanned <= sizes).all()
        assert (scanned[rej == 1] == 0).all()
        # Sec. IV-D: the AABB step never changes an answer
        no_box = np.tile(np.array([-np.inf] * 3 + [np.inf] * 3, np.float32), (t.N, 1))
        hit2, _, rej2, _ = orc.query(t.N, t.D, t.T, no_box, t.off, pts[t.idx], sph)
        assert (hit2 == want).all() and rej2.sum() == 0


def test_lemma1_dense_grid_tiny_cloud(orc):
    pts = CLOUDS["five"]
    t = orc.build_tree(pts, 0.01, 0.04)
    ax = np.linspace(-0.05, 0.15, 41)
    g = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    for r in (0.01, 0.025, 0.04):
        sph = np.concatenate([g, np.full((len(g), 1), r)], 1).astype(np.float32)
        assert (orc.query_tree(t, pts, sph)[0] == orc.brute_f32(pts, sph)).all()


def test_nonfinite_query_centres(orc):
    pts = CLOUDS["uniform-200"]
    t = orc.build_tree(pts, 0.01, 0.05)
    sph = np.array([[np.nan, 0.5, 0.5, 0.05], [0.5, np.nan, 0.5, 0.05], [np.inf, 0.5, 0.5, 0.05],
                    [-np.inf, -np.inf, -np.inf, 0.05], [0.5, 0.5, np.nan, 0.05]], np.float32)
    assert orc.query_tree(t, pts, sph)[0].tolist() == [0] * 5


# ---------------------------------------------------------------------------
# Split axis per depth (the alternative to the cyclic rule, Sec. IV-A)
# ---------------------------------------------------------------------------
AXES = {
    "random": np.random.default_rng(71).integers(0, 3, 64).astype(np.uint8),
    "x-only": np.zeros(64, np.uint8),
    "z-y": np.tile(np.array([2, 1], np.uint8), 32),
}


def test_cyclic_axes_equal_the_default(orc):
    for name in ("uniform-200", "dups-50", "pow2p1"):
        pts = CLOUDS[name]
        a = orc.build_tree(pts, 0.01, 0.05)
        b = orc.build_tree(pts, 0.01, 0.05, axes=np.arange(64) % 3)
        for f in ("T", "rep", "cell", "aabb", "pruned", "off", "idx"):
            assert np.array_equal(getattr(a, f), getattr(b, f)), (name, f)


@pytest.mark.parametrize("seq", sorted(AXES))
@pytest.mark.parametrize("name", ["uniform-200", "uniform-37", "dups-50", "collinear-33", "coplanar-48", "pow2p1"])
def test_structure_invariants_any_axes(orc, name, seq):
    pts = CLOUDS[name]
    n = len(pts)
    axes = AXES[seq]
    t = orc.build_tree(pts, 0.01, 0.05, axes=axes)
    assert sorted(t.rep.tolist()) == list(range(t.N))
    padded = np.concatenate([pts, np.full((t.N - n, 3), np.inf, np.float32)])
    for i in range(t.N - 1):
        ax = int(axes[int(np.floor(np.log2(i + 1)))])
        left, right = _node_points(t, 2 * i + 1), _node_points(t, 2 * i + 2)
        order = sorted(np.concatenate([left, right]).tolist(), key=lambda j: (padded[j, ax], j))
        assert set(order[:len(left)]) == set(left.tolist())
        assert t.T[i] == padded[order[len(left) - 1], ax]
    for l in range(t.N):
        p = padded[t.rep[l]]
        assert (t.cell[l, :3] <= p).all() and (p <= t.cell[l, 3:]).all()


@pytest.mark.parametrize("seq", sorted(AXES))
@pytest.mark.parametrize("name", ["uniform-37", "lattice-64", "coplanar-48", "pow2p1"])
def test_sets_match_direct_definition_any_axes(orc, name, seq):
    pts = CLOUDS[name]
    t = orc.build_tree(pts, 0.0, 0.05, axes=AXES[seq])
    rmax = Fraction(float(np.float32(0.05)))
    R = rmax * (1 + Fraction(1, 2 ** 20))
    for l in range(t.N):
        s = set(t.set_of(l).tolist())
        for j in range(len(pts)):
            d2 = _exact_cell_dist2(pts[j], t.cell[l])
            if d2 is not None and d2 <= rmax ** 2:
                assert j in s, (l, j)
            if j in s:
                assert d2 is not None and d2 <= R ** 2, (l, j)


@pytest.mark.parametrize("seq", sorted(AXES))
@pytest.mark.parametrize("name", ["uniform-200", "dups-50", "collinear-33", "lattice-64"])
def test_lemma1_any_axes(orc, name, seq):
    pts = CLOUDS[name]
    rng = np.random.default_rng(17)
    t = orc.build_tree(pts, 0.01, 0.05, axes=AXES[seq])
    lo, hi = pts.min(0) - 0.1, pts.max(0) + 0.1
    cen = lo + rng.random((4000, 3)) * (hi - lo)
    # and centres on split planes of the given axes
    planes = []
    for i in rng.integers(0, max(t.N - 1, 1), 1000):
        if t.N == 1 or not np.isfinite(t.T[i]):
            continue
        q = pts[rng.integers(0, len(pts))].astype(np.float64)
        q[int(AXES[seq][int(np.floor(np.log2(i + 1)))])] = t.T[i]
        planes.append(q)
    cen = np.concatenate([cen, np.array(planes).reshape(-1, 3)])
    rad = rng.uniform(0.01, 0.05, len(cen))
    sph = np.concatenate([cen, rad[:, None]], 1).astype(np.float32)
    hit = orc.query_tree(t, pts, sph)[0]
    assert (hit == orc.brute_f32(pts, sph)).all()
    # the wrong axes at query time send spheres to the wrong leaves
    if seq != "random" and name in ("uniform-200", "lattice-64"):
        wrong = orc.query(t.N, t.D, t.T, t.aabb, t.off, pts[t.idx], sph, axes=(AXES[seq] + 1) % 3)[0]
        assert not (wrong == hit).all()
