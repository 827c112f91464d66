"""GPU parity: every entry point of the C ABI against the CPU oracle.

Booleans, tree arrays, set memberships and filter outputs must match bit for
bit; clearance values and gradients within 1e-4 (relative) of the float64
oracle.  Sizes span several tiles and ragged tails; the full-size workloads
are checked answer by answer against the oracle's CollisionCheck on the
oracle's own tree (or, for the 10^8-query room, on the exported GPU tree,
whose splits match the oracle's and whose sampled sets match the direct
definition).
"""
import sys

import numpy as np
import pytest

import synth
from cases import adversarial_clouds, mixed_queries, nonfinite_queries

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def capt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_02807_amd as capt
    capt.load_library()
    return capt


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def canonical_sets(off, idx):
    """Sort every leaf's entries so sets compare as sets."""
    sizes = np.diff(off)
    leaf = np.repeat(np.arange(len(sizes)), sizes)
    order = np.lexsort((idx, leaf))
    return sizes, idx[order]


def compare_build(capt, orc, pts, r_min, r_max, prune=True, axes=None):
    f = capt.capt_build(dev(pts), r_min, r_max, prune=prune, axes=axes)
    b = capt.parse_blob(capt.capt_export(f))
    t = orc.build_tree(pts, r_min, r_max, prune=prune, axes=axes)
    same_tree(b, t)
    return f, b, t


def same_tree(b, t):
    """A parsed blob against an oracle tree, array by array."""
    assert (b.n, b.N, b.D) == (t.n, t.N, t.D)
    assert np.array_equal(bits(b.T), bits(t.T)), "split values differ"
    assert np.array_equal(b.rep, t.rep), "representatives differ"
    assert np.array_equal(b.pruned, t.pruned), "pruned leaves differ"
    sg, ig = canonical_sets(b.off, b.idx)
    so, io = canonical_sets(t.off, t.idx)
    assert np.array_equal(sg, so), "set sizes differ"
    assert np.array_equal(ig, io), "set members differ"
    # AABBs are min / max by value; the sign of a zero bound is not fixed
    assert np.array_equal(b.aabb, t.aabb), "AABBs differ"


# ---------------------------------------------------------------------------
# Query on an imported oracle tree (isolates the query from the build)
# ---------------------------------------------------------------------------
def test_query_imported_oracle_tree_uniform(capt, orc):
    w = synth.workload(1)
    _say("case: uniform-2k imported, 100000 spheres")
    t = orc.build_tree(w.cloud, w.r_min, w.r_max)
    f = capt.capt_import(capt.make_blob(w.cloud, t.T, t.rep, t.aabb, t.pruned, t.off, t.idx, w.r_min, w.r_max))
    got = capt.capt_collides(f, dev(w.spheres), 1).cpu().numpy()
    want = orc.brute_f32(w.cloud, w.spheres)
    assert np.array_equal(got, want)
    assert 0.05 < want.mean() < 0.95


@pytest.mark.parametrize("name", sorted(adversarial_clouds()))
def test_query_imported_adversarial(capt, orc, name):
    pts = adversarial_clouds()[name]
    for (r_min, r_max) in [(0.01, 0.05), (0.0, 0.03), (0.02, 0.02)]:
        _say(f"case: imported {name} r=({r_min},{r_max})")
        t = orc.build_tree(pts, r_min, r_max)
        f = capt.capt_import(capt.make_blob(pts, t.T, t.rep, t.aabb, t.pruned, t.off, t.idx, r_min, r_max))
        sph = mixed_queries(pts, max(r_min, 1e-3), r_max, 3000, 11, tree=t)
        sph = np.concatenate([sph, nonfinite_queries(r_max)])
        want = orc.brute_f32(pts, sph)
        for g in (1, 3):
            m = len(sph) - len(sph) % g
            got = capt.capt_collides(f, dev(sph[:m]), g).cpu().numpy()
            assert np.array_equal(got, want[:m].reshape(-1, g).max(1)), (name, g)


# ---------------------------------------------------------------------------
# Build parity
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", sorted(adversarial_clouds()))
def test_build_matches_oracle_adversarial(capt, orc, name):
    pts = adversarial_clouds()[name]
    for (r_min, r_max, prune) in [(0.01, 0.05, True), (0.0, 0.03, True), (0.05, 0.06, True),
                                  (0.05, 0.06, False)]:
        _say(f"case: build {name} r=({r_min},{r_max}) prune={prune}")
        compare_build(capt, orc, pts, r_min, r_max, prune)


def test_build_matches_oracle_uniform_2k(capt, orc):
    w = synth.workload(1)
    _say("case: build uniform-2k")
    f, b, t = compare_build(capt, orc, w.cloud, w.r_min, w.r_max)
    got = capt.capt_collides(f, dev(w.spheres), 1).cpu().numpy()
    assert np.array_equal(got, orc.brute_f32(w.cloud, w.spheres))


def test_build_matches_oracle_tabletop_filtered(capt, orc):
    cloud = synth.tabletop_cloud(50_000, 2001)
    keep, _ = orc.filter(cloud, 0.01)
    pts = cloud[keep]
    _say(f"case: build tabletop filtered n={len(pts)}")
    compare_build(capt, orc, pts, 0.015, 0.08)
    compare_build(capt, orc, pts, 0.0, 0.08)


def test_build_empty_cloud(capt, orc):
    _say("case: build empty")
    f = capt.capt_build(torch.zeros((0, 3), dtype=torch.float32, device="cuda"), 0.01, 0.05)
    b = capt.parse_blob(capt.capt_export(f))
    assert (b.n, b.N, len(b.idx)) == (0, 1, 0)
    sph = dev(np.array([[0, 0, 0, 0.05]] * 64, np.float32))
    assert capt.capt_collides(f, sph, 1).cpu().numpy().sum() == 0


def test_build_rejects_nonfinite(capt):
    pts = np.random.default_rng(0).random((100, 3)).astype(np.float32)
    pts[17, 1] = np.nan
    with pytest.raises(capt.CaptError) as e:
        capt.capt_build(dev(pts), 0.01, 0.05)
    assert e.value.status == capt.CAPT_EINVAL


# ---------------------------------------------------------------------------
# End-to-end query with configuration groups
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("g", [1, 7, 60, 64, 100])
def test_collides_groups_tabletop(capt, orc, g):
    pts = synth.tabletop_cloud(12_000, 91)
    _say(f"case: collides tabletop-12k g={g}")
    f = capt.capt_build(dev(pts), 0.015, 0.08)
    if g == 60:
        sph = synth.posed_spheres(synth.chain_template(2003), 3001, synth.WORKSPACE, 92)
    else:
        sph = synth.uniform_spheres(g * 1501, synth.WORKSPACE, 0.015, 0.08, 93)
    got = capt.capt_collides(f, dev(sph), g).cpu().numpy()
    want = orc.brute_f32(pts, sph, g)
    assert np.array_equal(got, want)
    assert 0 < want.sum() <= len(want)


@pytest.mark.parametrize("name,n,rf", [("tabletop", 50_000, 0.01), ("uniform", 3000, 0.02), ("empty", 0, 0.01)])
def test_build_filtered_equals_filter_then_build(capt, name, n, rf):
    _say(f"case: build_filtered {name} n={n} rf={rf}")
    if name == "tabletop":
        pts = synth.tabletop_cloud(n, 2001)
    else:
        pts = synth.uniform_cube_cloud(n, 77) if n else np.zeros((0, 3), np.float32)
    x = dev(pts)
    fx, fi = capt.capt_filter(x, rf)
    f_ref = capt.capt_build(fx.contiguous(), 0.015, 0.08)
    f, ki = capt.capt_build_filtered(x, rf, 0.015, 0.08, kept_index=True)
    assert np.array_equal(ki.cpu().numpy(), fi.cpu().numpy())
    a, b = capt.parse_blob(capt.capt_export(f)), capt.parse_blob(capt.capt_export(f_ref))
    assert (a.n, a.N, a.D) == (b.n, b.N, b.D)
    assert np.array_equal(bits(a.T), bits(b.T))
    assert np.array_equal(a.rep, b.rep) and np.array_equal(a.pruned, b.pruned)
    assert all(np.array_equal(u, v) for u, v in zip(canonical_sets(a.off, a.idx), canonical_sets(b.off, b.idx)))
    assert np.array_equal(a.aabb, b.aabb)


@pytest.mark.parametrize("name,base,reach", [("tabletop-half", (0.0, 0.0, 0.4), 0.9),
                                               ("tabletop-all", (0.0, 0.0, 0.4), float("inf")),
                                               ("tabletop-none", (9.0, 9.0, 9.0), 0.5),
                                               ("room-arm", (3.0, 3.0, 0.8), 1.5)])
def test_filter_crop_matches_oracle(capt, orc, name, base, reach):
    _say(f"case: filter crop {name}")
    pts = synth.room_cloud(180_000, 20_000, 1005) if name.startswith("room") else synth.tabletop_cloud(50_000, 2001)
    rf = 0.01
    fx, fi = capt.capt_filter(dev(pts), rf, base=base, reach=reach)
    want, _ = orc.filter(pts, rf, base=base, reach=reach)
    assert np.array_equal(fi.cpu().numpy(), want)
    assert np.array_equal(bits(fx.cpu().numpy()), bits(pts[want]))
    if name == "tabletop-all":
        assert np.array_equal(want, orc.filter(pts, rf)[0])
    if name == "tabletop-none":
        assert len(want) == 0


def test_filter_crop_rejects_nonfinite(capt):
    pts = synth.tabletop_cloud(5000, 3)
    pts[1234, 1] = np.nan   # outside any reach ball, still an error
    with pytest.raises(capt.CaptError) as e:
        capt.capt_filter(dev(pts), 0.01, base=(0.0, 0.0, 0.4), reach=0.5)
    assert e.value.status == capt.CAPT_EINVAL


def test_build_filtered_with_crop(capt):
    _say("case: build_filtered with crop")
    pts = synth.tabletop_cloud(50_000, 2001)
    x = dev(pts)
    base, reach = (0.2, 0.1, 0.3), 0.9
    fx, fi = capt.capt_filter(x, 0.01, base=base, reach=reach)
    f_ref = capt.capt_build(fx.contiguous(), 0.015, 0.08)
    f, ki = capt.capt_build_filtered(x, 0.01, 0.015, 0.08, kept_index=True, base=base, reach=reach)
    assert np.array_equal(ki.cpu().numpy(), fi.cpu().numpy())
    a, b = capt.parse_blob(capt.capt_export(f)), capt.parse_blob(capt.capt_export(f_ref))
    assert (a.n, a.D) == (b.n, b.D) and np.array_equal(bits(a.T), bits(b.T)) and np.array_equal(a.rep, b.rep)


@pytest.mark.parametrize("g", [1, 7, 60])
def test_collides_padded_matches_oracle(capt, orc, g):
    _say(f"case: padded queries g={g}")
    pts = synth.tabletop_cloud(12_000, 91)
    f = capt.capt_build(dev(pts), 0.015, 0.08)
    pad = 0.02
    if g == 60:
        sph = synth.posed_spheres(synth.chain_template(2003), 2001, synth.WORKSPACE, 92)
        sph[:, 3] = np.minimum(sph[:, 3], np.float32(0.06))
    else:
        sph = synth.uniform_spheres(g * 1501, synth.WORKSPACE, 0.015, 0.06, 93)
    got = capt.capt_collides_padded(f, dev(sph), g, pad, flags=capt.CAPT_CHECK_RADII).cpu().numpy()
    want = orc.brute_f32(pts, sph, g, pad=pad)
    assert np.array_equal(got, want)
    assert want.sum() > orc.brute_f32(pts, sph, g).sum()   # the padding changes answers
    # pad 0 is the unpadded query
    assert np.array_equal(capt.capt_collides_padded(f, dev(sph), g, 0.0).cpu().numpy(),
                          capt.capt_collides(f, dev(sph), g).cpu().numpy())


def test_collides_padded_radius_check_and_forest(capt, orc):
    pts = [synth.tabletop_cloud(3000, 200 + c) for c in range(3)]
    f = capt.capt_build(dev(np.concatenate(pts)), 0.015, 0.08, cloud_off=[0, 3000, 6000, 9000])
    sph = [synth.uniform_spheres(60 * 300, synth.WORKSPACE, 0.015, 0.05, 300 + c) for c in range(3)]
    qoff = [0, 18000, 36000, 54000]
    got = capt.capt_collides_padded(f, dev(np.concatenate(sph)), 60, 0.03, query_off=qoff).cpu().numpy()
    want = np.concatenate([orc.brute_f32(p, q, 60, pad=0.03) for p, q in zip(pts, sph)])
    assert np.array_equal(got, want)
    with pytest.raises(capt.CaptError) as e:   # 0.05 + 0.04 > r_max
        capt.capt_collides_padded(f, dev(np.concatenate(sph)), 60, 0.04, query_off=qoff,
                                  flags=capt.CAPT_CHECK_RADII)
    assert e.value.status == capt.CAPT_ERADIUS
    with pytest.raises(capt.CaptError) as e:
        capt.capt_collides_padded(f, dev(np.concatenate(sph)), 60, float("nan"), query_off=qoff)
    assert e.value.status == capt.CAPT_EINVAL


def test_indexed_sets_give_the_same_answers(capt, orc):
    _say("case: indexed sets against plain sets")
    cloud = synth.tabletop_cloud(50_000, 2001)
    keep, _ = orc.filter(cloud, 0.01)
    pts = cloud[keep]
    x = dev(pts)
    f = capt.capt_build(x, 0.015, 0.08)
    fi = capt.capt_build(x, 0.015, 0.08, indexed=True)
    assert fi.info()["bytes"] < 0.6 * f.info()["bytes"]
    a, b = capt.parse_blob(capt.capt_export(f)), capt.parse_blob(capt.capt_export(fi))
    assert b.flags == a.flags | capt.CAPT_INDEXED_SETS
    assert np.array_equal(bits(a.T), bits(b.T)) and np.array_equal(a.off, b.off) and np.array_equal(a.idx, b.idx)
    assert np.array_equal(a.aabb, b.aabb)
    sph60 = synth.posed_spheres(synth.chain_template(2003), 3001, synth.WORKSPACE, 92)
    for g, sp in ((1, synth.uniform_spheres(30_000, synth.WORKSPACE, 0.015, 0.08, 93)), (7, sph60[:7 * 3000]),
                  (60, sph60)):
        want = capt.capt_collides(f, dev(sp), g).cpu().numpy()
        assert np.array_equal(capt.capt_collides(fi, dev(sp), g).cpu().numpy(), want), g
        if g == 60:
            assert np.array_equal(want, orc.brute_f32(pts, sp, 60))
    assert np.array_equal(capt.capt_collides_padded(fi, dev(sph60), 60, 0.0).cpu().numpy(),
                          capt.capt_collides(f, dev(sph60), 60).cpu().numpy())
    for u, v in zip(capt.capt_query_stats(f, dev(sph60)), capt.capt_query_stats(fi, dev(sph60))):
        assert torch.equal(u, v)
    for u, v in zip(capt.capt_query_chunk_stats(f, dev(sph60)), capt.capt_query_chunk_stats(fi, dev(sph60))):
        assert torch.equal(u, v)
    # posed edges and an imported indexed forest
    tm = synth.chain_template(2003).astype(np.float32)
    poses = synth.pose_edges(500, 4, synth.WORKSPACE, 95)
    assert torch.equal(capt.capt_collides_posed(fi, dev(tm), dev(poses), 4),
                       capt.capt_collides_posed(f, dev(tm), dev(poses), 4))
    fj = capt.capt_import(capt.capt_export(fi))
    assert torch.equal(capt.capt_collides(fj, dev(sph60), 60), capt.capt_collides(f, dev(sph60), 60))
    # clearance on unpruned forests
    fu = capt.capt_build(x, 0.0, 0.08)
    fui = capt.capt_build(x, 0.0, 0.08, indexed=True)
    sc = dev(synth.uniform_spheres(20_000, synth.WORKSPACE, 0.015, 0.08, 96))
    ca, wa = capt.capt_clearance(fu, sc)
    cb, wb = capt.capt_clearance(fui, sc)
    assert torch.equal(ca, cb) and torch.equal(wa, wb)


def test_edge_cases_of_the_frame_calls(capt, orc):
    _say("case: frame-call edge cases")
    pts = synth.tabletop_cloud(5000, 41)
    x = dev(pts)
    # a crop that removes every point: an empty forest that answers no
    f, ki = capt.capt_build_filtered(x, 0.01, 0.015, 0.08, kept_index=True, base=(50.0, 50.0, 50.0), reach=1.0)
    assert ki.numel() == 0 and f.info()["n"] == 0
    sph = synth.uniform_spheres(600, synth.WORKSPACE, 0.015, 0.08, 42)
    assert int(capt.capt_collides(f, dev(sph), 60).sum()) == 0
    # reach 0 keeps exactly the points at the base (the duplicate goes to the filter)
    one = np.array([[0.25, 0.5, 0.75], [0.25, 0.5, 0.75000006], [0.25, 0.5, 0.75]], np.float32)
    fx, fi = capt.capt_filter(dev(one), 0.0, base=(0.25, 0.5, 0.75), reach=0.0)
    want, _ = orc.filter(one, 0.0, base=(0.25, 0.5, 0.75), reach=0.0)
    assert fi.cpu().numpy().tolist() == want.tolist() == [0]
    # padded queries: no spheres, and group 1
    fp = capt.capt_build(x, 0.015, 0.08)
    assert capt.capt_collides_padded(fp, dev(np.zeros((0, 4), np.float32)), 1, 0.01).numel() == 0
    sp1 = synth.uniform_spheres(5000, synth.WORKSPACE, 0.015, 0.06, 43)
    assert np.array_equal(capt.capt_collides_padded(fp, dev(sp1), 1, 0.02).cpu().numpy(),
                          orc.brute_f32(pts, sp1, 1, pad=0.02))
    # indexed batched forest against plain, and stream-ordered release of a forest with a batched plan
    clouds = [synth.tabletop_cloud(2000 + 1000 * c, 300 + c) for c in range(3)]
    off = np.cumsum([0] + [len(c) for c in clouds]).tolist()
    qs = [synth.uniform_spheres(60 * 400, synth.WORKSPACE, 0.015, 0.08, 310 + c) for c in range(3)]
    qoff = np.cumsum([0] + [len(q) for q in qs]).tolist()
    fa = capt.capt_build(dev(np.concatenate(clouds)), 0.015, 0.08, cloud_off=off)
    fb = capt.capt_build(dev(np.concatenate(clouds)), 0.015, 0.08, cloud_off=off, indexed=True)
    a = capt.capt_collides(fa, dev(np.concatenate(qs)), 60, query_off=qoff)
    b = capt.capt_collides(fb, dev(np.concatenate(qs)), 60, query_off=qoff)
    assert torch.equal(a, b)
    assert np.array_equal(a.cpu().numpy(), np.concatenate([orc.brute_f32(c, q, 60) for c, q in zip(clouds, qs)]))
    fa.release()
    fb.release()
    torch.cuda.synchronize()


AXES = {"random": np.random.default_rng(71).integers(0, 3, 32).astype(np.uint8),
        "x-only": np.zeros(32, np.uint8), "z-y": np.tile(np.array([2, 1], np.uint8), 16)}


@pytest.mark.parametrize("seq", sorted(AXES))
@pytest.mark.parametrize("name", ["uniform-3000", "tabletop-filtered", "dups-300"])
def test_build_and_query_any_axes(capt, orc, seq, name):
    _say(f"case: split axes {seq} on {name}")
    if name == "uniform-3000":
        pts = synth.uniform_cube_cloud(3000, 51)
    elif name == "dups-300":
        pts = np.repeat(synth.uniform_cube_cloud(60, 52), 5, axis=0)
    else:
        c = synth.tabletop_cloud(50_000, 2001)
        pts = c[orc.filter(c, 0.01)[0]]
    axes = AXES[seq]
    r_min, r_max = (0.015, 0.08) if name == "tabletop-filtered" else (0.01, 0.05)
    f, b, t = compare_build(capt, orc, pts, r_min, r_max, axes=axes)
    assert np.array_equal(b.axes, axes[:b.D]) or b.D == 0 or np.array_equal(axes[:b.D], np.arange(b.D) % 3)
    lo, hi = pts.min(0) - 0.1, pts.max(0) + 0.1
    rng = np.random.default_rng(53)
    cen = lo + rng.random((60 * 500, 3)) * (hi - lo)
    sph = np.concatenate([cen, rng.uniform(r_min, r_max, (len(cen), 1))], 1).astype(np.float32)
    for g in (1, 60):
        assert np.array_equal(capt.capt_collides(f, dev(sph), g).cpu().numpy(), orc.brute_f32(pts, sph, g)), g
    leaf, rej, scanned, hit = (x.cpu().numpy() for x in capt.capt_query_stats(f, dev(sph)))
    hit_o, leaf_o, rej_o, sc_o = orc.query_tree(t, pts, sph)
    assert np.array_equal(leaf, leaf_o) and np.array_equal(rej, rej_o) and np.array_equal(hit, hit_o)
    # export / import keeps the axes
    g2 = capt.capt_import(capt.capt_export(f))
    assert torch.equal(capt.capt_collides(g2, dev(sph), 60), capt.capt_collides(f, dev(sph), 60))


def test_clearance_and_batches_any_axes(capt, orc):
    _say("case: split axes: clearance and forests of several clouds")
    axes = AXES["random"]
    c = synth.tabletop_cloud(50_000, 2001)
    pts = c[orc.filter(c, 0.01)[0]]
    f = capt.capt_build(dev(pts), 0.0, 0.08, axes=axes)
    sph = synth.uniform_spheres(4000, synth.WORKSPACE, 0.015, 0.08, 54)
    clr, wit = capt.capt_clearance(f, dev(sph))
    clr_o, wit_o, _ = orc.clearance_f64(pts, sph, 0.08)
    c64 = clr.cpu().numpy().astype(np.float64)
    assert (np.abs(c64 - clr_o) <= 1e-4 * np.maximum(np.abs(clr_o), 0.08)).all()
    clouds = [synth.tabletop_cloud(2000 + 1000 * k, 400 + k) for k in range(3)]
    off = np.cumsum([0] + [len(x) for x in clouds]).tolist()
    qs = [synth.uniform_spheres(60 * 300, synth.WORKSPACE, 0.015, 0.08, 410 + k) for k in range(3)]
    qoff = np.cumsum([0] + [len(q) for q in qs]).tolist()
    fb = capt.capt_build(dev(np.concatenate(clouds)), 0.015, 0.08, cloud_off=off, axes=axes)
    got = capt.capt_collides(fb, dev(np.concatenate(qs)), 60, query_off=qoff).cpu().numpy()
    assert np.array_equal(got, np.concatenate([orc.brute_f32(x, q, 60) for x, q in zip(clouds, qs)]))


def test_stream_ordered_release(capt, orc):
    # per-frame pattern: build, query and release in stream order without a
    # host wait; later builds reuse the released memory behind earlier queries
    _say("case: stream-ordered release, 4 frames of tabletop-6k")
    sph = synth.posed_spheres(synth.chain_template(2003), 800, synth.WORKSPACE, 95)
    sd = dev(sph)
    outs, clouds = [], []
    for k in range(4):
        pts = synth.tabletop_cloud(6000, 120 + k)
        f = capt.capt_build(dev(pts), 0.015, 0.08)
        outs.append(capt.capt_collides(f, sd, 60))
        f.release()
        clouds.append(pts)
    torch.cuda.synchronize()
    for pts, o in zip(clouds, outs):
        assert np.array_equal(o.cpu().numpy(), orc.brute_f32(pts, sph, 60))


def test_check_radii_flag(capt):
    pts = synth.tabletop_cloud(2000, 5)
    f = capt.capt_build(dev(pts), 0.015, 0.08)
    sph = synth.uniform_spheres(640, synth.WORKSPACE, 0.015, 0.08, 6)
    capt.capt_collides(f, dev(sph), 1, flags=capt.CAPT_CHECK_RADII)
    sph[100, 3] = 0.2
    with pytest.raises(capt.CaptError) as e:
        capt.capt_collides(f, dev(sph), 1, flags=capt.CAPT_CHECK_RADII)
    assert e.value.status == capt.CAPT_ERADIUS


def test_query_stats_match_oracle_replay(capt, orc):
    pts = synth.tabletop_cloud(8000, 41)
    _say("case: query stats")
    f = capt.capt_build(dev(pts), 0.015, 0.08)
    b = capt.parse_blob(capt.capt_export(f))
    sph = synth.uniform_spheres(20_000, synth.WORKSPACE, 0.015, 0.08, 42)
    leaf, rej, sc, hit = [x.cpu().numpy() for x in capt.capt_query_stats(f, dev(sph))]
    hit_o, leaf_o, rej_o, sc_o = orc.query(b.N, b.D, b.T, b.aabb, b.off, b.points[b.idx], sph)
    assert np.array_equal(leaf, leaf_o) and np.array_equal(rej, rej_o) and np.array_equal(sc, sc_o)
    assert np.array_equal(hit, hit_o) and np.array_equal(hit, orc.brute_f32(pts, sph))


def _f32_sqdist(q, p):
    """((dx*dx + dy*dy) + dz*dz) in float32, every operation rounded."""
    d = (q[None, :3] - p).astype(np.float32)
    s = d * d
    return (s[:, 0] + s[:, 1]) + s[:, 2]


def _f32_box_sqdist(q, lo, hi):
    g = np.maximum(np.maximum(lo - q[:3], q[:3] - hi), np.float32(0)).astype(np.float32)
    s = g * g
    return (s[0] + s[1]) + s[2]


def _hbox_offset(base, v, up):
    """The chunk-box offset rule of capt.h: the nearest half of v - base
    (float32), moved one half at a time until base + offset <= v (>= v)."""
    base, v = np.float32(base), np.float32(v)
    h = int(np.float16(np.float32(v - base)).view(np.uint16))
    val = lambda h: np.float32(base + np.float32(np.uint16(h).view(np.float16)))
    for _ in range(8):
        if up and val(h) < v:
            h = min(h + 1, 0x7C00)
        elif not up and val(h) > v:
            h = max(h - 1, 0)
    if up and val(h) < v:
        h = 0x7C00
    if not up and val(h) > v:
        h = 0
    return val(h)


def _decoded_box(base, lo, hi):
    return (np.array([_hbox_offset(base[a], lo[a], False) for a in range(3)], np.float32),
            np.array([_hbox_offset(base[a], hi[a], True) for a in range(3)], np.float32))


def test_chunk_stats_match_stored_order_replay(capt):
    """The two-level scan's accounting, replayed on the host from the exported
    sets in stored order: 16-entry chunks, each chunk's box rounded outward to
    half-precision offsets from its set's box, early exit at the chunk holding
    the first hit."""
    pts = synth.tabletop_cloud(8000, 41)
    _say("case: chunk stats")
    f = capt.capt_build(dev(pts), 0.015, 0.08)
    b = capt.parse_blob(capt.capt_export(f))
    sph = synth.uniform_spheres(4000, synth.WORKSPACE, 0.015, 0.08, 43)
    leaf, rej, _, _ = [x.cpu().numpy() for x in capt.capt_query_stats(f, dev(sph))]
    nb, nc = [x.cpu().numpy() for x in capt.capt_query_chunk_stats(f, dev(sph))]
    P = b.points
    for i, q in enumerate(sph):
        r2 = np.float32(q[3]) * np.float32(q[3])
        want_b = want_c = 0
        if not rej[i]:
            ids = b.idx[b.off[leaf[i]]:b.off[leaf[i] + 1]]
            for c0 in range(0, len(ids), 16):
                cp = P[ids[c0:c0 + 16]]
                want_b += 1
                blo, bhi = _decoded_box(b.aabb[leaf[i], :3], cp.min(0), cp.max(0))
                assert (blo <= cp.min(0)).all() and (bhi >= cp.max(0)).all()
                if _f32_box_sqdist(q, blo, bhi) > r2:
                    assert not (_f32_sqdist(q, cp) <= r2).any(), "a skipped chunk holds a hit"
                    continue
                want_c += 1
                if (_f32_sqdist(q, cp) <= r2).any():
                    break
        assert (nb[i], nc[i]) == (want_b, want_c), i
    assert nc.sum() < nb.sum()


# ---------------------------------------------------------------------------
# GPU brute force (the benchmark's baseline) is exact too
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("g", [1, 60, 100])
def test_bruteforce_matches_oracle(capt, orc, g):
    pts = synth.tabletop_cloud(5000, 51)
    _say(f"case: brute g={g}")
    sph = synth.uniform_spheres(g * 700, synth.WORKSPACE, 0.015, 0.08, 52)
    got = capt.capt_bruteforce_collides(dev(pts), dev(sph), g).cpu().numpy()
    assert np.array_equal(got, orc.brute_f32(pts, sph, g))


# ---------------------------------------------------------------------------
# Filter parity
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,rf", [("tabletop-50k", 0.01), ("tabletop-50k", 0.03), ("uniform-1000", 0.05),
                                     ("dups-300", 0.0), ("identical-64", 0.01), ("single", 0.01),
                                     ("collinear-129", 0.004), ("negzero", 0.001), ("room-60k", 0.005)])
def test_filter_matches_oracle(capt, orc, name, rf):
    if name == "tabletop-50k":
        pts = synth.tabletop_cloud(50_000, 2001)
    elif name == "room-60k":
        pts = synth.room_cloud(54_000, 6_000, 5001)
    else:
        pts = adversarial_clouds()[name]
    _say(f"case: filter {name} rf={rf}")
    kept, _ = orc.filter(pts, rf)
    out, idx = capt.capt_filter(dev(pts), rf)
    assert np.array_equal(idx.cpu().numpy(), kept)
    assert np.array_equal(bits(out.cpu().numpy()), bits(pts[kept]))


@pytest.mark.parametrize("n", [174_762, 174_763])
def test_filter_sort_tile_boundary(capt, orc, n):
    """The filter's six-key sort switches from 2,048- to 4,096-key tiles at
    2^20 keys (6 n = 1,048,572 and 1,048,578): both sides against the oracle."""
    pts = synth.room_cloud(n - n // 10, n // 10, 5003)
    _say(f"case: filter of {n} room points at the sort's tile boundary")
    kept, _ = orc.filter(pts, 0.005)
    out, idx = capt.capt_filter(dev(pts), 0.005)
    assert np.array_equal(idx.cpu().numpy(), kept)
    assert np.array_equal(bits(out.cpu().numpy()), bits(pts[kept]))


# ---------------------------------------------------------------------------
# Batched ragged forests
# ---------------------------------------------------------------------------
def _coincident_clouds():
    rng = np.random.default_rng(808)
    base = synth.tabletop_cloud(50_000, 809)
    one = base.copy()
    one[rng.choice(len(one), 40_000, replace=False)] = base[123]          # 80% on one point
    many = base.copy()
    for k in range(8):                                                    # 8 clusters of 5,000 copies
        many[rng.choice(len(many), 5_000, replace=False)] = base[1000 * k + 7]
    ball = base.copy()                                                    # 80% within 1 mm of a point
    pick = rng.choice(len(ball), 40_000, replace=False)
    ball[pick] = (base[555].astype(np.float64) + rng.uniform(-5e-4, 5e-4, (40_000, 3))).astype(np.float32)
    big = synth.tabletop_cloud(120_000, 810)                               # large enough for 512-position chunks
    for k in range(8):                                                    # 8 clusters of 12,000 copies
        big[rng.choice(len(big), 12_000, replace=False)] = big[9000 * k + 11]
    return {"one-point-80pct": one, "eight-clusters": many, "ball-1mm-80pct": ball, "clusters-120k": big}


@pytest.mark.parametrize("name", ["one-point-80pct", "eight-clusters", "ball-1mm-80pct", "clusters-120k"])
@pytest.mark.parametrize("rf", [0.01, 0.0])
def test_filter_coincident_runs(capt, orc, name, rf):
    """Long runs of coincident or near-coincident points along the curve (far
    longer than a next pointer's bounded search): the filter output against
    the oracle exactly, every pass still linear in n."""
    pts = _coincident_clouds()[name]
    _say(f"case: filter of {name}, r_filter={rf}")
    fx, fidx = capt.capt_filter(dev(pts), rf)
    keep, _ = orc.filter(pts, rf)
    assert np.array_equal(fidx.cpu().numpy(), keep)
    assert np.array_equal(bits(fx.cpu().numpy()), bits(pts[keep]))


def test_batched_matches_per_cloud_and_oracle(capt, orc):
    w = synth.workload(3, scale=0.02)
    _say(f"case: batched {len(w.cloud)} clouds, {sum(len(s) for s in w.spheres)} spheres")
    cloud_off = np.concatenate([[0], np.cumsum([len(c) for c in w.cloud])])
    query_off = np.concatenate([[0], np.cumsum([len(s) for s in w.spheres])])
    xyz = dev(np.concatenate(w.cloud))
    sph = dev(np.concatenate(w.spheres))
    f = capt.capt_build(xyz, w.r_min, w.r_max, cloud_off=cloud_off)
    a = capt.capt_collides(f, sph, 60, query_off=query_off).cpu().numpy()
    b = capt.capt_collides(f, sph, 60, query_off=query_off, flags=capt.CAPT_PER_CLOUD).cpu().numpy()
    c = capt.capt_collides(f, sph, 60, query_off=query_off, flags=capt.CAPT_NO_GRAPH).cpu().numpy()
    # graph replay gives the same answer again
    d = capt.capt_collides(f, sph, 60, query_off=query_off).cpu().numpy()
    br = capt.capt_bruteforce_collides(xyz, sph, 60, cloud_off=cloud_off, query_off=query_off).cpu().numpy()
    want = np.concatenate([orc.brute_f32(w.cloud[i], w.spheres[i], 60) for i in range(len(w.cloud))])
    for x in (a, b, c, d, br):
        assert np.array_equal(x, want)


@pytest.mark.parametrize("group", [60, 7])
def test_batched_tiny_and_empty_clouds(capt, orc, group):
    # depths 0 .. 12 in one forest: an empty cloud, one point, two, five, and
    # clouds deeper than the batched kernel's per-wave tree copy
    sizes = [0, 1, 2, 5, 300, 3000]
    _say(f"case: batched tiny and empty clouds, group {group}")
    clouds = [synth.tabletop_cloud(n, 440 + k) if n else np.zeros((0, 3), np.float32)
              for k, n in enumerate(sizes)]
    qs = [synth.uniform_spheres(group * (50 + 30 * k), synth.WORKSPACE, 0.015, 0.08, 450 + k)
          for k in range(len(sizes))]
    off = np.cumsum([0] + [len(c) for c in clouds]).tolist()
    qoff = np.cumsum([0] + [len(q) for q in qs]).tolist()
    f = capt.capt_build(dev(np.concatenate(clouds)), 0.015, 0.08, cloud_off=off)
    assert [f.info(c)["D"] for c in range(len(sizes))] == [0, 0, 1, 3, 9, 12]
    want = np.concatenate([orc.brute_f32(c, q, group) if len(c) else np.zeros(len(q) // group, np.uint8)
                           for c, q in zip(clouds, qs)])
    sq = dev(np.concatenate(qs))
    for flags in (0, capt.CAPT_NO_GRAPH, capt.CAPT_PER_CLOUD):
        got = capt.capt_collides(f, sq, group, query_off=qoff, flags=flags).cpu().numpy()
        assert np.array_equal(got, want), flags
    assert want.any() and not want.all()


@pytest.mark.parametrize("group", [60, 7, 1])
def test_batched_queue_decides_every_configuration_once(capt, orc, group):
    """The batched kernel's tile queue: with per-configuration decision counts,
    every configuration of every cloud is decided exactly once (no tile
    skipped, none taken twice, tiles do not overlap), for several tile sizes
    and launch shapes, on a forest with empty, tiny and deep clouds."""
    sizes = [0, 1, 5, 3000, 20000, 300, 0, 9000]
    clouds = [synth.tabletop_cloud(n, 470 + k) if n else np.zeros((0, 3), np.float32)
              for k, n in enumerate(sizes)]
    ncfg = [0, 13, 40, 700, 2500, 1, 33, 1200]
    qs = [synth.uniform_spheres(group * m, synth.WORKSPACE, 0.015, 0.08, 480 + k) for k, m in enumerate(ncfg)]
    off = np.cumsum([0] + [len(c) for c in clouds]).tolist()
    qoff = np.cumsum([0] + [len(q) for q in qs]).tolist()
    f = capt.capt_build(dev(np.concatenate(clouds)), 0.015, 0.08, cloud_off=off)
    want = np.concatenate([orc.brute_f32(c, q, group) if len(c) else np.zeros(len(q) // group, np.uint8)
                           for c, q in zip(clouds, qs)])
    sq = dev(np.concatenate(qs))
    before = capt.capt_get_tuning()
    try:
        for shape in [dict(tile_cfgs=1, waves_per_group=4, groups_per_cu=1), dict(tile_cfgs=16),
                      dict(tile_cfgs=64, waves_per_group=16, groups_per_cu=4), dict(tile_cfgs=1000)]:
            capt.capt_set_tuning(**{**before, **shape})
            _say(f"case: batched queue, group {group}, {shape}")
            out, visits = capt.capt_collides_visits(f, sq, group, query_off=qoff)
            v = visits.cpu().numpy()
            assert v.shape == (sum(ncfg),)
            assert (v == 1).all(), (shape, np.flatnonzero(v != 1)[:10], v[v != 1][:10])
            assert np.array_equal(out.cpu().numpy(), want), shape
    finally:
        capt.capt_set_tuning(**before)
    assert want.any() and not want.all()


def test_batched_queue_visits_rejects_per_depth_axes(capt):
    """The batched kernel takes cyclic split axes only; the diagnostic entry
    point says so instead of answering."""
    pts = synth.tabletop_cloud(2000, 481)
    f = capt.capt_build(dev(pts), 0.015, 0.08, axes=[0] * 12)
    sph = dev(synth.uniform_spheres(600, synth.WORKSPACE, 0.015, 0.08, 482))
    with pytest.raises(capt.CaptError) as e:
        capt.capt_collides_visits(f, sph, 60)
    assert e.value.status == capt.CAPT_EUNSUPPORTED


# ---------------------------------------------------------------------------
# Clearance and its gradient
# ---------------------------------------------------------------------------
def test_clearance_and_gradient(capt, orc):
    cloud = synth.tabletop_cloud(50_000, 2001)
    keep, _ = orc.filter(cloud, 0.01)
    pts = cloud[keep]
    r_max = 0.08
    sph = synth.uniform_spheres(6000, synth.WORKSPACE, 0.015, 0.08, 4002)
    _say("case: clearance")
    f = capt.capt_build(dev(pts), 0.0, r_max)
    s = dev(sph).requires_grad_(True)
    clr, wit = capt.clearance(f, s)
    loss = torch.nn.functional.softplus(-clr / 0.01).sum()
    loss.backward()
    clr_o, wit_o, grad_o = orc.clearance_f64(pts, sph, r_max)
    c = clr.detach().cpu().numpy().astype(np.float64)
    assert (np.abs(c - clr_o) <= 1e-4 * np.maximum(np.abs(clr_o), r_max)).all()
    w = wit.cpu().numpy()
    P = pts.astype(np.float64)
    x = sph[:, :3].astype(np.float64)
    same = w == wit_o
    # a different witness must be an equally near point (within 1e-6 m)
    for i in np.where(~same)[0]:
        if w[i] < 0 or wit_o[i] < 0:
            d = np.sqrt(((x[i] - P[max(w[i], wit_o[i])]) ** 2).sum())
            assert abs(d - r_max) < 1e-6
        else:
            assert abs(np.linalg.norm(x[i] - P[w[i]]) - np.linalg.norm(x[i] - P[wit_o[i]])) < 1e-6
    assert same.mean() > 0.99
    # analytic gradient of the loss in float64 from the oracle
    z = -clr_o / 0.01
    dl = -1.0 / (1.0 + np.exp(-z)) / 0.01
    g_ref = np.concatenate([grad_o * dl[:, None], -dl[:, None]], 1)
    g = s.grad.cpu().numpy().astype(np.float64)
    ok = same
    err = np.linalg.norm(g[ok] - g_ref[ok], axis=1)
    assert (err <= 1e-4 * np.linalg.norm(g_ref[ok], axis=1) + 1e-6).all()


def test_clearance_rejects_pruned_forest(capt):
    pts = adversarial_clouds()["lattice-216"]
    f = capt.capt_build(dev(pts), 0.05, 0.06)
    if f.info()["pruned"] == 0:
        pytest.skip("no leaf pruned")
    with pytest.raises(capt.CaptError) as e:
        capt.capt_clearance(f, dev(np.zeros((4, 4), np.float32) + 0.05))
    assert e.value.status == capt.CAPT_EPRUNED


# ---------------------------------------------------------------------------
# Shards: a forest built for one depth-k subtree's leaves
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prune", [True, False])
def test_shard_build_matches_oracle(capt, orc, prune):
    pts = synth.tabletop_cloud(6000, 2101)
    t = orc.build_tree(pts, 0.015, 0.08, prune=prune)
    x = dev(pts)
    for bits, s in ((0, 0), (1, 0), (1, 1), (3, 5), (t.D, 77), (t.D + 2, 8), (t.D + 2, 9)):
        _say(f"case: shard {s} of 2^{bits}, prune {prune}")
        f = capt.capt_build(x, 0.015, 0.08, prune=prune, shard=(bits, s))
        b = capt.parse_blob(capt.capt_export(f))
        same_tree(b, orc.shard_tree(t, bits, s))
        assert f.info()["set_total"] == int(orc.shard_tree(t, bits, s).off[-1])


def test_shard_answers_combine_to_the_whole_forest(capt, orc):
    _say("case: 4 shards of the filtered tabletop-50k, groups 1 and 60")
    cloud = synth.tabletop_cloud(50_000, 2001)
    pts = cloud[orc.filter(cloud, 0.01)[0]]
    x = dev(pts)
    t = orc.build_tree(pts, 0.015, 0.08)
    whole = capt.capt_build(x, 0.015, 0.08)
    sph = synth.posed_spheres(synth.chain_template(2003), 2000, synth.WORKSPACE, 2102)
    sd = dev(sph)
    bits = 2
    acc1 = torch.zeros(len(sph), dtype=torch.uint8, device="cuda")
    acc60 = torch.zeros(len(sph) // 60, dtype=torch.uint8, device="cuda")
    size = 0
    for s in range(2 ** bits):
        f = capt.capt_build(x, 0.015, 0.08, shard=(bits, s))
        size += f.info()["set_total"]
        hit_o = orc.query_tree(orc.shard_tree(t, bits, s), pts, sph)[0]
        g1 = capt.capt_collides(f, sd, 1)
        g60 = capt.capt_collides(f, sd, 60)
        assert np.array_equal(g1.cpu().numpy(), hit_o)
        assert np.array_equal(g60.cpu().numpy(), hit_o.reshape(-1, 60).any(1).astype(np.uint8))
        assert torch.equal(capt.capt_collides_padded(f, sd, 60, 0.0), g60)
        acc1 |= g1
        acc60 |= g60
    assert size == whole.info()["set_total"]
    assert torch.equal(acc1, capt.capt_collides(whole, sd, 1))
    assert torch.equal(acc60, capt.capt_collides(whole, sd, 60))
    assert np.array_equal(acc60.cpu().numpy(), orc.brute_f32(pts, sph, 60))


def test_shard_clearance_combines_by_min(capt, orc):
    _say("case: clearance over 2 shards of an unpruned forest")
    cloud = synth.tabletop_cloud(50_000, 2001)
    pts = cloud[orc.filter(cloud, 0.01)[0]]
    x = dev(pts)
    r_max = 0.08
    t = orc.build_tree(pts, 0.0, r_max)
    sph = synth.uniform_spheres(8000, synth.WORKSPACE, 0.015, 0.08, 2103)
    sd = dev(sph)
    leaf = orc.query_tree(t, pts, sph)[1]
    clr_o, _, _ = orc.clearance_f64(pts, sph, r_max)
    cw, ww = capt.capt_clearance(capt.capt_build(x, 0.0, r_max), sd)
    best = torch.full_like(cw, np.inf)
    for s in range(2):
        f = capt.capt_build(x, 0.0, r_max, shard=(1, s))
        c, w = capt.capt_clearance(f, sd)
        mine = np.isin(leaf, np.array(orc.shard_leaves(t.N, 1, s)))
        c64 = c.cpu().numpy().astype(np.float64)
        assert (np.abs(c64[mine] - clr_o[mine]) <= 1e-4 * np.maximum(np.abs(clr_o[mine]), r_max)).all()
        clamp = (np.float32(r_max) - sph[~mine, 3]).astype(np.float32)
        assert np.array_equal(c.cpu().numpy()[~mine], clamp)
        assert (w.cpu().numpy()[~mine] == -1).all()
        m = torch.from_numpy(mine).cuda()
        assert torch.equal(w[m], ww[m])
        best = torch.minimum(best, c)
    assert torch.equal(best, cw)


def test_shard_of_batched_indexed_clouds_and_blob(capt, orc):
    _say("case: shard 1 of 2 over 3 clouds with indexed sets, export and import")
    clouds = [synth.tabletop_cloud(2000 + 1500 * k, 420 + k) for k in range(3)]
    off = np.cumsum([0] + [len(c) for c in clouds]).tolist()
    qs = [synth.uniform_spheres(60 * 400, synth.WORKSPACE, 0.015, 0.08, 430 + k) for k in range(3)]
    qoff = np.cumsum([0] + [len(q) for q in qs]).tolist()
    f = capt.capt_build(dev(np.concatenate(clouds)), 0.015, 0.08, cloud_off=off, indexed=True, shard=(1, 1))
    want = []
    for c, (pts, q) in enumerate(zip(clouds, qs)):
        t = orc.shard_tree(orc.build_tree(pts, 0.015, 0.08), 1, 1)
        same_tree(capt.parse_blob(capt.capt_export(f, c)), t)
        want.append(orc.query_tree(t, pts, q)[0].reshape(-1, 60).any(1).astype(np.uint8))
    sq = dev(np.concatenate(qs))
    got = capt.capt_collides(f, sq, 60, query_off=qoff).cpu().numpy()
    assert np.array_equal(got, np.concatenate(want))
    fi = capt.capt_import(capt.capt_export(f, 2))
    assert np.array_equal(capt.capt_collides(fi, dev(qs[2]), 60).cpu().numpy(), want[2])


# ---------------------------------------------------------------------------
# Full-size workloads in the benchmark's launch configuration
# ---------------------------------------------------------------------------
def test_full_size_tabletop_1M_configurations(capt, orc):
    """Tabletop at full size: the filter exactly, the GPU tree against the
    oracle's Construct array by array, and all 1,000,000 configuration answers
    against the oracle's CollisionCheck (Alg. 3) on the oracle's tree."""
    w = synth.workload(2)
    _say("case: full tabletop 1M configurations")
    xyz = dev(w.cloud)
    fx, fidx = capt.capt_filter(xyz, w.r_filter)
    keep, _ = orc.filter(w.cloud, w.r_filter)
    assert np.array_equal(fidx.cpu().numpy(), keep)
    pts = w.cloud[keep]
    assert np.array_equal(bits(fx.cpu().numpy()), bits(pts))
    f, b, t = compare_build(capt, orc, pts, w.r_min, w.r_max)
    got = capt.capt_collides(f, dev(w.spheres), 60).cpu().numpy()
    f.close()
    hit, _, _, _ = orc.query_tree(t, pts, w.spheres)
    want = hit.reshape(-1, 60).any(1).astype(np.uint8)
    assert np.array_equal(got, want)
    assert 0.3 < want.mean() < 0.95


def test_autotuned_shapes_give_identical_answers(capt, orc):
    from paper_2406_02807_amd import autotune
    pts = synth.tabletop_cloud(6000, 61)
    f = capt.capt_build(dev(pts), 0.015, 0.08)
    sph = synth.posed_spheres(synth.chain_template(2003), 2000, synth.WORKSPACE, 62)
    before = capt.capt_get_tuning()
    try:
        space = {"waves_per_group": [4, 16], "groups_per_cu": [1, 4], "lds_levels": [8, 14],
                 "scan_unroll": [1, 2, 4]}
        best, hist = autotune.autotune(f, dev(sph), 60, space=space, reps=1, rounds=1)
        assert len(hist) >= 5
        got = capt.capt_collides(f, dev(sph), 60).cpu().numpy()
        assert np.array_equal(got, orc.brute_f32(pts, sph, 60))
    finally:
        capt.capt_set_tuning(**before)


def test_full_size_room_1e8_spheres(capt, orc):
    """Room scene at full size: 1.2M points filtered at 5 mm, 10^8
    single-sphere queries.  The filter exactly; the GPU tree's splits and
    representatives against the oracle's Construct; the sets of 2,000 leaves
    (random, pruned, largest) against the direct definition (Lemma 1, case 1)
    and the r_min pruning rule (Sec. IV-B); all 10^8 answers against the
    oracle's CollisionCheck on the exported tree."""
    w = synth.workload(5)
    _say(f"case: full room {len(w.cloud)} points, {len(w.spheres)} spheres")
    xyz = dev(w.cloud)
    fx, fidx = capt.capt_filter(xyz, w.r_filter)
    keep, _ = orc.filter(w.cloud, w.r_filter)
    assert np.array_equal(fidx.cpu().numpy(), keep)
    pts = w.cloud[keep]
    f = capt.capt_build(fx.contiguous(), w.r_min, w.r_max)
    b = capt.parse_blob(capt.capt_export(f))
    _say(f"  built n={b.n} D={b.D} set entries={len(b.idx)}")
    assert np.array_equal(bits(b.points), bits(pts))
    T, rep = orc.build_splits(pts)
    assert np.array_equal(bits(b.T), bits(T)), "split values differ"
    assert np.array_equal(b.rep, rep), "representatives differ"
    cells = orc.leaf_cells(b.N, b.D, b.T)
    rng = np.random.default_rng(55)
    sizes = np.diff(b.off)
    pruned = np.flatnonzero(b.pruned)
    assert len(pruned) > 0
    big = np.argsort(sizes)[-5000:]
    sel = np.unique(np.concatenate([rng.choice(b.N, 1000, replace=False),
                                    rng.choice(pruned, min(500, len(pruned)), replace=False),
                                    rng.choice(big, 500, replace=False)]))
    off, idx = orc.afford_direct(pts, cells[sel], w.r_max)
    for k, l in enumerate(sel):
        s_gpu = np.sort(b.set_of(l))
        r = int(b.rep[l])
        real = r < b.n
        pr = real and orc.prunable(cells[l], pts[r], w.r_min)
        assert bool(b.pruned[l]) == pr, l
        if pr:
            assert s_gpu.tolist() == [r], l
        else:
            assert np.array_equal(s_gpu, idx[off[k]:off[k + 1]]), l
        if len(s_gpu):
            sp = pts[s_gpu]
            assert (b.aabb[l, :3] == sp.min(0)).all() and (b.aabb[l, 3:] == sp.max(0)).all(), l
    got = capt.capt_collides(f, dev(w.spheres), 1).cpu().numpy()
    f.close()
    want, _, _, _ = orc.query(b.N, b.D, b.T, b.aabb, b.off, b.points[b.idx], w.spheres)
    assert np.array_equal(got, want)
    assert 0.2 < want.mean() < 0.9


def _witness_ties_ok(pts, spheres, wg, wo, r_max, tol=1e-6):
    """Where the GPU's witness differs from the oracle's, both are nearest
    within `tol` m in float64, or the one that exists lies within `tol` of
    r_max while the other side clamps (R15)."""
    P = pts.astype(np.float64)
    X = spheres[:, :3].astype(np.float64)
    k = np.flatnonzero(wg != wo)
    if len(k) == 0:
        return True
    dg = np.where(wg[k] >= 0, np.linalg.norm(X[k] - P[np.maximum(wg[k], 0)], axis=1), r_max)
    do = np.where(wo[k] >= 0, np.linalg.norm(X[k] - P[np.maximum(wo[k], 0)], axis=1), r_max)
    return bool((np.abs(dg - do) <= tol).all())


def test_full_size_clearance_1M(capt, orc):
    """Clearance workload at full size: the unpruned GPU tree against the
    oracle's; every collision answer of the 10^6 spheres from capt_collides on
    that tree against the oracle's CollisionCheck (R17); every clearance
    against the float64 oracle's exact minimum over the whole cloud; every
    witness the oracle's or a float64 tie; every gradient against the float64
    gradient of the GPU's own witness."""
    w = synth.workload(4)
    _say(f"case: full clearance {len(w.spheres)} spheres")
    keep, _ = orc.filter(w.cloud, w.r_filter)
    pts = w.cloud[keep]
    f, b, t = compare_build(capt, orc, pts, 0.0, w.r_max)
    s = dev(w.spheres).requires_grad_(True)
    clr, wit = capt.clearance(f, s)
    clr.sum().backward()
    got = capt.capt_collides(f, s.detach(), 1).cpu().numpy()
    hit, _, _, _ = orc.query_tree(t, pts, w.spheres)
    assert np.array_equal(got, hit)
    P = torch.from_numpy(pts.astype(np.float64)).cuda()
    x = s.detach().double()
    wl = wit.long()
    has = wl >= 0
    d = torch.full_like(clr, w.r_max, dtype=torch.float64)
    diff = x[has, :3] - P[wl[has]]
    d[has] = diff.norm(dim=1)
    # every clearance equals the distance to its witness (clamped at r_max) minus r
    ref = torch.clamp(d, max=w.r_max) - x[:, 3]
    assert (torch.abs(clr.double() - ref) <= 1e-4 * torch.clamp(torch.abs(ref), min=w.r_max)).all()
    # the gradient of sum(clr): unit vector from the witness, -1 for the radius
    g = s.grad.double()
    gref = torch.zeros_like(g)
    inside = has & (d > 0)   # a witness within r_max; zero distance has no direction
    gref[inside, :3] = (x[inside, :3] - P[wl[inside]]) / d[inside, None]
    gref[:, 3] = -1.0
    assert (torch.linalg.norm(g - gref, dim=1) <= 1e-4 * torch.linalg.norm(gref, dim=1) + 1e-6).all()
    f.close()
    # every sphere against the exact minimum over all points
    clr_o, wit_o, _ = orc.clearance_f64(pts, w.spheres, w.r_max)
    c = clr.detach().cpu().numpy().astype(np.float64)
    assert (np.abs(c - clr_o) <= 1e-4 * np.maximum(np.abs(clr_o), w.r_max)).all()
    wg = wit.cpu().numpy()
    assert (wg == wit_o).mean() > 0.99
    assert _witness_ties_ok(pts, w.spheres, wg, wit_o, w.r_max)


def test_full_size_batched_64_clouds(capt, orc):
    """Batched workload at full size: 64 clouds, ragged query ranges, one graph
    launch and its replay; every cloud's GPU tree against the oracle's
    Construct and every answer against the oracle's CollisionCheck on that
    tree (the oracle builds run on a thread pool)."""
    import concurrent.futures as cf
    import os
    w = synth.workload(3)
    cloud_off = np.concatenate([[0], np.cumsum([len(c) for c in w.cloud])])
    query_off = np.concatenate([[0], np.cumsum([len(s) for s in w.spheres])])
    _say(f"case: full batched {len(w.cloud)} clouds, {query_off[-1]} spheres")
    xyz = dev(np.concatenate(w.cloud))
    sph = dev(np.concatenate(w.spheres))
    f = capt.capt_build(xyz, w.r_min, w.r_max, cloud_off=cloud_off)
    got = capt.capt_collides(f, sph, 60, query_off=query_off)
    again = capt.capt_collides(f, sph, 60, query_off=query_off)   # graph replay
    assert torch.equal(again, got)
    got = got.cpu().numpy()
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        futs = {ex.submit(orc.build_tree, w.cloud[c], w.r_min, w.r_max): c for c in range(len(w.cloud))}
        for fut in cf.as_completed(futs):
            c = futs[fut]
            t = fut.result()
            same_tree(capt.parse_blob(capt.capt_export(f, c)), t)
            hit, _, _, _ = orc.query_tree(t, w.cloud[c], w.spheres[c])
            want = hit.reshape(-1, 60).any(1).astype(np.uint8)
            assert np.array_equal(got[query_off[c] // 60:query_off[c + 1] // 60], want), c
            del t, hit
    f.close()


def test_depth_frame_filter_and_build(capt, orc):
    """A 640 x 480 synthetic depth frame (307,200 points): the filter at the three
    radii of the per-frame experiment against the oracle, and the tree built
    from the 1 cm frame (the largest, 56M set entries) against the oracle
    build, then queried."""
    frame = synth.depth_frame()
    xyz = dev(frame)
    kept = {}
    for rf in (0.01, 0.015, 0.02):
        _say(f"case: depth frame filter r_filter={rf}")
        fx, fidx = capt.capt_filter(xyz, rf)
        keep, _ = orc.filter(frame, rf)
        assert np.array_equal(fidx.cpu().numpy(), keep)
        kept[rf] = keep
    pts = frame[kept[0.01]]
    _say(f"case: depth frame build n={len(pts)} (1 cm filter)")
    f, b, t = compare_build(capt, orc, pts, 0.015, 0.08)
    sph = synth.uniform_spheres(60 * 2000, np.array([[-3.0, 3.0], [-3.0, 3.0], [0.0, 2.2]]), 0.015, 0.08, 7002)
    got = capt.capt_collides(f, dev(sph), 60).cpu().numpy()
    assert np.array_equal(got, orc.brute_f32(pts, sph, 60))


@pytest.mark.parametrize("edge", [1, 4, 25])
def test_posed_edges_match_oracle(capt, orc, edge):
    """Posed template queries with edge-level early exit against the oracle's
    posed spheres, and against capt_collides on the same spheres."""
    pts = synth.tabletop_cloud(20_000, 71)
    tmpl = synth.chain_template(2003).astype(np.float32)
    poses = synth.pose_edges(3000 // edge, edge, synth.WORKSPACE, 72)
    _say(f"case: posed edges edge={edge}")
    f = capt.capt_build(dev(pts), 0.015, 0.08)
    got = capt.capt_collides_posed(f, dev(tmpl), dev(poses), edge).cpu().numpy()
    sph = orc.pose_spheres(tmpl, poses)
    want = orc.brute_f32(pts, sph, edge * len(tmpl))
    assert np.array_equal(got, want)
    assert np.array_equal(capt.capt_collides(f, dev(sph), edge * len(tmpl)).cpu().numpy(), want)
    assert 0 < want.sum() < len(want) or edge > 1


def test_clearance_backward_boundary(capt, orc):
    """capt_clearance_backward writes grad_center [M, 3] and, unless NULL,
    grad_radius [M]; both against the float64 oracle's analytic gradient."""
    _say("case: clearance backward outputs, grad_radius NULL and not")
    pts = synth.tabletop_cloud(8000, 2203)
    f = capt.capt_build(dev(pts), 0.0, 0.08)
    sph = synth.uniform_spheres(5000, synth.WORKSPACE, 0.015, 0.08, 2204)
    s = dev(sph)
    clr, wit = capt.capt_clearance(f, s)
    g = torch.linspace(-2.0, 3.0, len(sph), device="cuda", dtype=torch.float32)
    gc, gr = capt.capt_clearance_backward(f, s, wit, g)
    gc2, none = capt.capt_clearance_backward(f, s, wit, g, radius=False)
    assert none is None and torch.equal(gc, gc2)
    assert torch.equal(gr, -g)
    _, wit_o, grad_o = orc.clearance_f64(pts, sph, 0.08)
    w = wit.cpu().numpy()
    same = w == wit_o
    assert same.mean() > 0.99
    assert _witness_ties_ok(pts, sph, w, wit_o, 0.08)
    # the reference gradient is the float64 one of the GPU's own witness: the
    # oracle's where the witnesses agree, recomputed where they tie (R15)
    gs = g.cpu().numpy().astype(np.float64)
    ref = grad_o * gs[:, None]
    k = np.flatnonzero(~same & (w >= 0))
    dv = sph[k, :3].astype(np.float64) - pts[w[k]].astype(np.float64)
    nv = np.linalg.norm(dv, axis=1)
    ref[k] = np.where(nv[:, None] > 0, dv / np.where(nv > 0, nv, 1.0)[:, None], 0.0) * gs[k, None]
    ref[~same & (w < 0)] = 0.0
    err = np.linalg.norm(gc.cpu().numpy().astype(np.float64) - ref, axis=1)
    assert (err <= 1e-4 * np.linalg.norm(ref, axis=1) + 1e-6).all()
    assert (gc.cpu().numpy()[w < 0] == 0).all()
