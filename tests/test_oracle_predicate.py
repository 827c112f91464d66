"""Pins for the oracle's collision predicate and brute force (O1, O2).

The float32 predicate is checked against hand-worked IEEE cases (including the
summation order) and against exact integer arithmetic on dyadic inputs where
every float32 operation is exact; the float64 variant is checked against the
float32 one through the mismatch band |d^2 - r^2| < 1e-6 r^2.
"""
import numpy as np
import pytest

from conftest import golden

pytestmark = pytest.mark.filterwarnings("ignore")


def test_hand_worked_predicates(orc):
    g = golden("morton_and_predicates.json")
    for case in g["predicate"]:
        s = np.array([case["sphere"]], dtype=np.float32)
        p = np.array([case["point"]], dtype=np.float32)
        got = orc.brute_f32(p, s)[0]
        assert got == case["hit"], case
        f64, _ = orc.brute_f64(p, s)
        assert f64[0] == case["exact"], case


def test_dyadic_inputs_match_exact_integer_arithmetic(orc):
    # Coordinates are multiples of 2^-8 in [0, 1] and radii multiples of 2^-8:
    # every difference, square and sum is exact in float32, so the float32
    # predicate must equal the exact answer computed with Python integers.
    rng = np.random.default_rng(7)
    pts_i = rng.integers(0, 257, size=(300, 3))
    sph_i = rng.integers(-16, 273, size=(400, 3))
    rad_i = rng.integers(1, 40, size=400)
    pts = (pts_i / 256.0).astype(np.float32)
    sph = np.concatenate([sph_i / 256.0, rad_i[:, None] / 256.0], axis=1).astype(np.float32)
    got = orc.brute_f32(pts, sph)
    d2 = ((sph_i[:, None, :] - pts_i[None, :, :]) ** 2).sum(-1)   # exact, units of 2^-16
    want = (d2 <= (rad_i ** 2)[:, None]).any(1).astype(np.uint8)
    assert (got == want).all()
    # per-configuration OR
    got4 = orc.brute_f32(pts, sph, group=4)
    assert (got4 == want.reshape(-1, 4).max(1)).all()


def test_fp32_vs_fp64_band(orc):
    # Any disagreement between the float32 and float64 answers needs a witness
    # point within the band |d^2 - r^2| < 1e-6 r^2.
    import synth
    pts = synth.tabletop_cloud(1500, 11)
    sph = synth.uniform_spheres(200_000, synth.WORKSPACE, 0.015, 0.08, 12)
    f32 = orc.brute_f32(pts, sph)
    f64, margin = orc.brute_f64(pts, sph)
    diff = f32 != f64
    assert (margin[diff] < 1e-6).all()
    assert 0.05 < f32.mean() < 0.95


def test_band_cases_exist_and_are_explained(orc):
    # Spheres placed exactly on a point's distance shell: float32 and float64
    # may disagree, but only inside the band.
    rng = np.random.default_rng(3)
    pts = rng.random((64, 3)).astype(np.float32)
    dirs = rng.normal(size=(2000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    r = rng.uniform(0.01, 0.05, 2000)
    base = pts[rng.integers(0, 64, 2000)].astype(np.float64)
    sph = np.concatenate([base + dirs * r[:, None], r[:, None]], axis=1).astype(np.float32)
    f32 = orc.brute_f32(pts, sph)
    f64, margin = orc.brute_f64(pts, sph)
    assert (margin[f32 != f64] < 1e-6).all()
    assert np.median(margin) < 1e-6   # the construction really sits on the boundary


def test_nonfinite_centres_never_collide(orc):
    pts = np.array([[0, 0, 0], [1, 1, 1]], dtype=np.float32)
    sph = np.array([[np.nan, 0, 0, 1], [np.inf, 0, 0, 1], [-np.inf, 1, 1, 1],
                    [0, np.nan, 0, 0.5]], dtype=np.float32)
    assert orc.brute_f32(pts, sph).tolist() == [0, 0, 0, 0]


def test_empty_cloud(orc):
    pts = np.zeros((0, 3), dtype=np.float32)
    sph = np.array([[0, 0, 0, 1]], dtype=np.float32)
    assert orc.brute_f32(pts, sph).tolist() == [0]
