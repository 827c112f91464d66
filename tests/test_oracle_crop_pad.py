"""Pins for the oracle's reach crop and query padding (the filter variants of
Sec. IV-C and Sec. V-B).

- crop: points at hand-chosen distances around the boundary, reach = inf as
  the identity, and the paper's reason for the crop: a sphere that lies inside
  the reach ball answers the same on the cropped cloud as on the full one;
- padding: the filter lemma's argument (a point is dropped only when a kept
  point lies within r_filter of it) makes the padded query conservative: one
  pass with pad = r_filter, six passes with pad = 6 r_filter (the drops chain
  over the passes), checked against float64 brute force on the unfiltered
  cloud; and the padding is not vacuous (without it some collisions are lost).
"""
import numpy as np

import synth


def test_crop_boundary_hand_example(orc):
    # squared distances to the base (1, 2, 3): 1.0 (on the boundary, kept),
    # 0.25, (1 + 2^-23)^2 > 1 (cropped), 0.81, NaN (cropped), 1.0 along z
    p = np.array([[2, 2, 3], [1.5, 2, 3], [2.0000002, 2, 3], [1, 2, 3.9], [np.nan, 2, 3], [1, 2, 4]],
                 np.float32)
    assert orc.crop(p, [1, 2, 3], 1.0).tolist() == [0, 1, 3, 5]
    assert orc.crop(p, [1, 2, 3], 0.5).tolist() == [1]
    assert orc.crop(p, [10, 10, 10], 1.0).tolist() == []


def test_crop_infinite_reach_is_identity(orc):
    pts = synth.tabletop_cloud(4000, 31)
    a, ca = orc.filter(pts, 0.02)
    b, cb = orc.filter(pts, 0.02, base=[0.1, -0.2, 0.3], reach=np.inf)
    assert np.array_equal(a, b) and np.array_equal(ca, cb)


def test_crop_keeps_answers_inside_the_reach_ball(orc):
    pts = synth.tabletop_cloud(8000, 32)
    base = np.array([0.0, 0.0, 0.4], np.float32)
    reach = 0.8
    kept, _ = orc.filter(pts, 0.0, base=base, reach=reach)   # r_filter = 0: the crop alone
    assert 0 < len(kept) < len(pts)
    d = np.sqrt(((pts[kept].astype(np.float64) - base) ** 2).sum(-1))
    assert (d <= reach * (1 + 1e-6)).all()
    rng = np.random.default_rng(33)
    r = rng.uniform(0.015, 0.08, 3000)
    u = rng.normal(size=(3000, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    c = base + u * (rng.uniform(0, 1, (3000, 1)) * (reach - r[:, None] - 1e-3))   # inside the ball
    sph = np.concatenate([c, r[:, None]], 1).astype(np.float32)
    full = orc.brute_f32(pts, sph)
    assert full.sum() > 0
    assert np.array_equal(orc.brute_f32(pts[kept], sph), full)


def _spheres(n, seed):
    return synth.uniform_spheres(n, synth.WORKSPACE, 0.015, 0.08, seed)


def test_padding_is_conservative(orc):
    pts = synth.tabletop_cloud(6000, 34)
    sph = _spheres(20000, 35)
    hit64, margin = orc.brute_f64(pts, sph)
    clear = hit64.astype(bool) & (margin > 1e-4)   # collisions away from the float32 boundary
    assert clear.sum() > 1000
    rf = 0.02
    for npass, pad in ((1, rf), (6, 6 * rf)):
        kept, _ = orc.filter(pts, rf, npass=npass)
        padded = orc.brute_f32(pts[kept], sph, pad=pad).astype(bool)
        assert padded[clear].all(), (npass, pad)
    # without padding the filtered cloud misses some of those collisions
    kept, _ = orc.filter(pts, rf)
    assert not orc.brute_f32(pts[kept], sph).astype(bool)[clear].all()


def test_pad_radii_is_one_float32_add(orc):
    sph = np.array([[0, 0, 0, 0.1], [1, 1, 1, 0.3]], np.float32)
    out = orc.pad_radii(sph, 0.2)
    assert out[:, 3].tolist() == [np.float32(np.float32(0.1) + np.float32(0.2)),
                                  np.float32(np.float32(0.3) + np.float32(0.2))]
    assert np.array_equal(out[:, :3], sph[:, :3])
    assert np.array_equal(orc.pad_radii(sph, 0.0), sph)
