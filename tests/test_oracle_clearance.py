"""Pins for the oracle's clearance (nearest-point distance clamped at r_max,
minus r) and its gradient.

- one-point clouds: closed form with Pythagorean distances;
- two-point clouds: the witness switches on the bisector plane, ties go to the
  smaller index;
- float64 central differences (h = 1e-5) against the analytic gradient away
  from kinks;
- on an unpruned tree, the minimum over the leaf's affordance set equals the
  global minimum whenever it is below r_max (Lemma 1, case 1).
"""
import numpy as np

import synth


def test_single_point_closed_form(orc):
    pts = np.array([[1.0, 2.0, 3.0]], np.float32)
    sph = np.array([[4.0, 6.0, 3.0, 1.0],      # distance 5 < r_max = 8
                    [1.0, 2.0, 3.0, 0.5],      # on the point
                    [1.0, 2.0, 15.0, 2.0],     # distance 12 >= 8 -> clamped
                    [1.0, 2.0, 11.0, 2.0]],    # distance 8 == r_max -> clamped
                   np.float32)
    clr, wit, grad = orc.clearance_f64(pts, sph, 8.0)
    assert clr.tolist() == [4.0, -0.5, 6.0, 6.0]
    assert wit.tolist() == [0, 0, -1, -1]
    assert np.allclose(grad, [[0.6, 0.8, 0.0], [0, 0, 0], [0, 0, 0], [0, 0, 0]], atol=0)


def test_two_point_bisector_and_tie(orc):
    pts = np.array([[0, 0, 0], [1, 0, 0]], np.float32)
    xs = np.array([0.25, 0.5, 0.75], np.float32)
    sph = np.stack([xs, np.full(3, 0.0), np.full(3, 0.0), np.full(3, 0.125)], 1).astype(np.float32)
    clr, wit, grad = orc.clearance_f64(pts, sph, 1.0)
    assert wit.tolist() == [0, 0, 1]          # exact tie at x = 0.5 -> smaller index
    assert clr.tolist() == [0.125, 0.375, 0.125]
    assert grad[:, 0].tolist() == [1.0, 1.0, -1.0]


def _fd_grad(orc, pts, sph, r_max, h=1e-5):
    """Central differences in float64 of the float64 clearance definition."""
    g = np.zeros((len(sph), 3))
    P = pts.astype(np.float64)
    for a in range(3):
        for sgn in (+1, -1):
            x = sph[:, :3].astype(np.float64).copy()
            x[:, a] += sgn * h
            d = np.sqrt(((x[:, None, :] - P[None]) ** 2).sum(-1)).min(1)
            c = np.minimum(d, r_max) - sph[:, 3]
            g[:, a] += sgn * c / (2 * h)
    return g


def test_fd_matches_analytic_gradient(orc):
    pts = synth.tabletop_cloud(3000, 21)
    sph = synth.uniform_spheres(3000, synth.WORKSPACE, 0.015, 0.08, 22)
    r_max = 0.08
    clr, wit, grad = orc.clearance_f64(pts, sph, r_max)
    P = pts.astype(np.float64)
    d = np.sqrt(((sph[:, None, :3].astype(np.float64) - P[None]) ** 2).sum(-1))
    ds = np.sort(d, 1)
    ok = (ds[:, 1] - ds[:, 0] > 1e-4) & (np.abs(ds[:, 0] - r_max) > 1e-4) & (ds[:, 0] > 1e-3)
    sel = np.where(ok)[0][:1000]
    assert len(sel) >= 500
    fd = _fd_grad(orc, pts, sph[sel], r_max)
    err = np.linalg.norm(fd - grad[sel], axis=1)
    assert (err <= 1e-4 * np.linalg.norm(grad[sel], axis=1) + 1e-6).all()
    # both clamped and unclamped spheres are present
    assert (wit[sel] >= 0).any() and (wit[sel] < 0).any()


def test_affordance_set_minimum_equals_global(orc):
    pts = synth.tabletop_cloud(2500, 31)
    r_max = 0.08
    t = orc.build_tree(pts, 0.0, r_max)
    sph = synth.uniform_spheres(4000, synth.WORKSPACE, 0.015, 0.08, 32)
    clr, wit, _ = orc.clearance_f64(pts, sph, r_max)
    _, leaf, _, _ = orc.query_tree(t, pts, sph)
    P = pts.astype(np.float64)
    for s in range(len(sph)):
        idx = t.set_of(leaf[s])
        x = sph[s, :3].astype(np.float64)
        if len(idx):
            d2 = ((x - P[idx]) ** 2).sum(-1)
            k = np.argmin(d2)
            dmin = np.sqrt(d2[k])
        else:
            dmin = np.inf
        if dmin < r_max:
            assert wit[s] >= 0 and P[wit[s]].tolist() == P[idx[k]].tolist()
            assert dmin - np.float64(sph[s, 3]) == clr[s]
        else:
            assert wit[s] == -1
