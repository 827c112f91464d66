"""Pins for the oracle's posed template spheres (the posed query's input
definition): float32 products and sums in a fixed order.

- an independent float32 evaluation with numpy (every array operation rounds
  to float32), bit for bit;
- identity pose and pure translations leave the template's offsets exact
  where the sums are exact;
- a quarter turn about z permutes and negates coordinates exactly;
- the edge generator interpolates: the first and last configuration of an
  edge are its endpoints, every rotation is orthonormal to float32 accuracy.
"""
import numpy as np

import synth


def test_pose_spheres_match_float32_numpy(orc):
    rng = np.random.default_rng(3)
    tm = np.concatenate([rng.uniform(-0.5, 0.5, (37, 3)), rng.uniform(0.01, 0.1, (37, 1))], 1).astype(np.float32)
    poses = synth.pose_edges(50, 3, synth.WORKSPACE, 11)
    got = orc.pose_spheres(tm, poses)
    R = poses[:, :9].reshape(-1, 3, 3)
    t = poses[:, 9:]
    want = np.empty_like(got).reshape(len(poses), len(tm), 4)
    for i in range(3):
        a = R[:, i, 0][:, None] * tm[None, :, 0]
        b = R[:, i, 1][:, None] * tm[None, :, 1]
        s = a + b
        s = s + R[:, i, 2][:, None] * tm[None, :, 2]
        want[:, :, i] = s + t[:, i][:, None]
    want[:, :, 3] = tm[None, :, 3]
    assert want.dtype == np.float32
    assert np.array_equal(got.view(np.uint32), want.reshape(-1, 4).view(np.uint32))


def test_identity_translation_and_quarter_turn(orc):
    tm = np.array([[0.25, -0.5, 0.125, 0.05], [1.0, 2.0, -3.0, 0.02]], np.float32)
    ident = np.array([[1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0]], np.float32)
    assert np.array_equal(orc.pose_spheres(tm, ident), tm)
    shift = ident.copy()
    shift[0, 9:] = [0.5, 0.25, -1.0]
    got = orc.pose_spheres(tm, shift)
    assert np.array_equal(got[:, :3], tm[:, :3] + np.float32([0.5, 0.25, -1.0]))
    quarter = np.array([[0, -1, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0]], np.float32)   # +90 degrees about z
    got = orc.pose_spheres(tm, quarter)
    assert np.array_equal(got[:, 0], -tm[:, 1]) and np.array_equal(got[:, 1], tm[:, 0])
    assert np.array_equal(got[:, 2], tm[:, 2]) and np.array_equal(got[:, 3], tm[:, 3])


def test_edges_interpolate_between_endpoints():
    e = synth.pose_edges(20, 8, synth.WORKSPACE, 5).reshape(20, 8, 12).astype(np.float64)
    R = e[:, :, :9].reshape(20, 8, 3, 3)
    eye = np.einsum("eskj,eslj->eskl", R, R)
    assert np.abs(eye - np.eye(3)).max() < 1e-6
    t = e[:, :, 9:]
    steps = np.diff(t, axis=1)
    assert np.allclose(steps, steps[:, :1], atol=1e-6)   # constant translation steps
    one = synth.pose_edges(20, 1, synth.WORKSPACE, 5)
    assert one.shape == (20, 12)
