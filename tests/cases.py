"""Seeded clouds and query sets shared by the parity tests (inputs only)."""
import numpy as np

import synth


def adversarial_clouds():
    rng = np.random.default_rng(5)
    lat = np.stack(np.meshgrid(*[np.arange(6)] * 3, indexing="ij"), -1).reshape(-1, 3)
    return {
        "uniform-1000": rng.random((1000, 3)).astype(np.float32),
        "uniform-37": rng.random((37, 3)).astype(np.float32),
        "lattice-216": lat.astype(np.float32) * np.float32(0.02),
        "dups-300": np.repeat(rng.random((60, 3)), 5, axis=0).astype(np.float32) * np.float32(0.2),
        "collinear-129": np.stack([np.linspace(0, 0.3, 129), np.zeros(129), np.zeros(129)], 1).astype(np.float32),
        "coplanar-500": np.concatenate([rng.random((500, 2)) * 0.3, np.zeros((500, 1))], 1).astype(np.float32),
        "identical-64": np.full((64, 3), 0.25, np.float32),
        "single": np.array([[0.5, 0.25, 0.125]], np.float32),
        "pair": np.array([[0, 0, 0], [0.01, 0, 0]], np.float32),
        "three": rng.random((3, 3)).astype(np.float32),
        "pow2-4096": rng.random((4096, 3)).astype(np.float32),
        "pow2p1-4097": rng.random((4097, 3)).astype(np.float32),
        "tabletop-9000": synth.tabletop_cloud(9000, 77),
        "negzero": np.array([[-0.0, 0.0, 0.0], [0.0, -0.0, 0.0], [0.0, 0.0, -0.0], [0.01, 0, 0], [-0.01, 0, 0]], np.float32),
    }


def mixed_queries(pts, r_min, r_max, m, seed, tree=None):
    """Random spheres around the cloud, plus spheres centred on cloud points,
    on split planes and on leaf-cell corners (when a tree is given), with radii
    at r_min, r_max and in between."""
    rng = np.random.default_rng(seed)
    lo = pts.min(0).astype(np.float64) - r_max * 2
    hi = pts.max(0).astype(np.float64) + r_max * 2
    cen = [lo + rng.random((m, 3)) * (hi - lo)]
    cen.append(pts[rng.integers(0, len(pts), m // 4)].astype(np.float64))
    if tree is not None and tree.N > 1:
        cells = np.where(np.isfinite(tree.cell), tree.cell, 0.0)
        ls = rng.integers(0, tree.N, m // 4)
        pick = rng.random((len(ls), 3)) < 0.5
        cen.append(np.where(pick, cells[ls, :3], cells[ls, 3:]))
        nodes = rng.integers(0, tree.N - 1, m // 4)
        q = pts[rng.integers(0, len(pts), len(nodes))].astype(np.float64)
        depth = np.floor(np.log2(nodes + 1)).astype(int)
        tv = tree.T[nodes]
        ok = np.isfinite(tv)
        q[np.arange(len(nodes))[ok], (depth % 3)[ok]] = tv[ok]
        cen.append(q)
    cen = np.concatenate(cen)
    r = rng.uniform(r_min, r_max, len(cen))
    k = rng.random(len(cen))
    r = np.where(k < 0.15, r_min, np.where(k < 0.3, r_max, r))
    return np.concatenate([cen, r[:, None]], 1).astype(np.float32)


def nonfinite_queries(r):
    return np.array([[np.nan, 0.5, 0.5, r], [0.5, np.nan, 0.5, r], [np.inf, 0.5, 0.5, r],
                     [-np.inf, -np.inf, -np.inf, r], [0.5, 0.5, np.nan, r], [np.inf, np.inf, np.inf, r]],
                    np.float32)
