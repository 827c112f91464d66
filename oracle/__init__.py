"""CPU oracle for collision-affording point trees.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports or
links this package, and this package never imports the product.

The arithmetic lives in `capt_oracle.c` (plain C, float64 where the paper does
not fix the precision, float32 for the collision predicate the GPU must match
bit for bit); this module compiles it with gcc and marshals numpy arrays.

Functions and what they follow:
  brute_f32        plain definition of the collision answer (Alg. 3's test
                   against every point of the cloud; Lemma 1's right-hand side)
  brute_f64        the same test in float64, with the relative margin
                   |d^2 - r^2| / r^2 of the closest-to-boundary point
  clearance_f64    nearest-point distance clamped at r_max, minus r, and its
                   gradient (not in the paper; defined for the differentiable
                   query)
  prunable         Construct's r_min pruning test for one leaf (Sec. IV-B)
  build_tree       Construct (Alg. 1, Sec. IV-A/B) with r_min pruning; split
                   axis d mod 3, or a given axis per depth (the alternative
                   to the cyclic rule that Sec. IV-A mentions)
  build_splits     Construct's splits alone (T and representatives)
  leaf_cells       every leaf's closed cell from the test sequence (Alg. 1)
  afford_direct    the affordance set of given cells by its direct definition
                   (Lemma 1, case 1)
  query            CollisionCheck (Alg. 3, Sec. IV-D) on a tree given as arrays
  morton_key       Z-order key (Sec. II-B, Sec. IV-C)
  filter           Filter (Alg. 2, Sec. IV-C), optionally after crop
  crop             reach crop for fixed-base arms (Sec. IV-C)
  pad_radii        query padding r + r_filter (Sec. V-B, after the filter
                   lemma)
  shard_tree       one shard of a tree (Sec. VII: CAPTs each responsible for
                   a neighbourhood of a large cloud): the whole tree with the
                   sets of every leaf outside the shard's subtree emptied
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "capt_oracle.c")
# CAPT_ORACLE_LIB names a prebuilt copy to load instead (the sanitizer test
# builds one with AddressSanitizer and UBSan); it is never recompiled here.
_LIB = os.environ.get("CAPT_ORACLE_LIB") or os.path.join(_HERE, "libcapt_oracle.so")
_PREBUILT = bool(os.environ.get("CAPT_ORACLE_LIB"))
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wextra"]

_lib = None


def compile_library(force: bool = True) -> str:
    """Compile the oracle with gcc (contraction off, no fast-math)."""
    if _PREBUILT:
        return _LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not _PREBUILT and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            compile_library(force=True)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32, f32 = C.c_int64, C.c_int32, C.c_float
        sig = {
            "orc_sqdist_f32": (f32, [P, P]),
            "orc_brute_f32": (None, [P, i64, P, i64, i32, P]),
            "orc_pose_spheres": (None, [P, i32, P, i64, P]),
            "orc_brute_f64": (None, [P, i64, P, i64, P, P]),
            "orc_clearance_f64": (None, [P, i64, P, i64, f32, P, P, P]),
            "orc_build": (P, [P, i64, f32, f32, C.c_int, P]),
            "orc_tree_dims": (None, [P, P, P, P, P]),
            "orc_tree_copy": (None, [P, P, P, P, P, P, P, P]),
            "orc_tree_free": (None, [P]),
            "orc_query": (None, [i64, i32, P, P, P, P, P, i64, P, P, P, P, P]),
            "orc_query_serial": (None, [i64, i32, P, P, P, P, P, i64, i32, P, P]),
            "orc_morton_key": (C.c_uint64, [P, C.c_int]),
            "orc_morton_grid": (None, [P, i64, P, P]),
            "orc_morton_cell": (None, [P, P, C.c_double, P]),
            "orc_filter": (i64, [P, i64, f32, C.c_int, P, P]),
            "orc_prunable": (C.c_int, [P, P, f32]),
            "orc_set_threads": (None, [i32]),
            "orc_build_splits": (None, [P, i64, P, P, P]),
            "orc_leaf_cells": (None, [i64, i32, P, P, P]),
            "orc_afford_count": (None, [P, i64, P, i64, f32, P]),
            "orc_afford_fill": (None, [P, i64, P, i64, f32, P, P]),
            "orc_max_threads": (i32, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a, cols):
    a = np.ascontiguousarray(a, dtype=np.float32)
    assert a.ndim == 2 and a.shape[1] == cols, a.shape
    return a


def sqdist_f32(a, b) -> np.float32:
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    return np.float32(_load().orc_sqdist_f32(_p(a), _p(b)))


def pad_radii(spheres, pad: float) -> np.ndarray:
    """Query padding (Sec. V-B, after the filter lemma): every radius r
    becomes r + pad, one float32 addition."""
    sph = _f32(spheres, 4).copy()
    sph[:, 3] = sph[:, 3] + np.float32(pad)
    return sph


def brute_f32(points, spheres, group: int = 1, pad: float = 0.0) -> np.ndarray:
    pts, sph = _f32(points, 3), _f32(spheres, 4)
    if pad:
        sph = pad_radii(sph, pad)
    assert len(sph) % group == 0
    out = np.zeros(len(sph) // group, dtype=np.uint8)
    _load().orc_brute_f32(_p(pts), len(pts), _p(sph), len(sph), group, _p(out))
    return out


def prunable(cell, rep, r_min: float) -> bool:
    """The r_min pruning test of Construct (Alg. 1, Sec. IV-B) for one leaf:
    closed cell [lo xyz, hi xyz] (float32, all finite) and representative t:
    the float64 squared distance from t to the cell's farthest corner is at
    most r_min^2 (1 - 2^-18), r_min > 0."""
    c = np.ascontiguousarray(cell, dtype=np.float32).reshape(6)
    t = np.ascontiguousarray(rep, dtype=np.float32).reshape(3)
    return bool(_load().orc_prunable(_p(c), _p(t), np.float32(r_min)))


def pose_spheres(template, poses) -> np.ndarray:
    """Template spheres [g, 4] under rigid poses [P, 12] (row-major rotation,
    then translation), float32 arithmetic in the posed query's order:
    float32 [P * g, 4], configuration-major."""
    tm = _f32(template, 4)
    ps = _f32(poses, 12)
    out = np.zeros((len(ps) * len(tm), 4), dtype=np.float32)
    _load().orc_pose_spheres(_p(tm), len(tm), _p(ps), len(ps), _p(out))
    return out


def brute_f64(points, spheres):
    pts, sph = _f32(points, 3), _f32(spheres, 4)
    out = np.zeros(len(sph), dtype=np.uint8)
    margin = np.zeros(len(sph), dtype=np.float64)
    _load().orc_brute_f64(_p(pts), len(pts), _p(sph), len(sph), _p(out), _p(margin))
    return out, margin


def clearance_f64(points, spheres, r_max: float):
    pts, sph = _f32(points, 3), _f32(spheres, 4)
    m = len(sph)
    clr = np.zeros(m, dtype=np.float64)
    wit = np.zeros(m, dtype=np.int32)
    grad = np.zeros((m, 3), dtype=np.float64)
    _load().orc_clearance_f64(_p(pts), len(pts), _p(sph), m, np.float32(r_max),
                              _p(clr), _p(wit), _p(grad))
    return clr, wit, grad


@dataclass
class Tree:
    """A CAPT as plain arrays (Sec. IV-A): n real points padded to N = 2^D."""
    n: int
    N: int
    D: int
    r_min: float
    r_max: float
    T: np.ndarray        # float32 [N-1], Eytzinger order
    rep: np.ndarray      # int32 [N], representative per leaf (>= n: padding)
    cell: np.ndarray     # float32 [N, 6] lo xyz, hi xyz
    aabb: np.ndarray     # float32 [N, 6] lo xyz, hi xyz of the stored set
    pruned: np.ndarray   # uint8 [N]
    off: np.ndarray      # int64 [N+1]
    idx: np.ndarray      # int32 [off[N]], each set sorted by original index
    axes: np.ndarray = None   # uint8 [D] split axis per depth (None: d mod 3)

    def set_of(self, leaf: int) -> np.ndarray:
        return self.idx[self.off[leaf]:self.off[leaf + 1]]


def _axes(axes):
    return None if axes is None else np.ascontiguousarray(axes, dtype=np.uint8)


def build_tree(points, r_min: float, r_max: float, prune: bool = True, axes=None) -> Tree:
    """Construct; `axes` gives the split axis of each depth (default d mod 3)."""
    pts = _f32(points, 3)
    lib = _load()
    ax = _axes(axes)
    h = lib.orc_build(_p(pts), len(pts), np.float32(r_min), np.float32(r_max), int(prune), _p(ax))
    try:
        n, N, D, tot = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int64()
        lib.orc_tree_dims(h, C.byref(n), C.byref(N), C.byref(D), C.byref(tot))
        N_ = N.value
        T = np.zeros(max(N_ - 1, 0), dtype=np.float32)
        rep = np.zeros(N_, dtype=np.int32)
        cell = np.zeros((N_, 6), dtype=np.float32)
        aabb = np.zeros((N_, 6), dtype=np.float32)
        pruned = np.zeros(N_, dtype=np.uint8)
        off = np.zeros(N_ + 1, dtype=np.int64)
        idx = np.zeros(max(tot.value, 1), dtype=np.int32)
        lib.orc_tree_copy(h, _p(T) if N_ > 1 else None, _p(rep), _p(cell), _p(aabb),
                          _p(pruned), _p(off), _p(idx))
    finally:
        lib.orc_tree_free(h)
    return Tree(n.value, N_, D.value, float(np.float32(r_min)), float(np.float32(r_max)),
                T, rep, cell, aabb, pruned, off, idx[:tot.value], None if ax is None else ax[:D.value].copy())


def build_splits(points, axes=None):
    """Construct's splits alone (Sec. IV-A): (T float32 [N-1], rep int32 [N])."""
    pts = _f32(points, 3)
    n = len(pts)
    N = 1
    while N < n:
        N <<= 1
    T = np.zeros(max(N - 1, 1), dtype=np.float32)
    rep = np.zeros(N, dtype=np.int32)
    _load().orc_build_splits(_p(pts), n, _p(_axes(axes)), _p(T), _p(rep))
    return T[:N - 1], rep


def leaf_cells(N: int, D: int, T, axes=None) -> np.ndarray:
    """Closed cell [N, 6] (lo xyz, hi xyz) of every leaf from the test sequence."""
    T = np.ascontiguousarray(T, dtype=np.float32)
    cells = np.zeros((N, 6), dtype=np.float32)
    _load().orc_leaf_cells(N, D, _p(T) if len(T) else None, _p(_axes(axes)), _p(cells))
    return cells


def afford_direct(points, cells, r_max: float):
    """Lemma 1, case 1: for each cell, every point it affords at r_max
    (float64 distance to the closed cell <= r_max (1 + 2^-20)).  Returns
    (off int64 [k+1], idx int32 [off[k]]), members in increasing order."""
    pts = _f32(points, 3)
    cells = np.ascontiguousarray(cells, dtype=np.float32).reshape(-1, 6)
    k = len(cells)
    cnt = np.zeros(k, dtype=np.int64)
    lib = _load()
    lib.orc_afford_count(_p(pts), len(pts), _p(cells), k, np.float32(r_max), _p(cnt))
    off = np.zeros(k + 1, dtype=np.int64)
    off[1:] = np.cumsum(cnt)
    idx = np.zeros(max(int(off[-1]), 1), dtype=np.int32)
    lib.orc_afford_fill(_p(pts), len(pts), _p(cells), k, np.float32(r_max), _p(off), _p(idx))
    return off, idx[:off[-1]]


def query(N: int, D: int, T, aabb, off, setxyz, spheres, axes=None):
    """CollisionCheck (Alg. 3) per sphere on a tree given as arrays.  Returns
    (hit u8 [m], leaf i32 [m], aabb_rejected u8 [m], scanned i32 [m]).
    `axes`: split axis per depth (default d mod 3)."""
    sph = _f32(spheres, 4)
    m = len(sph)
    T = np.ascontiguousarray(T, dtype=np.float32)
    aabb = np.ascontiguousarray(aabb, dtype=np.float32).reshape(-1, 6)
    off = np.ascontiguousarray(off, dtype=np.int64)
    setxyz = np.ascontiguousarray(setxyz, dtype=np.float32).reshape(-1, 3)
    hit = np.zeros(m, dtype=np.uint8)
    leaf = np.zeros(m, dtype=np.int32)
    rej = np.zeros(m, dtype=np.uint8)
    scanned = np.zeros(m, dtype=np.int32)
    _load().orc_query(N, D, _p(T) if len(T) else None, _p(aabb), _p(off),
                      _p(setxyz) if len(setxyz) else None, _p(sph), m,
                      _p(hit), _p(leaf), _p(rej), _p(scanned), _p(_axes(axes)))
    return hit, leaf, rej, scanned


def shard_leaves(N: int, bits: int, shard: int) -> range:
    """Leaves l of a tree with N leaves that shard `shard` of 2**bits answers
    for: floor(l * 2**bits / N) == shard.  For bits <= log2 N they are the
    leaves under the depth-`bits` node `shard`; for more bits, every leaf
    is its own shard and the other shards hold none."""
    return range(-(-shard * N // 2 ** bits), -(-(shard + 1) * N // 2 ** bits))


def shard_tree(tree: Tree, bits: int, shard: int) -> Tree:
    """Shard `shard` of 2**bits of `tree`: splits, cells and representatives
    unchanged; every leaf outside shard_leaves keeps no set (count 0, the
    empty box lo = +inf, hi = -inf) and no pruning mark."""
    mine = np.zeros(tree.N, dtype=bool)
    mine[shard_leaves(tree.N, bits, shard)] = True
    cnt = np.where(mine, np.diff(tree.off), 0)
    off = np.zeros(tree.N + 1, dtype=np.int64)
    off[1:] = np.cumsum(cnt)
    idx = np.concatenate([tree.set_of(l) for l in range(tree.N) if mine[l]] + [np.zeros(0, np.int32)])
    aabb = tree.aabb.copy()
    aabb[~mine, :3] = np.inf
    aabb[~mine, 3:] = -np.inf
    pruned = np.where(mine, tree.pruned, 0).astype(np.uint8)
    return Tree(tree.n, tree.N, tree.D, tree.r_min, tree.r_max, tree.T.copy(), tree.rep.copy(),
                tree.cell.copy(), aabb, pruned, off, idx.astype(np.int32), tree.axes)


def query_tree(tree: Tree, points, spheres):
    """Alg. 3 on an oracle tree; set points are stored in sorted-index order."""
    pts = _f32(points, 3)
    return query(tree.N, tree.D, tree.T, tree.aabb, tree.off, pts[tree.idx], spheres, tree.axes)


def query_serial(N: int, D: int, T, aabb, off, setxyz, spheres, group: int, axes=None) -> np.ndarray:
    """Single-threaded Alg. 3 with per-configuration early exit."""
    sph = _f32(spheres, 4)
    T = np.ascontiguousarray(T, dtype=np.float32)
    aabb = np.ascontiguousarray(aabb, dtype=np.float32).reshape(-1, 6)
    off = np.ascontiguousarray(off, dtype=np.int64)
    setxyz = np.ascontiguousarray(setxyz, dtype=np.float32).reshape(-1, 3)
    out = np.zeros(len(sph) // group, dtype=np.uint8)
    _load().orc_query_serial(N, D, _p(T) if len(T) else None, _p(aabb), _p(off),
                             _p(setxyz) if len(setxyz) else None, _p(sph), len(sph),
                             group, _p(out), _p(_axes(axes)))
    return out


def set_threads(k: int) -> None:
    """Thread count of the oracle's OpenMP loops."""
    _load().orc_set_threads(int(k))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def morton_key(q, perm: int) -> int:
    q = np.ascontiguousarray(q, dtype=np.uint32)
    return int(_load().orc_morton_key(_p(q), perm))


def morton_grid(points):
    pts = _f32(points, 3)
    lo = np.zeros(3, dtype=np.float32)
    scale = C.c_double()
    _load().orc_morton_grid(_p(pts), len(pts), _p(lo), C.byref(scale))
    return lo, scale.value


def morton_cell(p, lo, scale: float) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float32)
    lo = np.ascontiguousarray(lo, dtype=np.float32)
    q = np.zeros(3, dtype=np.uint32)
    _load().orc_morton_cell(_p(p), _p(lo), scale, _p(q))
    return q


def crop(points, base, reach: float) -> np.ndarray:
    """Reach crop for a fixed-base arm (Sec. IV-C): indices, in input order,
    of the points whose float32 squared distance to the base,
    ((dx*dx + dy*dy) + dz*dz) with every operation rounded on its own, is at
    most fl(reach * reach).  Non-finite points fail the test."""
    pts = _f32(points, 3)
    b = np.asarray(base, dtype=np.float32).reshape(3)
    with np.errstate(invalid="ignore", over="ignore"):
        d = pts - b
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        keep = d2 <= np.float32(reach) * np.float32(reach)
    return np.nonzero(keep)[0].astype(np.int32)


def filter(points, r_filter: float, npass: int = 6, base=None, reach=None):  # noqa: A001
    """Filter (Alg. 2).  Returns (kept original indices in final order,
    counts after each pass).  With base and reach, the reach crop runs first
    and the filter sees only the cropped points, in input order."""
    if base is not None:
        keep = crop(points, base, reach)
        idx, counts = filter(_f32(points, 3)[keep], r_filter, npass)
        return keep[idx].astype(np.int32), counts
    pts = _f32(points, 3)
    out = np.zeros(max(len(pts), 1), dtype=np.int32)
    counts = np.zeros(npass, dtype=np.int64)
    k = _load().orc_filter(_p(pts), len(pts), np.float32(r_filter), npass, _p(out), _p(counts))
    return out[:k].copy(), counts
