"""MI355X collision-affording point trees (CAPTs).

Thin Python binding of the C ABI in ``include/capt.h`` (``libcapt.so``, built
in-tree by ``build_lib.py``).  Functions carry the C names and only marshal
arguments: torch tensors provide device memory, the current torch stream
provides ordering, and every step of filtering, building and querying runs in
the library's HIP kernels.  There is no CPU fallback: if the library is
missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import struct
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CAPT_LIBRARY names another build of the library to load (a sanitizer build of
# the host code, say); by default the in-tree libcapt.so.
LIB_PATH = os.environ.get("CAPT_LIBRARY") or os.path.join(_HERE, "libcapt.so")

CAPT_OK, CAPT_EINVAL, CAPT_ENOMEM, CAPT_EHIP, CAPT_ERADIUS, CAPT_EPRUNED, CAPT_EUNSUPPORTED = range(7)
CAPT_NO_PRUNE = 0x1
CAPT_CHECK_RADII = 0x2
CAPT_PER_CLOUD = 0x4
CAPT_NO_GRAPH = 0x8
CAPT_INDEXED_SETS = 0x10
CAPT_MAX_SHARD_BITS = 20
CAPT_NOALLOC_MAX_CLOUDS = 256

EXPORTS = [
    "capt_filter", "capt_filter_crop", "capt_build", "capt_build_axes", "capt_build_shard", "capt_build_filtered", "capt_collides",
    "capt_collides_noalloc", "capt_collides_visits",
    "capt_collides_padded", "capt_clearance", "capt_clearance_backward",
    "capt_destroy", "capt_destroy_async", "capt_last_error", "capt_forest_info", "capt_export", "capt_import",
    "capt_set_allocator", "capt_bruteforce_collides", "capt_query_stats", "capt_query_chunk_stats", "capt_set_tuning", "capt_collides_posed",
    "capt_get_tuning", "capt_probe_read", "capt_probe_gather",
]


class CaptError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"capt status {status}: {msg}")
        self.status = status


class capt_tuning(C.Structure):
    _fields_ = [("waves_per_group", C.c_int32), ("groups_per_cu", C.c_int32),
                ("tile_cfgs", C.c_int32), ("lds_levels", C.c_int32), ("scan_unroll", C.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libcapt.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_2406_02807_amd.build_lib` (no CPU fallback exists)")
    lib = C.CDLL(path)
    P, i64, i32, u32, f32 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint32, C.c_float
    sig = {
        "capt_filter": [P, i64, f32, P, P, P, P],
        "capt_build": [P, P, i32, f32, f32, u32, P, P],
        "capt_build_axes": [P, P, i32, f32, f32, u32, P, P, P],
        "capt_build_shard": [P, P, i32, f32, f32, u32, i32, i32, P, P],
        "capt_build_filtered": [P, i64, f32, P, f32, f32, u32, P, P, P, P],
        "capt_filter_crop": [P, i64, f32, P, P, P, P, P],
        "capt_collides_padded": [P, P, P, i32, f32, P, u32, P],
        "capt_collides": [P, P, P, i32, P, u32, P],
        "capt_collides_noalloc": [P, P, P, i32, P, u32, P],
        "capt_collides_visits": [P, P, P, i32, P, P, P],
        "capt_clearance": [P, P, P, P, P, P],
        "capt_clearance_backward": [P, P, P, P, P, P, P, P],
        "capt_forest_info": [P, i32, P, P, P, P, P],
        "capt_export": [P, i32, P, P],
        "capt_import": [P, C.c_size_t, P, P],
        "capt_set_allocator": [P, P, P],
        "capt_bruteforce_collides": [P, P, i32, P, P, i32, P, P],
        "capt_query_stats": [P, P, P, P, P, P, P, P],
        "capt_query_chunk_stats": [P, P, P, P, P, P],
        "capt_collides_posed": [P, P, i32, P, P, i32, P, u32, P],
        "capt_set_tuning": [P],
        "capt_get_tuning": [P],
        "capt_probe_read": [P, C.c_size_t, i32, i32, P, P],
        "capt_probe_gather": [P, i64, P, i64, P, P, P, i64, i32, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int32
    lib.capt_destroy.argtypes = [P]
    lib.capt_destroy.restype = None
    lib.capt_destroy_async.argtypes = [P, P]
    lib.capt_destroy_async.restype = None
    lib.capt_last_error.argtypes = []
    lib.capt_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(status: int):
    if status != CAPT_OK:
        raise CaptError(status, _lib.capt_last_error().decode())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype, cols=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
        raise ValueError(f"{name} must have shape [n, {cols}], got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


def _offsets(off, count):
    a = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    if a.shape != (count + 1,):
        raise ValueError(f"offsets must have {count + 1} entries")
    return a


# ---------------------------------------------------------------------------
# Forest handle
# ---------------------------------------------------------------------------
class Forest:
    """Owns a capt_forest; destroyed with the object."""

    def __init__(self, handle: int, ncloud: int, r_min: float, r_max: float, clouds=None):
        self._h = C.c_void_p(handle)
        self.ncloud = ncloud
        self.r_min = r_min
        self.r_max = r_max
        self._clouds = clouds     # keeps the build input alive for brute-force comparisons

    @property
    def handle(self):
        return self._h

    def info(self, cloud: int = 0) -> dict:
        lib = load_library()
        n, D, tot, pr, by = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib.capt_forest_info(self._h, cloud, C.byref(n), C.byref(D), C.byref(tot),
                                    C.byref(pr), C.byref(by)))
        return {"n": n.value, "D": D.value, "N": 1 << D.value, "set_total": tot.value,
                "pruned": pr.value, "bytes": by.value}

    def close(self):
        if self._h and self._h.value:
            load_library().capt_destroy(self._h)
            self._h = C.c_void_p(0)

    def release(self, stream=None):
        """Stream-ordered close: every use of the forest is already queued on
        `stream` (default: the current stream); the host does not wait."""
        if self._h and self._h.value:
            load_library().capt_destroy_async(self._h, _stream(stream))
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------
def _crop_arg(base, reach):
    if base is None:
        return None
    return (C.c_float * 4)(*[float(v) for v in base], float(reach))


def capt_filter(xyz, r_filter: float, base=None, reach=None, stream=None):
    """Alg. 2: returns (kept points [n', 3], original indices [n']).  With
    base (x, y, z) and reach, the reach crop runs first (capt_filter_crop)."""
    import torch
    lib = load_library()
    xyz = _dev(xyz, torch.float32, 3, "xyz")
    n = xyz.shape[0]
    out = torch.empty((max(n, 1), 3), dtype=torch.float32, device=xyz.device)
    idx = torch.empty((max(n, 1),), dtype=torch.int32, device=xyz.device)
    n_out = C.c_int64()
    crop = _crop_arg(base, reach)
    if crop is None:
        _check(lib.capt_filter(_ptr(xyz), n, float(r_filter), _ptr(out), _ptr(idx), C.byref(n_out),
                               _stream(stream)))
    else:
        _check(lib.capt_filter_crop(_ptr(xyz), n, float(r_filter), crop, _ptr(out), _ptr(idx),
                                    C.byref(n_out), _stream(stream)))
    k = n_out.value
    return out[:k], idx[:k]


def capt_build(xyz, r_min: float, r_max: float, prune: bool = True, cloud_off=None,
               stream=None, indexed: bool = False, axes=None, shard=None) -> Forest:
    """Alg. 1 for one cloud (xyz [n, 3]) or several (cloud_off host [ncloud+1]).
    indexed: the sets store point indices only (CAPT_INDEXED_SETS).
    axes: split axis of every depth (capt_build_axes), default d mod 3.
    shard: (shard_bits, s) builds shard s of 2^shard_bits (capt_build_shard)."""
    import torch
    lib = load_library()
    xyz = _dev(xyz, torch.float32, 3, "xyz")
    if cloud_off is None:
        cloud_off = [0, xyz.shape[0]]
    off = _offsets(cloud_off, len(cloud_off) - 1)
    if off[-1] != xyz.shape[0]:
        raise ValueError("cloud_off[-1] must equal the number of points")
    h = C.c_void_p()
    flags = (0 if prune else CAPT_NO_PRUNE) | (CAPT_INDEXED_SETS if indexed else 0)
    if shard is not None:
        if axes is not None:
            raise ValueError("shard and axes cannot be combined")
        bits, sid = shard
        _check(lib.capt_build_shard(_ptr(xyz), off.ctypes.data_as(C.c_void_p), len(off) - 1, float(r_min),
                                    float(r_max), flags, int(bits), int(sid), _stream(stream), C.byref(h)))
    elif axes is None:
        _check(lib.capt_build(_ptr(xyz), off.ctypes.data_as(C.c_void_p), len(off) - 1, float(r_min),
                              float(r_max), flags, _stream(stream), C.byref(h)))
    else:
        ax = np.zeros(32, np.uint8)
        a = np.asarray(axes, np.uint8)[:32]
        ax[:len(a)] = a
        _check(lib.capt_build_axes(_ptr(xyz), off.ctypes.data_as(C.c_void_p), len(off) - 1, float(r_min),
                                   float(r_max), flags, ax.ctypes.data_as(C.c_void_p), _stream(stream),
                                   C.byref(h)))
    return Forest(h.value, len(off) - 1, float(np.float32(r_min)), float(np.float32(r_max)),
                  clouds=(xyz, off))


def capt_build_filtered(xyz, r_filter: float, r_min: float, r_max: float, prune: bool = True,
                        kept_index: bool = False, base=None, reach=None, stream=None, indexed: bool = False):
    """Filter (Alg. 2) then build (Alg. 1) of one cloud in one library call.
    Returns the forest, or (forest, kept original indices [n']) with kept_index."""
    import torch
    lib = load_library()
    xyz = _dev(xyz, torch.float32, 3, "xyz")
    n = xyz.shape[0]
    idx = torch.empty((max(n, 1),), dtype=torch.int32, device=xyz.device) if kept_index else None
    h = C.c_void_p()
    m = C.c_int64()
    _check(lib.capt_build_filtered(_ptr(xyz), n, float(r_filter), _crop_arg(base, reach), float(r_min), float(r_max),
                                   (0 if prune else CAPT_NO_PRUNE) | (CAPT_INDEXED_SETS if indexed else 0),
                                   _ptr(idx),
                                   C.byref(m), _stream(stream), C.byref(h)))
    f = Forest(h.value, 1, float(np.float32(r_min)), float(np.float32(r_max)))
    return (f, idx[:m.value]) if kept_index else f


def capt_collides(forest: Forest, spheres, group: int = 1, query_off=None, flags: int = 0,
                  out=None, stream=None):
    """Alg. 3 with configuration-level early exit: uint8 [M / group]."""
    import torch
    lib = load_library()
    spheres = _dev(spheres, torch.float32, 4, "spheres")
    M = spheres.shape[0]
    if query_off is None:
        if forest.ncloud != 1:
            raise ValueError("query_off is required for a forest of several clouds")
        query_off = [0, M]
    off = _offsets(query_off, forest.ncloud)
    if out is None:
        out = torch.empty((M // group,), dtype=torch.uint8, device=spheres.device)
    _check(lib.capt_collides(forest.handle, _ptr(spheres), off.ctypes.data_as(C.c_void_p), group,
                             _ptr(out), flags, _stream(stream)))
    return out


def capt_collides_noalloc(forest: Forest, spheres, group: int, out, query_off=None, stream=None):
    """capt_collides without any device allocation inside the library: the
    caller passes `out` (uint8 [M / group]); the queue counters live in the
    library's own device array.  Returns `out`."""
    import torch
    lib = load_library()
    spheres = _dev(spheres, torch.float32, 4, "spheres")
    out = _dev(out, torch.uint8, None, "out")
    M = spheres.shape[0]
    if query_off is None:
        if forest.ncloud != 1:
            raise ValueError("query_off is required for a forest of several clouds")
        query_off = [0, M]
    off = _offsets(query_off, forest.ncloud)
    if out.numel() < M // group:
        raise ValueError(f"out holds {out.numel()} bytes, {M // group} needed")
    _check(lib.capt_collides_noalloc(forest.handle, _ptr(spheres), off.ctypes.data_as(C.c_void_p), group,
                                     _ptr(out), 0, _stream(stream)))
    return out


def capt_collides_visits(forest: Forest, spheres, group: int = 1, query_off=None, stream=None):
    """The batched kernel's answers and, per configuration, how many times it
    decided it (int32; 1 everywhere when every tile was taken exactly once).
    Returns (out uint8 [M / group], visits int32 [M / group])."""
    import torch
    lib = load_library()
    spheres = _dev(spheres, torch.float32, 4, "spheres")
    M = spheres.shape[0]
    if query_off is None:
        if forest.ncloud != 1:
            raise ValueError("query_off is required for a forest of several clouds")
        query_off = [0, M]
    off = _offsets(query_off, forest.ncloud)
    out = torch.empty((M // group,), dtype=torch.uint8, device=spheres.device)
    visits = torch.zeros((M // group,), dtype=torch.int32, device=spheres.device)
    _check(lib.capt_collides_visits(forest.handle, _ptr(spheres), off.ctypes.data_as(C.c_void_p), group,
                                    _ptr(out), _ptr(visits), _stream(stream)))
    return out, visits


def capt_collides_padded(forest: Forest, spheres, group: int, pad: float, query_off=None, flags: int = 0,
                         out=None, stream=None):
    """capt_collides with every radius r replaced by r + pad (query padding)."""
    import torch
    lib = load_library()
    spheres = _dev(spheres, torch.float32, 4, "spheres")
    M = spheres.shape[0]
    if query_off is None:
        if forest.ncloud != 1:
            raise ValueError("query_off is required for a forest of several clouds")
        query_off = [0, M]
    off = _offsets(query_off, forest.ncloud)
    if out is None:
        out = torch.empty((M // group,), dtype=torch.uint8, device=spheres.device)
    _check(lib.capt_collides_padded(forest.handle, _ptr(spheres), off.ctypes.data_as(C.c_void_p), group,
                                    float(pad), _ptr(out), flags, _stream(stream)))
    return out


def capt_collides_posed(forest: Forest, template, poses, edge: int = 1, pose_off=None, flags: int = 0,
                        out=None, stream=None):
    """CollisionCheck on posed template spheres, grouped into edges of `edge`
    configurations: uint8 [P / edge].  template [g, 4]; poses [P, 12]
    (row-major rotation, then translation)."""
    import torch
    lib = load_library()
    template = _dev(template, torch.float32, 4, "template")
    poses = _dev(poses, torch.float32, 12, "poses")
    P = poses.shape[0]
    if pose_off is None:
        if forest.ncloud != 1:
            raise ValueError("pose_off is required for a forest of several clouds")
        pose_off = [0, P]
    off = _offsets(pose_off, forest.ncloud)
    if out is None:
        out = torch.empty((P // edge,), dtype=torch.uint8, device=poses.device)
    _check(lib.capt_collides_posed(forest.handle, _ptr(template), template.shape[0], _ptr(poses),
                                   off.ctypes.data_as(C.c_void_p), edge, _ptr(out), flags, _stream(stream)))
    return out


def capt_clearance(forest: Forest, spheres, query_off=None, stream=None):
    """Clearance and witness (no autograd; see `clearance` for the autograd form)."""
    import torch
    lib = load_library()
    spheres = _dev(spheres, torch.float32, 4, "spheres")
    M = spheres.shape[0]
    off = _offsets([0, M] if query_off is None else query_off, forest.ncloud)
    clr = torch.empty((M,), dtype=torch.float32, device=spheres.device)
    wit = torch.empty((M,), dtype=torch.int32, device=spheres.device)
    _check(lib.capt_clearance(forest.handle, _ptr(spheres), off.ctypes.data_as(C.c_void_p),
                              _ptr(clr), _ptr(wit), _stream(stream)))
    return clr, wit


def capt_clearance_backward(forest: Forest, spheres, witness, grad_clearance, query_off=None,
                            radius: bool = True, stream=None):
    """Returns (grad_center [M, 3], grad_radius [M] or None when radius is False)."""
    import torch
    lib = load_library()
    spheres = _dev(spheres, torch.float32, 4, "spheres")
    witness = _dev(witness, torch.int32, None, "witness")
    grad_clearance = _dev(grad_clearance.contiguous(), torch.float32, None, "grad_clearance")
    M = spheres.shape[0]
    off = _offsets([0, M] if query_off is None else query_off, forest.ncloud)
    gc = torch.empty((M, 3), dtype=torch.float32, device=spheres.device)
    gr = torch.empty((M,), dtype=torch.float32, device=spheres.device) if radius else None
    _check(lib.capt_clearance_backward(forest.handle, _ptr(spheres), off.ctypes.data_as(C.c_void_p),
                                       _ptr(witness), _ptr(grad_clearance), _ptr(gc), _ptr(gr),
                                       _stream(stream)))
    return gc, gr


def capt_bruteforce_collides(xyz, spheres, group: int = 1, cloud_off=None, query_off=None,
                             stream=None):
    import torch
    lib = load_library()
    xyz = _dev(xyz, torch.float32, 3, "xyz")
    spheres = _dev(spheres, torch.float32, 4, "spheres")
    coff = _offsets([0, xyz.shape[0]] if cloud_off is None else cloud_off,
                    1 if cloud_off is None else len(cloud_off) - 1)
    ncl = len(coff) - 1
    qoff = _offsets([0, spheres.shape[0]] if query_off is None else query_off, ncl)
    out = torch.empty((spheres.shape[0] // group,), dtype=torch.uint8, device=spheres.device)
    _check(lib.capt_bruteforce_collides(_ptr(xyz), coff.ctypes.data_as(C.c_void_p), ncl,
                                        _ptr(spheres), qoff.ctypes.data_as(C.c_void_p), group,
                                        _ptr(out), _stream(stream)))
    return out


def capt_query_stats(forest: Forest, spheres, query_off=None, stream=None):
    """Per sphere: (leaf int32, aabb_rejected uint8, scanned int32, hit uint8)."""
    import torch
    lib = load_library()
    spheres = _dev(spheres, torch.float32, 4, "spheres")
    M = spheres.shape[0]
    off = _offsets([0, M] if query_off is None else query_off, forest.ncloud)
    leaf = torch.empty((M,), dtype=torch.int32, device=spheres.device)
    rej = torch.empty((M,), dtype=torch.uint8, device=spheres.device)
    sc = torch.empty((M,), dtype=torch.int32, device=spheres.device)
    hit = torch.empty((M,), dtype=torch.uint8, device=spheres.device)
    _check(lib.capt_query_stats(forest.handle, _ptr(spheres), off.ctypes.data_as(C.c_void_p),
                                _ptr(leaf), _ptr(rej), _ptr(sc), _ptr(hit), _stream(stream)))
    return leaf, rej, sc, hit


def capt_query_chunk_stats(forest: Forest, spheres, query_off=None, stream=None):
    """Per sphere: (chunk boxes tested int32, chunks scanned int32) of the
    two-level set scan, in stored order up to the chunk of the first hit."""
    import torch
    lib = load_library()
    spheres = _dev(spheres, torch.float32, 4, "spheres")
    M = spheres.shape[0]
    off = _offsets([0, M] if query_off is None else query_off, forest.ncloud)
    boxes = torch.empty((M,), dtype=torch.int32, device=spheres.device)
    chunks = torch.empty((M,), dtype=torch.int32, device=spheres.device)
    _check(lib.capt_query_chunk_stats(forest.handle, _ptr(spheres), off.ctypes.data_as(C.c_void_p),
                                      _ptr(boxes), _ptr(chunks), _stream(stream)))
    return boxes, chunks


def capt_probe_read(buf, passes: int = 1, blocks_per_cu: int = 2, stream=None):
    """Stream-read a device tensor `passes` times (bandwidth yardstick)."""
    import torch
    lib = load_library()
    if not isinstance(buf, torch.Tensor) or not buf.is_cuda or not buf.is_contiguous():
        raise TypeError("buf must be a contiguous CUDA tensor")
    sink = torch.zeros(1, dtype=torch.float32, device=buf.device)
    _check(lib.capt_probe_read(_ptr(buf), buf.numel() * buf.element_size(), passes, blocks_per_cu, _ptr(sink),
                               _stream(stream)))
    return sink


def capt_probe_gather(items, leaves, x, y, z, lanes_per_item: int = 16, out=None, stream=None):
    """The query's gather pattern without its arithmetic (bandwidth yardstick):
    items int32 [m, 4] (leaf, len, -, -), leaves int32 [nleaf, 8] records
    (float lo[3], hi[3] as bits, uint32 start, count), x, y, z float32 [entries]."""
    import torch
    lib = load_library()
    items = _dev(items, torch.int32, 4, "items")
    leaves = _dev(leaves, torch.int32, 8, "leaves")
    for name, t in (("x", x), ("y", y), ("z", z)):
        _dev(t, torch.float32, None, name)
    if not (x.numel() == y.numel() == z.numel()):
        raise ValueError("x, y and z must have the same length")
    m = items.shape[0]
    if out is None:
        out = torch.empty(m, dtype=torch.uint8, device=items.device)
    _check(lib.capt_probe_gather(_ptr(items), m, _ptr(leaves), leaves.shape[0], _ptr(x), _ptr(y), _ptr(z),
                                 x.numel(), lanes_per_item, _ptr(out), _stream(stream)))
    return out


def capt_set_tuning(waves_per_group=0, groups_per_cu=0, tile_cfgs=0, lds_levels=0, scan_unroll=0):
    t = capt_tuning(waves_per_group, groups_per_cu, tile_cfgs, lds_levels, scan_unroll)
    lib = load_library()
    _check(lib.capt_set_tuning(C.byref(t)))


def capt_get_tuning() -> dict:
    t = capt_tuning()
    lib = load_library()
    _check(lib.capt_get_tuning(C.byref(t)))
    return {k: getattr(t, k) for k, _ in capt_tuning._fields_}


def capt_export(forest: Forest, cloud: int = 0) -> bytes:
    lib = load_library()
    n = C.c_size_t()
    _check(lib.capt_export(forest.handle, cloud, None, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _check(lib.capt_export(forest.handle, cloud, buf, C.byref(n)))
    return buf.raw


def capt_import(blob: bytes, stream=None) -> Forest:
    lib = load_library()
    h = C.c_void_p()
    b = C.create_string_buffer(blob, len(blob))
    _check(lib.capt_import(b, len(blob), _stream(stream), C.byref(h)))
    hdr = parse_blob(blob)
    return Forest(h.value, 1, hdr.r_min, hdr.r_max)


# ---------------------------------------------------------------------------
# Blob format (documented in include/capt.h)
# ---------------------------------------------------------------------------
_HDR = struct.Struct("<IIqqiIffq")
BLOB_MAGIC = 0x54504143


def _a8(x):
    return (x + 7) & ~7


@dataclass
class Blob:
    n: int
    N: int
    D: int
    flags: int
    r_min: float
    r_max: float
    points: np.ndarray   # float32 [n, 3]
    T: np.ndarray        # float32 [N-1]
    rep: np.ndarray      # int32 [N]
    aabb: np.ndarray     # float32 [N, 6]
    pruned: np.ndarray   # uint8 [N]
    off: np.ndarray      # int64 [N+1]
    idx: np.ndarray      # int32 [S]
    axes: np.ndarray = None   # uint8 [D] split axis per depth (None: d mod 3)

    def set_of(self, leaf):
        return self.idx[self.off[leaf]:self.off[leaf + 1]]


def _layout(n, N, S, version=1):
    o = _a8(_HDR.size + (8 if version >= 2 else 0))   # version 2: the axis code follows the header
    lay = {}
    for name, size in (("pts", 12 * n), ("T", 4 * (N - 1)), ("rep", 4 * N), ("aabb", 24 * N),
                       ("pruned", N), ("off", 8 * (N + 1)), ("idx", 4 * S)):
        lay[name] = o
        o = _a8(o + size)
    lay["total"] = o
    return lay


def parse_blob(blob: bytes) -> Blob:
    magic, ver, n, N, D, flags, r_min, r_max, S = _HDR.unpack_from(blob, 0)
    if magic != BLOB_MAGIC or ver not in (1, 2):
        raise ValueError("not a CAPT blob")
    L = _layout(n, N, S, ver)
    axes = None
    if ver >= 2:
        code = struct.unpack_from("<Q", blob, _HDR.size)[0]
        axes = np.array([(code >> (2 * d)) & 3 for d in range(D)], np.uint8)
    f = np.frombuffer
    return Blob(n, N, D, flags, r_min, r_max,
                f(blob, np.float32, 3 * n, L["pts"]).reshape(n, 3).copy(),
                f(blob, np.float32, N - 1, L["T"]).copy(),
                f(blob, np.int32, N, L["rep"]).copy(),
                f(blob, np.float32, 6 * N, L["aabb"]).reshape(N, 6).copy(),
                f(blob, np.uint8, N, L["pruned"]).copy(),
                f(blob, np.int64, N + 1, L["off"]).copy(),
                f(blob, np.int32, S, L["idx"]).copy(), axes)


def make_blob(points, T, rep, aabb, pruned, off, idx, r_min, r_max, flags=0, axes=None) -> bytes:
    """Pack tree arrays (for example a tree built elsewhere) into the blob
    format that capt_import reads; `axes` (split axis per depth) gives a
    version-2 blob."""
    points = np.ascontiguousarray(points, np.float32).reshape(-1, 3)
    n = len(points)
    N = len(rep)
    D = N.bit_length() - 1
    idx = np.ascontiguousarray(idx, np.int32)
    S = len(idx)
    ver = 1 if axes is None else 2
    L = _layout(n, N, S, ver)
    buf = bytearray(L["total"])
    _HDR.pack_into(buf, 0, BLOB_MAGIC, ver, n, N, D, flags, float(r_min), float(r_max), S)
    if axes is not None:
        code = 0
        for d in range(D):
            code |= int(axes[d]) << (2 * d)
        struct.pack_into("<Q", buf, _HDR.size, code)
    for name, arr in (("pts", points), ("T", np.asarray(T, np.float32)), ("rep", np.asarray(rep, np.int32)),
                      ("aabb", np.asarray(aabb, np.float32)), ("pruned", np.asarray(pruned, np.uint8)),
                      ("off", np.asarray(off, np.int64)), ("idx", idx)):
        b = np.ascontiguousarray(arr).tobytes()
        buf[L[name]:L[name] + len(b)] = b
    return bytes(buf)


# ---------------------------------------------------------------------------
# Autograd form of the clearance query
# ---------------------------------------------------------------------------
def _clearance_fn():
    import torch

    class Clearance(torch.autograd.Function):
        """clr = min(d, r_max) - r per sphere; backward by capt_clearance_backward."""

        @staticmethod
        def forward(ctx, spheres, forest, query_off):
            clr, wit = capt_clearance(forest, spheres, query_off)
            ctx.save_for_backward(spheres, wit)
            ctx.forest = forest
            ctx.query_off = query_off
            ctx.mark_non_differentiable(wit)
            return clr, wit

        @staticmethod
        def backward(ctx, grad_clr, grad_wit):
            spheres, wit = ctx.saved_tensors
            gc, gr = capt_clearance_backward(ctx.forest, spheres, wit, grad_clr, ctx.query_off)
            # the two kernel outputs side by side in the layout of `spheres`
            return torch.cat([gc, gr[:, None]], 1), None, None

    return Clearance


_Clearance = None


def clearance(forest: Forest, spheres, query_off=None):
    """Differentiable clearance: returns (clearance [M], witness [M]); gradients
    flow to `spheres` ([M, 4]: centre and radius)."""
    global _Clearance
    if _Clearance is None:
        _Clearance = _clearance_fn()
    return _Clearance.apply(spheres, forest, query_off)
