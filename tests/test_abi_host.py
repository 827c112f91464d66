"""Host-side checks of the C ABI that need no GPU: the library loads, every
symbol declared in include/capt.h is exported, and argument validation
rejects bad calls with CAPT_EINVAL before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    import paper_2406_02807_amd as capt
    if not os.path.exists(capt.LIB_PATH):
        from paper_2406_02807_amd import build_lib
        build_lib.build()
    return capt.load_library()


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "capt.h")).read()
    return sorted(set(re.findall(r"^\s*(?:capt_status|void|const char \*)\s*(capt_\w+)\s*\(", src, re.M)))


def test_header_declares_the_five_hot_path_calls():
    names = declared_symbols()
    for n in ["capt_filter", "capt_build", "capt_collides", "capt_clearance", "capt_clearance_backward"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    import paper_2406_02807_amd as capt
    names = declared_symbols()
    assert sorted(names) == sorted(capt.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_no_gpu_needed_for_validation(lib):
    import paper_2406_02807_amd as capt
    P = C.c_void_p
    h = C.c_void_p()
    off = np.array([0, 10], np.int64)
    offp = off.ctypes.data_as(P)
    # NULL output handle
    assert lib.capt_build(P(1), offp, 1, 0.01, 0.05, 0, None, None) == capt.CAPT_EINVAL
    # r_min > r_max, negative radius, NaN radius
    assert lib.capt_build(P(1), offp, 1, 0.06, 0.05, 0, None, C.byref(h)) == capt.CAPT_EINVAL
    assert lib.capt_build(P(1), offp, 1, -0.01, 0.05, 0, None, C.byref(h)) == capt.CAPT_EINVAL
    assert lib.capt_build(P(1), offp, 1, 0.0, float("nan"), 0, None, C.byref(h)) == capt.CAPT_EINVAL
    assert b"r_min" in lib.capt_last_error()
    # non-monotone offsets, bad first offset, zero clouds, NULL points
    bad = np.array([0, 5, 3], np.int64)
    assert lib.capt_build(P(1), bad.ctypes.data_as(P), 2, 0.0, 0.05, 0, None, C.byref(h)) == capt.CAPT_EINVAL
    bad0 = np.array([1, 5], np.int64)
    assert lib.capt_build(P(1), bad0.ctypes.data_as(P), 1, 0.0, 0.05, 0, None, C.byref(h)) == capt.CAPT_EINVAL
    assert lib.capt_build(P(1), offp, 0, 0.0, 0.05, 0, None, C.byref(h)) == capt.CAPT_EINVAL
    assert lib.capt_build(None, offp, 1, 0.0, 0.05, 0, None, C.byref(h)) == capt.CAPT_EINVAL
    # unknown flag
    assert lib.capt_build(P(1), offp, 1, 0.0, 0.05, 0x80, None, C.byref(h)) == capt.CAPT_EINVAL
    assert h.value is None
    # queries on a NULL forest
    q = np.array([0, 60], np.int64)
    assert lib.capt_collides(None, P(1), q.ctypes.data_as(P), 60, P(1), 0, None) == capt.CAPT_EINVAL
    assert lib.capt_collides_noalloc(None, P(1), q.ctypes.data_as(P), 60, P(1), 0, None) == capt.CAPT_EINVAL
    assert lib.capt_collides_visits(None, P(1), q.ctypes.data_as(P), 60, P(1), P(1), None) == capt.CAPT_EINVAL
    assert lib.capt_clearance(None, P(1), q.ctypes.data_as(P), P(1), P(1), None) == capt.CAPT_EINVAL
    # posed queries: bad template size, NULL template, bad edge
    assert lib.capt_collides_posed(None, P(1), 0, P(1), q.ctypes.data_as(P), 1, P(1), 0, None) == capt.CAPT_EINVAL
    assert lib.capt_collides_posed(None, None, 60, P(1), q.ctypes.data_as(P), 1, P(1), 0, None) == capt.CAPT_EINVAL
    assert lib.capt_collides_posed(None, P(1), 60, P(1), q.ctypes.data_as(P), 0, P(1), 0, None) == capt.CAPT_EINVAL
    assert lib.capt_collides_posed(None, P(1), 60, P(1), q.ctypes.data_as(P), 1 << 20, P(1), 0, None) == capt.CAPT_EINVAL
    # filter: negative / NaN radius, NULL count
    n_out = C.c_int64()
    assert lib.capt_filter(P(1), 10, -1.0, P(1), None, C.byref(n_out), None) == capt.CAPT_EINVAL
    assert lib.capt_filter(P(1), 10, float("nan"), P(1), None, C.byref(n_out), None) == capt.CAPT_EINVAL
    assert lib.capt_filter(P(1), 10, 0.01, P(1), None, None, None) == capt.CAPT_EINVAL
    assert lib.capt_filter(P(1), 1 << 30, 0.01, P(1), None, C.byref(n_out), None) == capt.CAPT_EUNSUPPORTED
    # filter + build: NULL out, bad filter radius, bad build radii, unknown flags, bad crop
    m = C.c_int64()
    crop = (C.c_float * 4)(0.0, 0.0, 0.0, 1.0)
    bad_crop = (C.c_float * 4)(0.0, float("nan"), 0.0, 1.0)
    neg_reach = (C.c_float * 4)(0.0, 0.0, 0.0, -1.0)
    bf = lib.capt_build_filtered
    assert bf(P(1), 10, 0.01, None, 0.01, 0.05, 0, None, C.byref(m), None, None) == capt.CAPT_EINVAL
    assert bf(P(1), 10, -0.01, None, 0.01, 0.05, 0, None, C.byref(m), None, C.byref(h)) == capt.CAPT_EINVAL
    assert bf(P(1), 10, 0.01, None, 0.05, 0.01, 0, None, C.byref(m), None, C.byref(h)) == capt.CAPT_EINVAL
    assert bf(P(1), 10, 0.01, None, 0.01, 0.05, 0x80, None, C.byref(m), None, C.byref(h)) == capt.CAPT_EINVAL
    assert bf(None, 10, 0.01, None, 0.01, 0.05, 0, None, C.byref(m), None, C.byref(h)) == capt.CAPT_EINVAL
    assert bf(P(1), 10, 0.01, bad_crop, 0.01, 0.05, 0, None, C.byref(m), None, C.byref(h)) == capt.CAPT_EINVAL
    # split axes: NULL, not an axis
    ax = (C.c_uint8 * 32)(*([0] * 32))
    assert lib.capt_build_axes(P(1), offp, 1, 0.0, 0.05, 0, None, None, C.byref(h)) == capt.CAPT_EINVAL
    ax[3] = 3
    assert lib.capt_build_axes(P(1), offp, 1, 0.0, 0.05, 0, ax, None, C.byref(h)) == capt.CAPT_EINVAL
    # shards: bits or shard out of range, then the radii checks of capt_build
    bs = lib.capt_build_shard
    assert bs(P(1), offp, 1, 0.0, 0.05, 0, -1, 0, None, C.byref(h)) == capt.CAPT_EINVAL
    assert bs(P(1), offp, 1, 0.0, 0.05, 0, capt.CAPT_MAX_SHARD_BITS + 1, 0, None, C.byref(h)) == capt.CAPT_EINVAL
    assert bs(P(1), offp, 1, 0.0, 0.05, 0, 3, 8, None, C.byref(h)) == capt.CAPT_EINVAL
    assert bs(P(1), offp, 1, 0.0, 0.05, 0, 3, -1, None, C.byref(h)) == capt.CAPT_EINVAL
    assert bs(P(1), offp, 1, 0.06, 0.05, 0, 3, 7, None, C.byref(h)) == capt.CAPT_EINVAL
    assert bs(P(1), offp, 1, 0.0, 0.05, 0, 3, 7, None, None) == capt.CAPT_EINVAL
    assert h.value is None
    # cropped filter: NULL / non-finite base / negative reach / NULL count
    fc = lib.capt_filter_crop
    assert fc(P(1), 10, 0.01, None, P(1), None, C.byref(m), None) == capt.CAPT_EINVAL
    assert fc(P(1), 10, 0.01, bad_crop, P(1), None, C.byref(m), None) == capt.CAPT_EINVAL
    assert fc(P(1), 10, 0.01, neg_reach, P(1), None, C.byref(m), None) == capt.CAPT_EINVAL
    assert fc(P(1), 10, 0.01, crop, P(1), None, None, None) == capt.CAPT_EINVAL
    assert fc(P(1), 1 << 30, 0.01, crop, P(1), None, C.byref(m), None) == capt.CAPT_EUNSUPPORTED
    # padded queries: NULL forest, bad pad, unknown flags
    cp = lib.capt_collides_padded
    assert cp(None, P(1), q.ctypes.data_as(P), 1, 0.01, P(1), 0, None) == capt.CAPT_EINVAL
    # brute force: group not dividing the range
    q7 = np.array([0, 7], np.int64)
    assert lib.capt_bruteforce_collides(P(1), offp, 1, P(1), q7.ctypes.data_as(P), 2, P(1), None) == capt.CAPT_EINVAL
    # import: garbage blob
    junk = C.create_string_buffer(b"\x00" * 64, 64)
    assert lib.capt_import(junk, 64, None, C.byref(h)) == capt.CAPT_EINVAL
    # tuning ranges
    t = capt.capt_tuning(17, 0, 0, 0, 0)
    assert lib.capt_set_tuning(C.byref(t)) == capt.CAPT_EINVAL
    t = capt.capt_tuning(0, 0, 0, 0, 3)
    assert lib.capt_set_tuning(C.byref(t)) == capt.CAPT_EINVAL
    # allocator: both or neither
    assert lib.capt_set_allocator(P(1), None, None) == capt.CAPT_EINVAL
    assert lib.capt_set_allocator(None, None, None) == capt.CAPT_OK


def test_blob_roundtrip_pack_parse():
    import paper_2406_02807_amd as capt
    rng = np.random.default_rng(0)
    pts = rng.random((5, 3)).astype(np.float32)
    N = 8
    T = rng.random(N - 1).astype(np.float32)
    rep = np.arange(N, dtype=np.int32)
    aabb = rng.random((N, 6)).astype(np.float32)
    pr = np.zeros(N, np.uint8)
    off = np.array([0, 1, 2, 3, 4, 5, 5, 5, 5], np.int64)
    idx = np.arange(5, dtype=np.int32)
    b = capt.make_blob(pts, T, rep, aabb, pr, off, idx, 0.01, 0.05)
    p = capt.parse_blob(b)
    assert (p.n, p.N, p.D) == (5, 8, 3)
    assert np.array_equal(p.points, pts) and np.array_equal(p.T, T) and np.array_equal(p.idx, idx)
    assert np.array_equal(p.aabb, aabb) and np.array_equal(p.off, off)
    assert p.axes is None
    # version 2 carries the split axis of every depth
    b2 = capt.make_blob(pts, T, rep, aabb, pr, off, idx, 0.01, 0.05, axes=[2, 0, 1])
    p2 = capt.parse_blob(b2)
    assert p2.axes.tolist() == [2, 0, 1]
    assert np.array_equal(p2.points, pts) and np.array_equal(p2.T, T) and np.array_equal(p2.idx, idx)
    assert len(b2) == len(b) + 8


def test_product_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2406_02807_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "capt_oracle" not in txt, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c", ".h")):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2406_02807_amd" not in txt and "capt_internal" not in txt, f


def test_import_rejects_bad_offsets_before_reading_sets(lib):
    """A blob whose set offsets run past the idx section (or wrap) is refused
    on the host, before any set entry is read."""
    import paper_2406_02807_amd as capt
    rng = np.random.default_rng(1)
    pts = rng.random((5, 3)).astype(np.float32)
    N = 8
    T = np.sort(rng.random(N - 1)).astype(np.float32)
    rep = np.arange(N, dtype=np.int32)
    aabb = np.tile(np.array([np.inf] * 3 + [-np.inf] * 3, np.float32), (N, 1))
    pr = np.zeros(N, np.uint8)
    idx = np.zeros(0, np.int32)
    h = C.c_void_p()
    for off in ([0, 1_000_000_000, 0, 0, 0, 0, 0, 0, 0],        # far past S, then back
                [0, 0, 0, 0, 0, 0, 0, 2 ** 40, 0],                # huge, would wrap an index
                [0, 0, 0, 0, 0, 0, 0, 0, 1]):                     # ends past S = 0
        b = capt.make_blob(pts, T, rep, aabb, pr, np.array(off, np.int64), idx, 0.01, 0.05)
        buf = C.create_string_buffer(b, len(b))
        assert lib.capt_import(buf, len(b), None, C.byref(h)) == capt.CAPT_EINVAL
        assert b"offset" in lib.capt_last_error()
        assert h.value is None
    # a set_total of 2^30 or more is refused from the header alone
    b = bytearray(capt.make_blob(pts, T, rep, aabb, pr, np.zeros(N + 1, np.int64), idx, 0.01, 0.05))
    b[40:48] = (1 << 31).to_bytes(8, "little")
    buf = C.create_string_buffer(bytes(b), len(b))
    assert lib.capt_import(buf, len(b), None, C.byref(h)) == capt.CAPT_EINVAL
    assert b"header" in lib.capt_last_error()


def test_clearance_backward_validation(lib):
    import paper_2406_02807_amd as capt
    P = C.c_void_p
    q = np.array([0, 4], np.int64)
    assert lib.capt_clearance_backward(None, P(1), q.ctypes.data_as(P), P(1), P(1), P(1), None,
                                       None) == capt.CAPT_EINVAL
