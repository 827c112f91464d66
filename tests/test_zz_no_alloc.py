"""capt_collides_noalloc: the collision query that allocates nothing.

Its answers are checked against capt_collides (and the oracle's brute force)
on two calls in a row, the second with fewer spheres, for the slot kernel
(group 60) and the one-sphere kernel (group 1), on a forest of several clouds,
and with allocator hooks installed that count calls and fail every one.
"""
import ctypes as C
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def capt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_02807_amd as capt
    capt.load_library()
    return capt


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


class FailingAllocator:
    """Allocator hooks that count their calls and fail every allocation."""
    ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
    RELEASE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

    def __init__(self, lib):
        self.lib = lib
        self.calls = 0

        def alloc(nbytes, stream, ctx):
            self.calls += 1
            return None

        def release(ptr, stream, ctx):
            self.calls += 1

        self._a, self._r = self.ALLOC(alloc), self.RELEASE(release)

    def __enter__(self):
        assert self.lib.capt_set_allocator(C.cast(self._a, C.c_void_p), C.cast(self._r, C.c_void_p), None) == 0
        return self

    def __exit__(self, *exc):
        assert self.lib.capt_set_allocator(None, None, None) == 0


@pytest.mark.parametrize("group,n_big,n_small", [(60, 3000, 700), (1, 150_000, 20_001)])
def test_noalloc_matches_collides_on_two_calls(capt, orc, group, n_big, n_small):
    import torch
    pts = synth.tabletop_cloud(12_000, 901)
    f = capt.capt_build(dev(pts), 0.015, 0.08)
    tpl = synth.chain_template(2003)
    if group == 60:
        big = synth.posed_spheres(tpl, n_big, synth.WORKSPACE, 902)
        small = synth.posed_spheres(tpl, n_small, synth.WORKSPACE, 903)
    else:
        big = synth.uniform_spheres(n_big, synth.WORKSPACE, 0.015, 0.08, 902)
        small = synth.uniform_spheres(n_small, synth.WORKSPACE, 0.015, 0.08, 903)
    out = torch.full((len(big) // group,), 7, dtype=torch.uint8, device="cuda")
    lib = capt.load_library()
    for name, sph in (("big", big), ("small", small)):
        _say(f"case: noalloc group={group} {name} call, {len(sph)} spheres")
        s = dev(sph)
        k = len(sph) // group
        with FailingAllocator(lib) as hooks:
            capt.capt_collides_noalloc(f, s, group, out)
            torch.cuda.synchronize()
        assert hooks.calls == 0
        want = capt.capt_collides(f, s, group)
        assert torch.equal(out[:k], want)
        assert np.array_equal(out[:k].cpu().numpy(), orc.brute_f32(pts, sph, group))
    # the bytes past the small call's answers are the big call's, untouched
    assert torch.equal(out[len(small) // group:], capt.capt_collides(f, dev(big), group)[len(small) // group:])
    f.close()


def test_noalloc_forest_of_several_clouds(capt, orc):
    import torch
    clouds = [synth.tabletop_cloud(5000, 911), np.zeros((0, 3), np.float32), synth.tabletop_cloud(800, 912)]
    cloud_off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])])
    tpl = synth.chain_template(2003)
    for rep, ncfg in enumerate(((400, 30, 250), (90, 0, 17))):
        sph = [synth.posed_spheres(tpl, k, synth.WORKSPACE, 913 + 10 * rep + i) for i, k in enumerate(ncfg)]
        query_off = np.concatenate([[0], np.cumsum([len(s) for s in sph])])
        _say(f"case: noalloc forest of 3 clouds, call {rep}, configurations {ncfg}")
        f = capt.capt_build(dev(np.concatenate(clouds)), 0.015, 0.08, cloud_off=cloud_off)
        s = dev(np.concatenate(sph))
        out = torch.empty(int(query_off[-1]) // 60, dtype=torch.uint8, device="cuda")
        with FailingAllocator(capt.load_library()) as hooks:
            capt.capt_collides_noalloc(f, s, 60, out, query_off=query_off)
            torch.cuda.synchronize()
        assert hooks.calls == 0
        assert torch.equal(out, capt.capt_collides(f, s, 60, query_off=query_off))
        got = out.cpu().numpy()
        for c in range(3):
            want = orc.brute_f32(clouds[c], sph[c], 60)
            assert np.array_equal(got[query_off[c] // 60:query_off[c + 1] // 60], want), c
        f.close()


def test_noalloc_limits_and_flags(capt):
    import torch
    n = capt.CAPT_NOALLOC_MAX_CLOUDS + 1
    _say(f"case: noalloc refuses a forest of {n} clouds and nonzero flags")
    pts = synth.uniform_cube_cloud(n, 921)
    f = capt.capt_build(dev(pts), 0.0, 0.05, cloud_off=np.arange(n + 1))
    sph = dev(synth.uniform_spheres(n, [[0, 1]] * 3, 0.01, 0.05, 922))
    out = torch.empty(n, dtype=torch.uint8, device="cuda")
    with pytest.raises(capt.CaptError) as e:
        capt.capt_collides_noalloc(f, sph, 1, out, query_off=np.arange(n + 1))
    assert e.value.status == capt.CAPT_EUNSUPPORTED
    f.close()
    f = capt.capt_build(dev(pts), 0.0, 0.05)
    lib = capt.load_library()
    q = np.array([0, n], np.int64)
    st = lib.capt_collides_noalloc(f.handle, C.c_void_p(sph.data_ptr()), q.ctypes.data_as(C.c_void_p), 1,
                                   C.c_void_p(out.data_ptr()), capt.CAPT_CHECK_RADII, None)
    assert st == capt.CAPT_EINVAL
    f.close()
