// Morton-curve point-cloud filter (Alg. 2, Sec. IV-C) on the GPU.
//
// Per axis permutation (six passes, each on the previous pass's survivors):
//  1. 63-bit Z-order keys on a 2^21-per-axis grid over the input's cubic
//     bounding box, then a stable 64-bit radix sort (ties keep the current
//     order, as a stable sort of the list would);
//  2. the sequential rule "keep j iff it is farther than r_filter from the
//     last kept point" is made parallel: next[j] = first k > j farther than
//     r_filter from j, so the kept points are exactly the chain
//     0 -> next[0] -> next[next[0]] -> ...  The chain is marked with pointer
//     doubling: jump tables J_t = next^(2^t), then, for t from high to low,
//     every node marked at a level above t marks J_t of itself;
//  3. a scan of the marks compacts the survivors in curve order.
// Only the final count crosses to the host.
#include <cmath>

#include "capt_internal.h"

namespace capt {

namespace {

constexpr int TB = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + TB - 1) / TB); }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct FState {
    float lo[3];
    float hi[3];
    double scale;
    int64_t m;          // current number of points
    unsigned int bad;   // non-finite coordinates
};

__global__ void k_fstate_init(FState *st, int64_t n) {
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) {
            st->lo[a] = INFINITY;
            st->hi[a] = -INFINITY;
        }
        st->m = n;
        st->bad = 0;
        st->scale = 0.0;
    }
}

__device__ __forceinline__ void atomic_min_f(float *a, float v) {
    // order-preserving integer view of a float (no NaN here)
    int iv = __float_as_int(v);
    if (iv >= 0) atomicMin(reinterpret_cast<int *>(a), iv);
    else atomicMax(reinterpret_cast<unsigned int *>(a), (unsigned int)iv);
}

__device__ __forceinline__ void atomic_max_f(float *a, float v) {
    int iv = __float_as_int(v);
    if (iv >= 0) atomicMax(reinterpret_cast<int *>(a), iv);
    else atomicMin(reinterpret_cast<unsigned int *>(a), (unsigned int)iv);
}

__global__ void k_bbox(const float *__restrict__ xyz, int64_t n, FState *st) {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    unsigned int bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        for (int a = 0; a < 3; ++a) {
            float v = xyz[3 * j + a];
            if (!isfinite(v)) {
                ++bad;
                continue;
            }
            lo[a] = fminf(lo[a], v);
            hi[a] = fmaxf(hi[a], v);
        }
    }
    for (int a = 0; a < 3; ++a) {
        for (int off = WAVE / 2; off >= 1; off >>= 1) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], off, WAVE));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off, WAVE));
        }
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        for (int a = 0; a < 3; ++a) {
            // the sign of a zero minimum does not change any cell coordinate
            atomic_min_f(&st->lo[a], lo[a]);
            atomic_max_f(&st->hi[a], hi[a]);
        }
    }
    if (bad) atomicAdd(&st->bad, bad);
}

__global__ void k_grid(FState *st) {
    if (threadIdx.x != 0) return;
    double E = 0.0;
    for (int a = 0; a < 3; ++a) {
        double e = __dsub_rn((double)st->hi[a], (double)st->lo[a]);
        if (e > E) E = e;
    }
    st->scale = E > 0.0 ? 2097152.0 / E : 0.0;
}

__global__ void k_iota(uint32_t *__restrict__ v, int64_t n) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) v[j] = (uint32_t)j;
}

// Spread the low 21 bits of v to every third bit (bit b -> bit 3b).
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1FFFFFull;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint32_t cell_of(float v, float lo, double scale) {
    double t = floor(__dmul_rn(__dsub_rn((double)v, (double)lo), scale));
    if (t < 0.0) t = 0.0;
    if (t > 2097151.0) t = 2097151.0;
    return (uint32_t)t;
}

// Axis order of each permutation: xyz, xzy, yxz, yzx, zxy, zyx.
__constant__ int c_perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

__global__ void k_morton(const float *__restrict__ xyz, const uint32_t *__restrict__ cur, int64_t n,
                         const FState *__restrict__ st, int p, uint64_t *__restrict__ keys,
                         uint32_t *__restrict__ vals) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t m = st->m;
    if (j >= m) {
        keys[j] = ~0ull;
        vals[j] = 0xFFFFFFFFu;
        return;
    }
    const uint32_t id = cur[j];
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) q[a] = cell_of(xyz[3 * (int64_t)id + a], st->lo[a], st->scale);
    // axis X[j] fills key bits 3b + (2 - j)
    keys[j] = (spread3(q[c_perm[p][0]]) << 2) | (spread3(q[c_perm[p][1]]) << 1) | spread3(q[c_perm[p][2]]);
    vals[j] = id;
}

__global__ void k_next(const float *__restrict__ xyz, const uint32_t *__restrict__ ord, int64_t n,
                       const FState *__restrict__ st, float rf2, uint32_t *__restrict__ next) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t m = st->m;
    if (j > m || j >= n + 1) return;
    if (j == m) {
        next[j] = (uint32_t)m;
        return;
    }
    const uint32_t a = ord[j];
    const float ax = xyz[3 * (int64_t)a], ay = xyz[3 * (int64_t)a + 1], az = xyz[3 * (int64_t)a + 2];
    int64_t k = j + 1;
    for (; k < m; ++k) {
        const uint32_t b = ord[k];
        if (sqdist(ax, ay, az, xyz[3 * (int64_t)b], xyz[3 * (int64_t)b + 1], xyz[3 * (int64_t)b + 2]) > rf2) break;
    }
    next[j] = (uint32_t)k;
}

__global__ void k_jump(const uint32_t *__restrict__ Jp, uint32_t *__restrict__ Jn, int64_t n,
                       const FState *__restrict__ st) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > st->m || j >= n + 1) return;
    Jn[j] = Jp[Jp[j]];
}

__global__ void k_mark_init(int8_t *__restrict__ mark, int64_t n, int top) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n + 1) mark[j] = (int8_t)(j == 0 ? top : -1);
}

__global__ void k_mark_step(const uint32_t *__restrict__ J, int8_t *__restrict__ mark, int64_t n,
                            const FState *__restrict__ st, int t) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t m = st->m;
    if (j >= m || j >= n) return;
    if (mark[j] > t) {
        const uint32_t k = J[j];
        if ((int64_t)k < m) mark[k] = (int8_t)t;
    }
}

__global__ void k_keep_flags(const int8_t *__restrict__ mark, int64_t n, const FState *__restrict__ st,
                             uint32_t *__restrict__ flags) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    flags[j] = (j < st->m && mark[j] >= 0) ? 1u : 0u;
}

__global__ void k_compact(const uint32_t *__restrict__ ord, const uint32_t *__restrict__ flags,
                          const uint32_t *__restrict__ pos, int64_t n, const FState *__restrict__ st,
                          uint32_t *__restrict__ cur) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n || j >= st->m) return;
    if (flags[j]) cur[pos[j]] = ord[j];
}

__global__ void k_set_count(FState *st, const uint32_t *total) {
    if (threadIdx.x == 0) st->m = (int64_t)*total;
}

__global__ void k_output(const float *__restrict__ xyz, const uint32_t *__restrict__ cur, int64_t n,
                         const FState *__restrict__ st, float *__restrict__ out_xyz,
                         int32_t *__restrict__ out_index) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n || j >= st->m) return;
    const uint32_t id = cur[j];
    out_xyz[3 * j] = xyz[3 * (int64_t)id];
    out_xyz[3 * j + 1] = xyz[3 * (int64_t)id + 1];
    out_xyz[3 * j + 2] = xyz[3 * (int64_t)id + 2];
    if (out_index) out_index[j] = (int32_t)id;
}

}  // namespace

capt_status filter(const float *xyz, int64_t n, float r_filter, float *out_xyz, int32_t *out_index,
                   int64_t *n_out, hipStream_t s) {
    if (n == 0) {
        *n_out = 0;
        return CAPT_OK;
    }
    int levels = 1;
    while (((int64_t)1 << levels) < n + 1) ++levels;
    levels += 1;   // J_0 .. J_{levels-1} reach past the chain's end
    const size_t wn = (size_t)n + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t oSt = take(sizeof(FState));
    const size_t oCur = take(sizeof(uint32_t) * wn);
    const size_t oK0 = take(sizeof(uint64_t) * wn);
    const size_t oK1 = take(sizeof(uint64_t) * wn);
    const size_t oV0 = take(sizeof(uint32_t) * wn);
    const size_t oV1 = take(sizeof(uint32_t) * wn);
    const size_t oJ = take(sizeof(uint32_t) * wn * (size_t)levels);
    const size_t oMark = take(wn);
    const size_t oFlag = take(sizeof(uint32_t) * wn);
    const size_t oPos = take(sizeof(uint32_t) * wn);
    const size_t oTot = take(sizeof(uint32_t) * 4);
    const size_t oRad = take(sizeof(uint32_t) * radix_tmp_words((int64_t)wn));
    const size_t oScan = take(sizeof(uint32_t) * scan_tmp_words((int64_t)wn));
    Scratch sc;
    if (!sc.alloc(off, s)) {
        set_error("device allocation of %zu filter scratch bytes failed", off);
        return CAPT_ENOMEM;
    }
    char *B = sc.as<char>();
    FState *st = reinterpret_cast<FState *>(B + oSt);
    uint32_t *cur = reinterpret_cast<uint32_t *>(B + oCur);
    uint64_t *k0 = reinterpret_cast<uint64_t *>(B + oK0);
    uint64_t *k1 = reinterpret_cast<uint64_t *>(B + oK1);
    uint32_t *v0 = reinterpret_cast<uint32_t *>(B + oV0);
    uint32_t *v1 = reinterpret_cast<uint32_t *>(B + oV1);
    uint32_t *J = reinterpret_cast<uint32_t *>(B + oJ);
    int8_t *mark = reinterpret_cast<int8_t *>(B + oMark);
    uint32_t *flags = reinterpret_cast<uint32_t *>(B + oFlag);
    uint32_t *pos = reinterpret_cast<uint32_t *>(B + oPos);
    uint32_t *tot = reinterpret_cast<uint32_t *>(B + oTot);
    uint32_t *rad = reinterpret_cast<uint32_t *>(B + oRad);
    uint32_t *stmp = reinterpret_cast<uint32_t *>(B + oScan);

    const float rf2 = r_filter * r_filter;
    CAPT_HIP(hipMemsetAsync(rad, 0, sizeof(uint32_t) * 64, s));
    hipLaunchKernelGGL(k_fstate_init, dim3(1), dim3(64), 0, s, st, n);
    CAPT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bbox, dim3(std::min<unsigned>(nblk(n), 1024u)), dim3(TB), 0, s, xyz, n, st);
    CAPT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_grid, dim3(1), dim3(64), 0, s, st);
    CAPT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_iota, dim3(nblk(n)), dim3(TB), 0, s, cur, n);
    CAPT_LAUNCH_CHECK();
    for (int p = 0; p < 6; ++p) {
        hipLaunchKernelGGL(k_morton, dim3(nblk(n)), dim3(TB), 0, s, xyz, cur, n, st, p, k0, v0);
        CAPT_LAUNCH_CHECK();
        int where = 0;
        capt_status e = radix_sort_u64(k0, v0, k1, v1, n, 64, rad, s, &where);
        if (e) return e;
        const uint32_t *ord = where ? v1 : v0;
        hipLaunchKernelGGL(k_next, dim3(nblk(n + 1)), dim3(TB), 0, s, xyz, ord, n, st, rf2, J);
        CAPT_LAUNCH_CHECK();
        for (int t = 1; t < levels; ++t) {
            hipLaunchKernelGGL(k_jump, dim3(nblk(n + 1)), dim3(TB), 0, s, J + (size_t)(t - 1) * wn,
                               J + (size_t)t * wn, n, st);
            CAPT_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_mark_init, dim3(nblk(n + 1)), dim3(TB), 0, s, mark, n, levels);
        CAPT_LAUNCH_CHECK();
        for (int t = levels - 1; t >= 0; --t) {
            hipLaunchKernelGGL(k_mark_step, dim3(nblk(n)), dim3(TB), 0, s, J + (size_t)t * wn, mark, n, st, t);
            CAPT_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_keep_flags, dim3(nblk(n)), dim3(TB), 0, s, mark, n, st, flags);
        CAPT_LAUNCH_CHECK();
        capt_status e2 = scan_exclusive_u32(flags, pos, n, nullptr, tot, stmp, s);
        if (e2) return e2;
        hipLaunchKernelGGL(k_compact, dim3(nblk(n)), dim3(TB), 0, s, ord, flags, pos, n, st, cur);
        CAPT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_set_count, dim3(1), dim3(64), 0, s, st, tot);
        CAPT_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_output, dim3(nblk(n)), dim3(TB), 0, s, xyz, cur, n, st, out_xyz, out_index);
    CAPT_LAUNCH_CHECK();
    FState h;
    uint32_t sort_err = 0;
    CAPT_HIP(hipMemcpyAsync(&h, st, sizeof(FState), hipMemcpyDeviceToHost, s));
    CAPT_HIP(hipMemcpyAsync(&sort_err, rad, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    CAPT_HIP(hipStreamSynchronize(s));
    if (sort_err) {
        set_error("internal: radix sort look-back bound exceeded in the filter");
        return CAPT_EHIP;
    }
    if (h.bad) {
        set_error("input holds %u non-finite coordinates", h.bad);
        return CAPT_EINVAL;
    }
    *n_out = h.m;
    return CAPT_OK;
}

}  // namespace capt
