// Differentiable clearance against CAPTs: forward (nearest affordance-set
// point, clamped at r_max) and its hand-written backward.
//
// Forward mapping: a wavefront takes 64 spheres (one per lane), descends the
// tree and applies the AABB shortcut (if even the leaf box is at least r_max
// away, the clamp is active and no point needs reading).  The remaining
// spheres are then processed one after another by the whole wave: the 64
// lanes stream the sphere's set in coalesced 64-entry steps keeping a running
// minimum of one 64-bit key per entry (squared distance above index), and one
// branch-free wave minimum of the keys per sphere yields the argmin (ties ->
// smallest original index).  Sets here are full scans, so lanes across the
// set keep loads contiguous and every lane busy.
//
// Backward: thread per sphere; reads the witness point from the cloud copy
// kept in the forest: 16 (sphere) + 4 (witness) + 4 (incoming gradient) + 12
// (witness point) read, 12 (d/dx, d/dy, d/dz) + 4 (d/dr, optional) written.
#include <climits>
#include <cmath>

#include "capt_internal.h"

namespace capt {

namespace {

__device__ __forceinline__ uint32_t descend_c(const float4 &q, const float *Tl, int L,
                                              const float *__restrict__ Tg, int D, uint64_t axes) {
    uint32_t i = 0;
    for (int lv = 0; lv < D; ++lv) {
        const float t = lv < L ? Tl[i] : Tg[i];
        const int a = axis_at(axes, lv);
        const float x = a == 0 ? q.x : (a == 1 ? q.y : q.z);
        i = 2 * i + 1 + (x > t ? 1u : 0u);
    }
    return i;
}

// The nearest point as one 64-bit key: the bits of the float32 squared
// distance (never negative, so its bit pattern orders like its value) above
// the point's original index, so the minimum key is the nearest point with
// ties to the smallest index.  A NaN distance orders above every key that
// can win, as a NaN never compares below a distance.
constexpr uint64_t KEY_NONE = ((uint64_t)0x7f800000u << 32) | 0x7fffffffu;   // (+inf, INT_MAX)

__device__ __forceinline__ uint64_t key_min(uint64_t a, uint64_t b) { return b < a ? b : a; }

// Minimum over one DPP-permuted copy of v: ctrl picks the source lane inside
// each row of 16.
template <int CTRL> __device__ __forceinline__ uint64_t dpp_min(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, 0xf, 0xf, false);
    return key_min(v, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t lane_key(uint64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Minimum key over the wave (every lane active): swaps of neighbours and of
// pairs inside each quad, then the mirror images inside each half row and
// each row leave every lane of a row with the row's minimum; the four rows
// are then combined from one lane each.
__device__ __forceinline__ uint64_t wave_min_key(uint64_t v) {
    v = dpp_min<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v = dpp_min<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v = dpp_min<0x141>(v);   // row_half_mirror
    v = dpp_min<0x140>(v);   // row_mirror
    return key_min(key_min(lane_key(v, 0), lane_key(v, 16)), key_min(lane_key(v, 32), lane_key(v, 48)));
}

__global__ void k_clearance(CloudDev C, const float4 *__restrict__ sph, int64_t nsph, float r_max,
                            float *__restrict__ clr, int32_t *__restrict__ wit, int L) {
    extern __shared__ float Tl[];
    const int nT = (1 << L) - 1;
    for (int i = threadIdx.x; i < nT; i += blockDim.x) Tl[i] = C.T[i];
    __syncthreads();
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int64_t ntiles = (nsph + WAVE - 1) / WAVE;
    const int64_t N = (int64_t)1 << C.D;
    for (int64_t t = wid; t < ntiles; t += waves) {
        const int64_t s = t * WAVE + lane;
        const bool valid = s < nsph;
        const float4 q = valid ? sph[s] : make_float4(0.f, 0.f, 0.f, 0.f);
        const uint32_t lf = descend_c(q, Tl, L, C.T, C.D, C.axes) - (uint32_t)(N - 1);
        uint32_t start = 0, count = 0;
        bool need = false;
        if (valid) {
            const Leaf leaf = C.leaf[lf];
            start = leaf.start;
            count = leaf.count;
            if (count > 0) {
                const float b2 = box_sqdist(q.x, q.y, q.z, leaf.lo, leaf.hi);
                need = !(sqrtf(b2) >= r_max);
            }
        }
        uint64_t best = KEY_NONE;   // the key of this lane's sphere
        uint64_t todo = __ballot(need);
        while (todo) {
            const int o = __builtin_ctzll(todo);
            todo &= todo - 1;
            const float ox = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.x), o));
            const float oy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.y), o));
            const float oz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.z), o));
            const uint32_t st = (uint32_t)__builtin_amdgcn_readlane((int)start, o);
            const uint32_t ct = (uint32_t)__builtin_amdgcn_readlane((int)count, o);
            uint64_t m = KEY_NONE;
            for (uint32_t k = lane; k < ct; k += WAVE) {
                const uint32_t e = st + k;
                float x, y, z;
                set_point(C, e, x, y, z);
                const float d2 = sqdist(ox, oy, oz, x, y, z);
                const uint64_t key = ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)C.pidx[e];
                m = key < m ? key : m;
            }
            m = wave_min_key(m);
            if (lane == o) best = m;
        }
        if (valid) {
            const float d = need ? sqrtf(__uint_as_float((uint32_t)(best >> 32))) : INFINITY;
            if (d < r_max) {
                clr[s] = __fsub_rn(d, q.w);
                wit[s] = (int32_t)(uint32_t)best;
            } else {
                clr[s] = __fsub_rn(r_max, q.w);
                wit[s] = -1;
            }
        }
    }
}

__global__ void k_clearance_bwd(const float *__restrict__ pts, const float4 *__restrict__ sph,
                                int64_t nsph, const int32_t *__restrict__ wit,
                                const float *__restrict__ grad, float *__restrict__ gc,
                                float *__restrict__ gr) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsph) return;
    const float g = grad[s];
    const int32_t w = wit[s];
    float rx = 0.f, ry = 0.f, rz = 0.f;
    if (w >= 0) {
        const float4 q = sph[s];
        const float dx = __fsub_rn(q.x, pts[3 * (int64_t)w]);
        const float dy = __fsub_rn(q.y, pts[3 * (int64_t)w + 1]);
        const float dz = __fsub_rn(q.z, pts[3 * (int64_t)w + 2]);
        const float d = sqrtf(__fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz)));
        if (d > 0.0f) {
            const float k = g / d;
            rx = k * dx;
            ry = k * dy;
            rz = k * dz;
        }
    }
    gc[3 * s] = rx;
    gc[3 * s + 1] = ry;
    gc[3 * s + 2] = rz;
    if (gr) gr[s] = -g;
}

// Launch shape: four 512-thread blocks per CU fill its 32 wave slots, which
// hides the set gathers far better than more tree levels in LDS at fewer
// blocks (the 12 levels take 16 KB per block; 14 levels, 64 KB, would allow
// only two blocks).
constexpr int CLR_LDS_LEVELS = 12;
constexpr int CLR_BLOCKS_PER_CU = 4;

int lds_levels_c(int D) {
    int L = std::min(D, CLR_LDS_LEVELS);
    const size_t cap = (size_t)device_info().lds_per_block;
    while (L > 0 && sizeof(float) * (size_t)((1 << L) - 1) > cap) --L;
    return L;
}

}  // namespace

capt_status clearance_fwd(capt_forest_s *f, const float *spheres, const int64_t *qoff, float *clr,
                          int32_t *witness, hipStream_t s) {
    const int nc = (int)f->clouds.size();
    for (int c = 0; c < nc; ++c) {
        const int64_t m = qoff[c + 1] - qoff[c];
        if (m <= 0) continue;
        const CloudDev &C = f->clouds[c].dev;
        const int L = lds_levels_c(C.D);
        const int threads = 512;
        const int64_t ntiles = (m + WAVE - 1) / WAVE;
        int64_t blocks = std::min<int64_t>((ntiles + 7) / 8, (int64_t)device_info().cus * CLR_BLOCKS_PER_CU);
        blocks = std::max<int64_t>(blocks, 1);
        const size_t lds = sizeof(float) * (size_t)((1 << L) - 1);
        hipLaunchKernelGGL(k_clearance, dim3((unsigned)blocks), dim3(threads), lds, s, C,
                           reinterpret_cast<const float4 *>(spheres + 4 * qoff[c]), m, f->r_max, clr + qoff[c],
                           witness + qoff[c], L);
        CAPT_LAUNCH_CHECK();
    }
    return CAPT_OK;
}

capt_status clearance_bwd(capt_forest_s *f, const float *spheres, const int64_t *qoff, const int32_t *witness,
                          const float *grad, float *grad_center, float *grad_radius, hipStream_t s) {
    const int nc = (int)f->clouds.size();
    for (int c = 0; c < nc; ++c) {
        const int64_t m = qoff[c + 1] - qoff[c];
        if (m <= 0) continue;
        hipLaunchKernelGGL(k_clearance_bwd, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                           f->clouds[c].dev.pts, reinterpret_cast<const float4 *>(spheres + 4 * qoff[c]), m,
                           witness + qoff[c], grad + qoff[c], grad_center + 3 * qoff[c],
                           grad_radius ? grad_radius + qoff[c] : nullptr);
        CAPT_LAUNCH_CHECK();
    }
    return CAPT_OK;
}

}  // namespace capt
