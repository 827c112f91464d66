// Achievable-bandwidth yardsticks for the memory roofline of the queries (not
// on the hot path; the benchmark divides the query's algorithmic bytes by
// what these kernels reach on the same chip).
//
//  k_probe_read    every lane streams float4s through one XCD's part of a
//                  buffer, `passes` times: HBM bandwidth when the buffer is
//                  far larger than the caches, L2 or MALL bandwidth when it
//                  fits in them (a part is only read by blocks on its XCD, so
//                  re-reads hit that XCD's L2).
//  k_probe_gather  the collision query's memory pattern without its
//                  arithmetic: per item a 16-byte descriptor (the size of a
//                  sphere), the 32-byte leaf record it names, then `len`
//                  consecutive entries of three float32 arrays from the
//                  record's start (a set scan over structure-of-arrays sets),
//                  and one output byte.  A group of 16 or 64 lanes serves one
//                  item, 16 or 64 consecutive entries per step.
#include <algorithm>

#include "capt_internal.h"

namespace capt {

namespace {

// The buffer is split into one part per XCD (blocks go to the XCDs round
// robin, so block b works on part b % 8); a thread walks (pass, float4) pairs
// of its part with a fixed stride, eight loads in flight.
__global__ void __launch_bounds__(256) k_probe_read(const float4 *__restrict__ p, int64_t n4, int passes,
                                                    float *__restrict__ sink) {
    constexpr int NX = 8, U = 8;
    const int nx = (int)min<int64_t>(NX, (int64_t)gridDim.x);
    const int part = (int)(blockIdx.x % (unsigned)nx);
    const int64_t pb = blockIdx.x / nx;
    const int64_t nb = ((int64_t)gridDim.x - part + nx - 1) / nx;   // blocks on this part
    const int64_t p0 = n4 * part / nx, p1 = n4 * (part + 1) / nx;
    const int64_t len = p1 - p0;
    if (len <= 0) return;
    const int64_t stride = nb * blockDim.x;
    const int64_t total = len * passes;
    int64_t done = pb * blockDim.x + threadIdx.x;
    int64_t q = done % len;
    const int64_t step = stride % len;
    float acc = 0.0f;
    for (; done < total; done += U * stride) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            v[u] = done + u * stride < total ? p[p0 + q] : make_float4(0.f, 0.f, 0.f, 0.f);
            q += step;
            q = q >= len ? q - len : q;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u].x + v[u].w;
    }
    // the buffer's contents decide whether anything is stored, so no load is dead
    if (acc == -1.0f) sink[0] = acc;
}

template <int LPI>
__global__ void __launch_bounds__(256) k_probe_gather(const int4 *__restrict__ items, int64_t m,
                                                      const Leaf *__restrict__ leaf, int64_t nleaf,
                                                      const float *__restrict__ x, const float *__restrict__ y,
                                                      const float *__restrict__ z, int64_t entries,
                                                      uint8_t *__restrict__ out) {
    constexpr int GPW = WAVE / LPI;   // items per wavefront step
    const int lane = (int)(threadIdx.x % WAVE);
    const int sub = lane % LPI, grp = lane / LPI;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / WAVE;
    for (int64_t base = wave * GPW; base < m; base += nwaves * GPW) {
        const int64_t k = base + grp;
        float acc = 0.0f;
        if (k < m) {
            const int4 it = items[k];
            if (it.x >= 0 && (int64_t)it.x < nleaf) {
                const Leaf L = leaf[it.x];
                acc = L.lo[0] + L.hi[2];
                const int64_t st = (int64_t)L.start;
                int64_t len = min((int64_t)max(it.y, 0), (int64_t)L.count);
                len = st >= entries ? 0 : min(len, entries - st);   // never past the arrays
#pragma unroll 2
                for (int64_t j = sub; j < len; j += LPI) acc += (x[st + j] + y[st + j]) + z[st + j];
            }
        }
        const uint64_t b = __ballot(acc == -1.0f);
        const uint64_t mask = LPI == WAVE ? ~0ull : ((1ull << LPI) - 1) << (grp * LPI);
        if (k < m && sub == 0) out[k] = (uint8_t)((b & mask) != 0);
    }
}

}  // namespace

capt_status probe_read(const void *buf, size_t bytes, int32_t passes, int32_t blocks_per_cu, float *sink,
                       hipStream_t s) {
    const int64_t n4 = (int64_t)(bytes / 16);
    if (n4 == 0 || passes <= 0) return CAPT_OK;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n4 + 255) / 256, (int64_t)device_info().cus * blocks_per_cu));
    hipLaunchKernelGGL(k_probe_read, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const float4 *>(buf), n4,
                       passes, sink);
    CAPT_LAUNCH_CHECK();
    return CAPT_OK;
}

capt_status probe_gather(const int32_t *items, int64_t m, const void *leaves, int64_t nleaf, const float *x,
                         const float *y, const float *z, int64_t entries, int32_t lanes_per_item, uint8_t *out,
                         hipStream_t s) {
    if (m <= 0) return CAPT_OK;
    const int per_block = 256 / lanes_per_item;   // items per block step
    const int64_t blocks =
        std::max<int64_t>(1, std::min<int64_t>((m + per_block - 1) / per_block, (int64_t)device_info().cus * 8));
    const int4 *it = reinterpret_cast<const int4 *>(items);
    const Leaf *lf = static_cast<const Leaf *>(leaves);
    if (lanes_per_item == 16)
        hipLaunchKernelGGL(k_probe_gather<16>, dim3((unsigned)blocks), dim3(256), 0, s, it, m, lf, nleaf, x, y, z,
                           entries, out);
    else
        hipLaunchKernelGGL(k_probe_gather<64>, dim3((unsigned)blocks), dim3(256), 0, s, it, m, lf, nleaf, x, y, z,
                           entries, out);
    CAPT_LAUNCH_CHECK();
    return CAPT_OK;
}

}  // namespace capt
