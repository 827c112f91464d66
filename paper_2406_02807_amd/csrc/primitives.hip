// Device-wide exclusive scan and stable LSD radix sort for wave64 (CDNA4).
//
// Both work on tiles of 2048 elements per 256-thread workgroup (8 per
// thread).  The scan is reduce -> scan of tile sums -> rescan-and-add.  The
// sort makes one pass per 8-bit digit: per-tile digit histogram -> scan of the
// digit-major histogram table -> stable scatter, where the rank of an element
// among equal digits inside a tile comes from wave ballots (eight ballots
// match the digit across the 64 lanes) and per-wave digit counts in LDS.
#include "capt_internal.h"

namespace capt {

namespace {

constexpr int TB = 256;            // threads per block
constexpr int IPT = 8;             // items per thread
constexpr int TILE = TB * IPT;     // 2048
constexpr int NW = TB / WAVE;      // waves per block

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint32_t t = __shfl_up(v, d, WAVE);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan across the 256 threads of a block; *total gets the block sum.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *lds_w, uint32_t *total) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    uint32_t inc = wave_incl_scan(v);
    if (lane == WAVE - 1) lds_w[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        uint32_t t = lds_w[i];
        off += (i < w) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__device__ __forceinline__ int64_t eff_n(int64_t n, const int64_t *n_dev) {
    if (n_dev) {
        int64_t m = *n_dev;
        return m < n ? m : n;
    }
    return n;
}

__global__ void k_scan_reduce(const uint32_t *__restrict__ in, int64_t n, const int64_t *n_dev,
                              uint32_t *__restrict__ sums) {
    __shared__ uint32_t lw[NW];
    const int64_t m = eff_n(n, n_dev);
    const int64_t base = (int64_t)blockIdx.x * TILE + (int64_t)threadIdx.x * IPT;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        int64_t j = base + i;
        s += (j < m) ? in[j] : 0u;
    }
    uint32_t tot;
    block_excl_scan(s, lw, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of nb tile sums, in place; total to *total.
__global__ void k_scan_sums(uint32_t *__restrict__ sums, int64_t nb, uint32_t *total) {
    __shared__ uint32_t lw[NW];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c = 0; c < nb; c += TILE) {
        const int64_t base = c + (int64_t)threadIdx.x * IPT;
        uint32_t v[IPT];
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            int64_t j = base + i;
            v[i] = (j < nb) ? sums[j] : 0u;
            s += v[i];
        }
        uint32_t tot;
        uint32_t off = block_excl_scan(s, lw, &tot) + carry;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            int64_t j = base + i;
            if (j < nb) sums[j] = off;
            off += v[i];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void k_scan_apply(const uint32_t *in, uint32_t *out, int64_t n, const int64_t *n_dev,
                             const uint32_t *__restrict__ sums) {
    __shared__ uint32_t lw[NW];
    const int64_t m = eff_n(n, n_dev);
    const int64_t base = (int64_t)blockIdx.x * TILE + (int64_t)threadIdx.x * IPT;
    uint32_t v[IPT];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        int64_t j = base + i;
        v[i] = (j < m) ? in[j] : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(s, lw, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        int64_t j = base + i;
        if (j < m) out[j] = off;
        off += v[i];
    }
}

// ---------------------------------------------------------------------------
// Radix sort
// ---------------------------------------------------------------------------
template <class K>
__global__ void k_radix_hist(const K *__restrict__ keys, int64_t n, int shift,
                             uint32_t *__restrict__ hist, int64_t nb) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * TILE;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        int64_t j = base + (int64_t)i * TB + threadIdx.x;
        if (j < n) {
            uint32_t d = (uint32_t)(keys[j] >> shift) & 255u;
            atomicAdd(&h[d], 1u);
        }
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

template <class K>
__global__ void k_radix_scatter(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                                K *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n,
                                int shift, const uint32_t *__restrict__ offs, int64_t nb) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t cnt[NW][256];
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    run[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * TILE;
    for (int r = 0; r < IPT; ++r) {
#pragma unroll
        for (int q = 0; q < NW; ++q) cnt[q][threadIdx.x] = 0;
        __syncthreads();
        const int64_t j = base + (int64_t)r * TB + threadIdx.x;
        const bool valid = j < n;
        K key = valid ? kin[j] : K(0);
        uint32_t val = valid ? vin[j] : 0u;
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        // lanes of this wave holding the same digit
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot(valid && ((d >> b) & 1u));
            same &= ((d >> b) & 1u) ? bal : ~bal;
        }
        uint32_t rank = __popcll(same & lt_mask);
        if (valid && rank == 0) cnt[w][d] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d];
            for (int q = 0; q < w; ++q) pos += cnt[q][d];
            pos += rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) add += cnt[q][threadIdx.x];
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

template <class K>
capt_status radix_sort(K *k0, uint32_t *v0, K *k1, uint32_t *v1, int64_t n, int bits,
                       uint32_t *tmp, hipStream_t s, int *where) {
    *where = 0;
    if (n <= 1 || bits <= 0) return CAPT_OK;
    const int64_t nb = (n + TILE - 1) / TILE;
    uint32_t *hist = tmp;                         // 256 * nb
    uint32_t *stmp = tmp + 256 * nb;              // scan scratch
    K *ki = k0, *ko = k1;
    uint32_t *vi = v0, *vo = v1;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist<K>, dim3((unsigned)nb), dim3(TB), 0, s, ki, n, shift, hist, nb);
        CAPT_LAUNCH_CHECK();
        capt_status st = scan_exclusive_u32(hist, hist, 256 * nb, nullptr, nullptr, stmp, s);
        if (st) return st;
        hipLaunchKernelGGL(k_radix_scatter<K>, dim3((unsigned)nb), dim3(TB), 0, s, ki, vi, ko, vo, n,
                           shift, hist, nb);
        CAPT_LAUNCH_CHECK();
        K *tk = ki; ki = ko; ko = tk;
        uint32_t *tv = vi; vi = vo; vo = tv;
        *where ^= 1;
    }
    return CAPT_OK;
}

}  // namespace

size_t scan_tmp_words(int64_t n) {
    int64_t nb = (n + TILE - 1) / TILE;
    return (size_t)(nb + 16);
}

capt_status scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, const int64_t *n_dev,
                               uint32_t *total, uint32_t *tmp, hipStream_t s) {
    if (n <= 0) {
        return CAPT_OK;
    }
    const int64_t nb = (n + TILE - 1) / TILE;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(TB), 0, s, in, n, n_dev, tmp);
    CAPT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(TB), 0, s, tmp, nb, total);
    CAPT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(TB), 0, s, in, out, n, n_dev, tmp);
    CAPT_LAUNCH_CHECK();
    return CAPT_OK;
}

size_t radix_tmp_words(int64_t n) {
    int64_t nb = (n + TILE - 1) / TILE;
    return (size_t)(256 * nb) + scan_tmp_words(256 * nb);
}

capt_status radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n,
                           int bits, uint32_t *tmp, hipStream_t s, int *where) {
    return radix_sort<uint64_t>(k0, v0, k1, v1, n, bits, tmp, s, where);
}

capt_status radix_sort_u32(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n,
                           int bits, uint32_t *tmp, hipStream_t s, int *where) {
    return radix_sort<uint32_t>(k0, v0, k1, v1, n, bits, tmp, s, where);
}

}  // namespace capt
