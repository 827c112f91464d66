// Device-wide exclusive scan and stable LSD radix sort for wave64 (CDNA4).
//
// Both work on tiles of 2048 elements per 256-thread workgroup (8 per
// thread).  The scan is reduce -> scan of tile sums -> rescan-and-add.  The
// sort counts all digits once, then makes one kernel per 8-bit digit with
// decoupled look-back for the tile offsets; the rank of an element among
// equal digits inside a tile comes from wave ballots (eight ballots match the
// digit across the 64 lanes) and per-wave running offsets in LDS.
#include "capt_internal.h"
#include "lookback.h"

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
// Radix sort (one sweep per digit)
// ---------------------------------------------------------------------------
// k_os_hist counts every digit of every pass in one read of the keys (LSD
// digit counts do not depend on the order).  Each pass is then ONE kernel:
// a workgroup takes the next tile id from a counter (so ids follow launch
// order), counts its tile's digits, publishes them, and obtains the count of
// each digit in all earlier tiles by looking back over their published words
// (decoupled look-back); the tile's ranks are then stable within the tile.
// Published word: bits 30-31 = 1 (tile count) or 2 (inclusive prefix), bits
// 0-29 = value.  A tile only waits for tiles with smaller ids, which started
// before it, so the waits end; they are also bounded (see LOOKBACK_SPINS).
constexpr uint32_t ST_AGG = 1u << 30;
constexpr uint32_t ST_PRE = 2u << 30;
constexpr uint32_t ST_VAL = (1u << 30) - 1u;
constexpr uint32_t LOOKBACK_SPINS = 1u << 20;

__device__ __forceinline__ uint32_t load_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// One-pass exclusive scan: tiles take ids from a counter (status[ntiles]) and
// find their offset by decoupled look-back over the earlier tiles' published
// sums (bits 30-31 = aggregate / inclusive prefix, bits 0-29 = value, so the
// total stays below 2^30).  status must hold ntiles + 1 zeroed words.
__global__ void __launch_bounds__(TB) k_scan_lb(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                int64_t n, uint32_t *__restrict__ status, int64_t ntiles,
                                                uint32_t *__restrict__ err) {
    __shared__ uint32_t lw[NW];
    __shared__ uint32_t s_tile, s_excl;
    if (threadIdx.x == 0) s_tile = atomicAdd(&status[ntiles], 1u);
    __syncthreads();
    const int64_t t = s_tile;
    const int64_t base = t * TILE + (int64_t)threadIdx.x * IPT;
    uint32_t v[IPT];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int64_t j = base + i;
        v[i] = j < n ? in[j] : 0u;
        sum += v[i];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(sum, lw, &tot);
    if (threadIdx.x < WAVE) {   // the first wavefront publishes and looks back
        uint32_t ex = 0;
        if (t == 0) {
            if (threadIdx.x == 0) store_agent(&status[0], ST_PRE | tot);
        } else {
            if (threadIdx.x == 0) store_agent(&status[t], ST_AGG | tot);
            ex = wave_lookback(status, t, LOOKBACK_SPINS, err, 16u);
            if (threadIdx.x == 0) store_agent(&status[t], ST_PRE | (ex + tot));
        }
        if (threadIdx.x == 0) s_excl = ex;
    }
    __syncthreads();
    off += s_excl;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int64_t j = base + i;
        if (j < n) out[j] = off;
        off += v[i];
    }
}


// Segments: the keys form `nseg` independent lists of `len` items each
// (segment g at g * len); every segment is sorted on its own.
// Histograms of every digit of every pass.  ATOMIC: blocks add theirs to
// ghist[pass][seg][256] (few blocks, small inputs); otherwise every block
// writes its own to part[block][seg][pass][256] and k_os_hist_sum adds them.
template <class K, bool ATOMIC>
__global__ void k_os_hist(const K *__restrict__ keys, int64_t len, int nseg, int npass, uint32_t *__restrict__ part) {
    extern __shared__ uint32_t h[];   // [nseg][npass][256]
    const int nh = nseg * npass * 256;
    for (int i = threadIdx.x; i < nh; i += TB) h[i] = 0;
    __syncthreads();
    const int64_t n = len * nseg;
    const int64_t stride = (int64_t)gridDim.x * TB;
    for (int64_t j = (int64_t)blockIdx.x * TB + threadIdx.x; j < n; j += stride) {
        const K k = keys[j];
        uint32_t *hs = h + (size_t)(j / len) * npass * 256;
        for (int p = 0; p < npass; ++p) atomicAdd(&hs[p * 256 + ((uint32_t)(k >> (8 * p)) & 255u)], 1u);
    }
    __syncthreads();
    if (ATOMIC) {
        for (int i = threadIdx.x; i < nh; i += TB) {
            const int g = i / (npass * 256), r = i % (npass * 256);
            const int p = r / 256, d = r % 256;
            if (h[i]) atomicAdd(&part[((size_t)p * nseg + g) * 256 + d], h[i]);
        }
        return;
    }
    uint32_t *out = part + (size_t)blockIdx.x * nh;
    for (int i = threadIdx.x; i < nh; i += TB) out[i] = h[i];
}

// ghist[pass][seg][256] = sum over blocks of part[block][seg][pass][256].
// A block takes HS_BINS bins; its TB / HS_BINS thread groups each add a
// strided share of the partials, then the shares are added in LDS.
constexpr int HS_BINS = 32;
__global__ void __launch_bounds__(TB) k_os_hist_sum(const uint32_t *__restrict__ part, int nblocks, int nseg,
                                                    int npass, uint32_t *__restrict__ ghist) {
    constexpr int NG = TB / HS_BINS;
    __shared__ uint32_t acc[NG][HS_BINS];
    const int nh = nseg * npass * 256;
    const int bl = threadIdx.x % HS_BINS, grp = threadIdx.x / HS_BINS;
    const int i = blockIdx.x * HS_BINS + bl;
    uint32_t t = 0;
    if (i < nh)
        for (int b = grp; b < nblocks; b += NG) t += part[(size_t)b * nh + i];
    acc[grp][bl] = t;
    __syncthreads();
    if (grp != 0 || i >= nh) return;
    for (int q = 1; q < NG; ++q) t += acc[q][bl];
    const int g = i / (npass * 256), r = i % (npass * 256);
    const int p = r / 256, d = r % 256;
    ghist[((size_t)p * nseg + g) * 256 + d] = t;
}

// Items per thread of a sort tile (the scatter holds a tile in registers and
// LDS): 16 for sorts of at least OS_BIG items, where the passes are short of
// neither tiles nor waves, else 8 (more, shorter tiles run at once).
constexpr int64_t OS_BIG = (int64_t)1 << 20;
inline int os_ipt(int nseg, int64_t len) { return (int64_t)nseg * len >= OS_BIG ? 16 : 8; }

// One digit pass.  Wave w of a tile owns the tile's items [w * OS_IPT * 64,
// (w + 1) * OS_IPT * 64) and walks them in OS_IPT rounds of 64; a lane's rank among the round's
// items with its digit comes from ballots, and each wave keeps its own running
// offset per digit in LDS, so the ranking needs no block barrier.  The ranked
// items are first placed in LDS in the tile's digit order, then written out
// by consecutive threads, so each digit's run of the tile leaves as one
// contiguous store sequence instead of scattered single items.
template <class K, int OS_IPT>
__global__ void __launch_bounds__(TB) k_os_scatter(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                   K *__restrict__ kout, uint32_t *__restrict__ vout, int64_t len,
                                                   int64_t tps, int shift, const uint32_t *__restrict__ ghist,
                                                   uint32_t *__restrict__ status, uint32_t *__restrict__ tile_ctr,
                                                   uint32_t *__restrict__ err) {
    constexpr int R = 256;
    constexpr int OS_TILE = TB * OS_IPT;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t start[R];     // where the tile's run of each digit begins in the segment
    __shared__ uint32_t tstart[R];    // ... and in the tile's digit order
    __shared__ uint32_t wrun[NW][R];  // per-wave digit counts, then per-wave running offsets
    __shared__ uint32_t lw[NW];
    __shared__ K skey[OS_TILE];          // the tile in digit order
    __shared__ uint32_t sval[OS_TILE];
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1u);
#pragma unroll
    for (int q = 0; q < NW; ++q) wrun[q][threadIdx.x] = 0;
    __syncthreads();
    const uint32_t t = s_tile;               // global tile id
    const int64_t g = (int64_t)t / tps;      // its segment
    const int64_t ts = (int64_t)t - g * tps; // tile within the segment
    const int64_t seg0 = g * len;
    const int64_t wbase = ts * OS_TILE + (int64_t)w * (OS_IPT * WAVE);   // this wave's first item in the segment
    // the wave's items stay in registers for the whole pass (one load round)
    K key[OS_IPT];
    uint32_t val[OS_IPT];
#pragma unroll
    for (int r = 0; r < OS_IPT; ++r) {
        const int64_t j = wbase + (int64_t)r * WAVE + lane;
        key[r] = j < len ? kin[seg0 + j] : K(0);
        val[r] = j < len ? vin[seg0 + j] : 0u;
    }
    // lanes with the same digit in each round (eight ballots match the digit)
    uint64_t same[OS_IPT];
#pragma unroll
    for (int r = 0; r < OS_IPT; ++r) {
        const bool valid = wbase + (int64_t)r * WAVE + lane < len;
        const uint32_t dg = (uint32_t)(key[r] >> shift) & 255u;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot(valid && ((dg >> b) & 1u));
            m &= ((dg >> b) & 1u) ? bal : ~bal;
        }
        same[r] = valid ? m : 0ull;
        // the lowest lane of each digit group adds the group's size (one
        // writer per address per round; a wave's LDS operations stay in order)
        if (valid && __popcll(m & lt_mask) == 0) wrun[w][dg] += (uint32_t)__popcll(m);
    }
    __syncthreads();
    // this tile's count of digit d: publish it, then look back over the
    // segment's earlier tiles
    const int d = threadIdx.x;
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) c += wrun[q][d];
    uint32_t excl = 0;
    if (ts == 0) {
        store_agent(&status[(size_t)t * R + d], ST_PRE | c);
    } else {
        store_agent(&status[(size_t)t * R + d], ST_AGG | c);
        int64_t q = (int64_t)t - 1;
        uint32_t spins = 0;
        while (true) {
            const uint32_t v = load_agent(&status[(size_t)q * R + d]);
            const uint32_t flag = v & ~ST_VAL;
            if (flag == 0) {
                if (++spins > LOOKBACK_SPINS) {
                    atomicOr(err, 1u);
                    break;
                }
                continue;
            }
            excl += v & ST_VAL;
            if (flag == ST_PRE) break;
            --q;   // a segment's first tile publishes a prefix, so q stays in the segment
        }
        store_agent(&status[(size_t)t * R + d], ST_PRE | (excl + c));
    }
    // start of every digit in the segment: counts of smaller digits
    uint32_t tot;
    const uint32_t gex = block_excl_scan(ghist[(size_t)g * R + d], lw, &tot);
    start[d] = gex + excl;
    uint32_t tcount;
    tstart[d] = block_excl_scan(c, lw, &tcount);
    // per-wave counts -> offsets of each wave's run inside the tile's run
    uint32_t run = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        const uint32_t k = wrun[q][d];
        wrun[q][d] = run;
        run += k;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < OS_IPT; ++r) {
        if (same[r] == 0ull) continue;   // lane holds no item in this round
        const uint32_t dg = (uint32_t)(key[r] >> shift) & 255u;
        const uint32_t rank = (uint32_t)__popcll(same[r] & lt_mask);
        const uint32_t lp = tstart[dg] + wrun[w][dg] + rank;   // place in the tile's digit order
        skey[lp] = key[r];
        sval[lp] = val[r];
        if (rank == 0) wrun[w][dg] += (uint32_t)__popcll(same[r]);
    }
    __syncthreads();
    // item i of the tile's digit order goes to its digit's segment start plus
    // its place in the digit's run of the tile
#pragma unroll
    for (int r = 0; r < OS_IPT; ++r) {
        const uint32_t i = (uint32_t)(r * TB) + threadIdx.x;
        if (i < tcount) {
            const K k = skey[i];
            const uint32_t dg = (uint32_t)(k >> shift) & 255u;
            const uint32_t pos = start[dg] + (i - tstart[dg]);
            kout[seg0 + pos] = k;
            vout[seg0 + pos] = sval[i];
        }
    }
}

constexpr int MAX_SEG = 8;
constexpr int HIST_BLOCKS = 256;          // blocks of the histogram pass (per-block partials)
constexpr int ATOMIC_HIST_BLOCKS = 64;    // blocks of the histogram pass (atomics, small inputs)

// tmp layout: [err (64 words)] [ghist npass*nseg*256] [tile counters 64]
// [status npass*nseg*tps*256] [per-block histograms HIST_BLOCKS*nseg*npass*256].  The error word (tmp[0], set if a look-back
// wait ever exceeds its bound) is not cleared here: callers clear it once and
// read it at their next sync.
template <class K>
capt_status radix_sort(K *k0, uint32_t *v0, K *k1, uint32_t *v1, int nseg, int64_t len, int bits, uint32_t *tmp,
                       hipStream_t s, int *where, bool cleared = false) {
    *where = 0;
    if (len <= 1 || bits <= 0 || nseg <= 0) return CAPT_OK;
    if (nseg > MAX_SEG || len >= ((int64_t)1 << 30)) {   // 30-bit counts per segment
        set_error("radix sort of %d x %lld keys exceeds the supported size", nseg, (long long)len);
        return CAPT_EUNSUPPORTED;
    }
    const int npass = (bits + 7) / 8;
    const int ipt = os_ipt(nseg, len);
    const int64_t tile = (int64_t)TB * ipt;
    const int64_t tps = (len + tile - 1) / tile;
    const int64_t ntiles = tps * nseg;
    uint32_t *err = tmp;
    uint32_t *ghist = tmp + 64;
    uint32_t *ctr = ghist + (size_t)npass * nseg * 256;
    uint32_t *status = ctr + 64;
    const int64_t words = 64 + (int64_t)npass * nseg * 256 + 64 + (int64_t)npass * ntiles * 256;
    if (!cleared) {
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 1024)), dim3(256), 0, s,
                           tmp + 64, words - 64, 0u);
        CAPT_LAUNCH_CHECK();
    }
    const size_t hl = sizeof(uint32_t) * (size_t)nseg * npass * 256;
    if (ntiles <= 4 * ATOMIC_HIST_BLOCKS) {
        // small inputs: one kernel, block histograms added with atomics
        hipLaunchKernelGGL((k_os_hist<K, true>), dim3((unsigned)std::min<int64_t>(ntiles, ATOMIC_HIST_BLOCKS)),
                           dim3(TB), hl, s, k0, len, nseg, npass, ghist);
        CAPT_LAUNCH_CHECK();
    } else {
        // large inputs: per-block histograms, then one add per bin
        const int hblocks = (int)std::min<int64_t>(HIST_BLOCKS, ntiles / 4);
        uint32_t *hpart = status + (size_t)npass * ntiles * 256;
        hipLaunchKernelGGL((k_os_hist<K, false>), dim3((unsigned)hblocks), dim3(TB), hl, s, k0, len, nseg, npass,
                           hpart);
        CAPT_LAUNCH_CHECK();
        const int nh = nseg * npass * 256;
        hipLaunchKernelGGL(k_os_hist_sum, dim3((unsigned)((nh + HS_BINS - 1) / HS_BINS)), dim3(TB), 0, s, hpart,
                           hblocks, nseg, npass, ghist);
        CAPT_LAUNCH_CHECK();
    }
    K *ki = k0, *ko = k1;
    uint32_t *vi = v0, *vo = v1;
    for (int p = 0; p < npass; ++p) {
        if (ipt == 16)
            hipLaunchKernelGGL((k_os_scatter<K, 16>), dim3((unsigned)ntiles), dim3(TB), 0, s, ki, vi, ko, vo, len, tps,
                               8 * p, ghist + (size_t)p * nseg * 256, status + (size_t)p * ntiles * 256, ctr + p, err);
        else
            hipLaunchKernelGGL((k_os_scatter<K, 8>), dim3((unsigned)ntiles), dim3(TB), 0, s, ki, vi, ko, vo, len, tps,
                               8 * p, ghist + (size_t)p * nseg * 256, status + (size_t)p * ntiles * 256, ctr + p, err);
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

size_t scan_lb_words(int64_t n) { return (size_t)((n + TILE - 1) / TILE + 1); }

capt_status scan_exclusive_u32_lb(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *status, uint32_t *err,
                                  hipStream_t s) {
    if (n <= 0) return CAPT_OK;
    if (n >= ((int64_t)1 << 30)) {
        set_error("one-pass scan of %lld values exceeds 2^30", (long long)n);
        return CAPT_EUNSUPPORTED;
    }
    const int64_t nt = (n + TILE - 1) / TILE;
    hipLaunchKernelGGL(k_scan_lb, dim3((unsigned)nt), dim3(TB), 0, s, in, out, n, status, nt, err);
    CAPT_LAUNCH_CHECK();
    return CAPT_OK;
}

size_t radix_tmp_words(int64_t n) { return radix_tmp_words_seg(1, n); }

size_t radix_tmp_words_seg(int nseg, int64_t len) {
    const int64_t tile = (int64_t)TB * os_ipt(nseg, len);
    const int64_t tps = (len + tile - 1) / tile;
    return (size_t)(64 + 8 * 256 * (int64_t)nseg + 64 + 8 * tps * nseg * 256 +
                    (int64_t)HIST_BLOCKS * nseg * 8 * 256 + 64);
}

capt_status radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n,
                           int bits, uint32_t *tmp, hipStream_t s, int *where) {
    return radix_sort<uint64_t>(k0, v0, k1, v1, 1, n, bits, tmp, s, where);
}

capt_status radix_sort_u64_seg(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int nseg, int64_t len,
                               int bits, uint32_t *tmp, hipStream_t s, int *where) {
    return radix_sort<uint64_t>(k0, v0, k1, v1, nseg, len, bits, tmp, s, where);
}

capt_status radix_sort_u32(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n,
                           int bits, uint32_t *tmp, hipStream_t s, int *where, bool cleared) {
    return radix_sort<uint32_t>(k0, v0, k1, v1, 1, n, bits, tmp, s, where, cleared);
}

capt_status radix_sort_u32_seg(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int nseg, int64_t len,
                               int bits, uint32_t *tmp, hipStream_t s, int *where, bool cleared) {
    return radix_sort<uint32_t>(k0, v0, k1, v1, nseg, len, bits, tmp, s, where, cleared);
}

int64_t radix_clear_words(int nseg, int64_t len, int bits) {
    if (len <= 1 || bits <= 0 || nseg <= 0) return 0;
    const int64_t npass = (bits + 7) / 8;
    const int64_t tile = (int64_t)TB * os_ipt(nseg, len);
    const int64_t ntiles = ((len + tile - 1) / tile) * nseg;
    return npass * nseg * 256 + 64 + npass * ntiles * 256;
}

}  // namespace capt
