// GPU construction of collision-affording point trees (Alg. 1, Sec. IV-A/B).
//
// Alg. 1 recurses with a cell c and an afforded set z; on a GPU the same tree
// is produced level-synchronously:
//  1. presort: the padded point ids sorted by (coordinate, id) on each axis,
//     the three lists in one segmented radix sort (pad points sit at +inf);
//  2. splits: at depth d every node is a contiguous, aligned segment of the
//     three lists.  The node's split value is the coordinate of the last
//     element of the lower half of the list sorted on axis d mod 3 (the lower
//     median under (coordinate, id)); the other two lists are stably
//     partitioned by "goes left", which keeps every half sorted on every
//     axis.  Levels whose segments exceed LMAX run as one kernel each (the
//     partition finds offsets by decoupled look-back and already emits the
//     next level's split values and flags); the remaining levels of each
//     LMAX-point subtree run in LDS in one launch.
//  3. leaf cells from the split values of each leaf's ancestors;
//  4. affordance sets: instead of carrying z down the recursion, each leaf
//     collects {p : dist(p, cell) <= R} directly from a uniform grid of the
//     points (bins of side R / 2, points sorted by bin), scanning the bin
//     range around its cell.  Both constructions give the same set
//     (Lemma 1, case 1); the float64 distance test is monotone under cell
//     shrinking, so they agree exactly.  A count pass sizes the sets, a scan
//     places them (each set starts at a multiple of SET_ALIGN entries), a fill
//     pass writes them with each leaf's AABB and the box of every 16-entry
//     chunk.
#include <cmath>
#include <string>
#include <thread>

#include "capt_internal.h"

namespace capt {

namespace {

constexpr int TB = 256;
constexpr int LMAX = 1024;   // subtree size finished in LDS (27 KB, so a block fits beside a running query)
constexpr int LMAX_LOG2 = 10;
constexpr int LTB = 512;     // threads of the LDS levels kernel (8 waves, so a block fits beside a running query)
constexpr int AU = 2;        // 64-candidate steps in flight in the affordance kernels
constexpr int GTILE = 2048;  // tile of the global partition passes
constexpr int BUILD_STREAMS = 4;   // streams a build of several clouds spreads them over

__device__ __forceinline__ uint32_t ord_key(float v) {
    if (v == 0.0f) v = 0.0f;  // -0 and +0 compare equal
    uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float coord_of(const float *xyz, int64_t n, uint32_t id, int a) {
    return (int64_t)id < n ? xyz[3 * (int64_t)id + a] : INFINITY;
}


__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


// Zero regions of a build's scratch in one launch: the totals, the two sorts' error words
// and the rest of their scratch (r1, r2 words after the error words), the bin
// counts, the scan and level status words.
__global__ void k_binit(unsigned long long *__restrict__ totals, uint32_t *__restrict__ errw,
                        uint32_t *__restrict__ errw2, uint32_t *__restrict__ cstart, int64_t ncs,
                        uint32_t *__restrict__ scan_st, int64_t nss, int64_t r1, int64_t r2,
                        uint32_t *__restrict__ lvl, int64_t nlvl) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 4) totals[t] = 0ull;
    if (t < 64) errw[t] = 0u;
    if (t < 64) errw2[t] = 0u;
    for (int64_t i = t; i < ncs; i += stride) cstart[i] = 0u;
    for (int64_t i = t; i < nss; i += stride) scan_st[i] = 0u;
    for (int64_t i = t; i < r1; i += stride) errw[64 + i] = 0u;
    for (int64_t i = t; i < r2; i += stride) errw2[64 + i] = 0u;
    for (int64_t i = t; i < nlvl; i += stride) lvl[i] = 0u;
}

// One read of the cloud: sort keys of all three axes (segment a of keys /
// vals holds axis a), the forest's copy of the points, the count of
// non-finite coordinates and the bounding box of the finite ones, both as
// per-block partials (bbp[6 b ..], badp[b]).
__global__ void __launch_bounds__(TB) k_presort_keys(const float *__restrict__ xyz, int64_t n, int64_t N,
                                                     uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                     float *__restrict__ pts, float *__restrict__ bbp,
                                                     uint32_t *__restrict__ badp) {
    __shared__ float sl[TB / WAVE][6];
    __shared__ uint32_t sb[TB / WAVE];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    uint32_t bad = 0;
    if (j < N) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float v = INFINITY;
            if (j < n) {
                v = xyz[3 * j + a];
                pts[3 * j + a] = v;
                if (isfinite(v)) {
                    lo[a] = v;
                    hi[a] = v;
                } else {
                    ++bad;
                }
            }
            keys[a * N + j] = j < n ? ord_key(v) : 0xFFFFFFFFu;
            vals[a * N + j] = (uint32_t)j;
        }
    }
    for (int off = WAVE / 2; off >= 1; off >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], off, WAVE));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off, WAVE));
        }
        bad += (uint32_t)__shfl_xor((int)bad, off, WAVE);
    }
    const int w = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        for (int a = 0; a < 3; ++a) {
            sl[w][a] = lo[a];
            sl[w][3 + a] = hi[a];
        }
        sb[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        float v = sl[0][threadIdx.x];
        for (int i = 1; i < TB / WAVE; ++i) v = threadIdx.x < 3 ? fminf(v, sl[i][threadIdx.x]) : fmaxf(v, sl[i][threadIdx.x]);
        bbp[6 * blockIdx.x + threadIdx.x] = v;
    }
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < TB / WAVE; ++i) t += sb[i];
        badp[blockIdx.x] = t;
    }
}

// Global level: split values and "goes left" flags from the list on axis a.
__global__ void k_glevel_split(const uint32_t *__restrict__ La, const float *__restrict__ xyz,
                               int64_t n, int64_t N, int d, int a, float *__restrict__ T,
                               uint8_t *__restrict__ left) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const int64_t s = N >> d, h = s >> 1;
    const int64_t k = q & (s - 1);
    uint32_t p = La[q];
    left[p] = (uint8_t)(k < h);
    const int lg = 63 - __builtin_clzll((unsigned long long)s);   // log2(s)
    if (k == h - 1) T[((int64_t)1 << d) - 1 + (q >> lg)] = coord_of(xyz, n, p, a);
}

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *lw, uint32_t *total) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    uint32_t inc = v;
#pragma unroll
    for (int dd = 1; dd < WAVE; dd <<= 1) {
        uint32_t t = __shfl_up(inc, dd, WAVE);
        if (lane >= dd) inc += t;
    }
    if (lane == WAVE - 1) lw[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) {
        uint32_t t = lw[i];
        off += (i < w) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// One global level d in one launch: the two lists not on the split axis are
// stably partitioned inside every segment of s = N >> d positions ("goes
// left" first), tiles of GTILE finding their offset inside the segment by
// decoupled look-back over the segment's earlier tiles (a segment's first
// tile publishes a prefix at once, so every wait ends; waits are also
// bounded).  When level d + 1 splits on another axis, the first of the two
// lists is on that axis (`an`) and its new order fixes that level: while
// scattering it the kernel writes level d + 1's split values and "goes left"
// flags (when `next` is set).
constexpr uint32_t LB_AGG = 1u << 30;
constexpr uint32_t LB_PRE = 2u << 30;
constexpr uint32_t LB_VAL = (1u << 30) - 1u;
constexpr uint32_t LB_SPINS = 1u << 20;

__global__ void __launch_bounds__(TB) k_glevel(const uint32_t *__restrict__ Lb1, const uint32_t *__restrict__ Lb2,
                                               uint32_t *__restrict__ Ob1, uint32_t *__restrict__ Ob2,
                                               const uint8_t *__restrict__ left, uint8_t *__restrict__ left_next,
                                               const float *__restrict__ xyz, int64_t n, int64_t N, int d, int next,
                                               int an, float *__restrict__ T, uint32_t *__restrict__ status,
                                               uint32_t *__restrict__ ctr, int64_t ntile, uint32_t *__restrict__ err) {
    __shared__ uint32_t lw[TB / WAVE];
    __shared__ uint32_t s_tile, s_excl;
    const int y = blockIdx.y;
    const uint32_t *L = y ? Lb2 : Lb1;
    uint32_t *O = y ? Ob2 : Ob1;
    uint32_t *St = status + (size_t)y * ntile;
    if (threadIdx.x == 0) s_tile = atomicAdd(&ctr[y], 1u);
    __syncthreads();
    const int64_t t = s_tile;
    const int64_t s = N >> d, h = s >> 1;
    const int64_t tps = s / GTILE;   // >= 2 on a global level
    const int64_t base = t * GTILE + (int64_t)threadIdx.x * 8;
    uint32_t p[8], f[8], c = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        p[i] = L[base + i];
        f[i] = left[p[i]];
        c += f[i];
    }
    uint32_t tot;
    uint32_t e = block_excl_scan(c, lw, &tot);
    if (threadIdx.x == 0) {
        const int64_t t0 = t & ~(tps - 1);   // the segment's first tile
        uint32_t ex = 0;
        if (t == t0) {
            st_agent(&St[t], LB_PRE | tot);
        } else {
            st_agent(&St[t], LB_AGG | tot);
            int64_t q = t - 1;
            uint32_t spins = 0;
            while (true) {
                const uint32_t v = ld_agent(&St[q]);
                const uint32_t flag = v & ~LB_VAL;
                if (flag == 0) {
                    if (++spins > LB_SPINS) {
                        atomicOr(err, 8u);
                        break;
                    }
                    continue;
                }
                ex += v & LB_VAL;
                if (flag == LB_PRE) break;
                --q;
            }
            st_agent(&St[t], LB_PRE | (ex + tot));
        }
        s_excl = ex;
    }
    __syncthreads();
    e += s_excl;   // left-goers of the segment before this thread's items
    const int64_t seg = base & ~(s - 1);
    const int64_t s2 = s >> 1, h2 = s2 >> 1;
    const int lg2 = 62 - __builtin_clzll((unsigned long long)s);   // log2(s / 2)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t q = base + i;
        const int64_t lc = (int64_t)e;
        const int64_t np = f[i] ? seg + lc : seg + h + (q - seg - lc);
        O[np] = p[i];
        e += f[i];
        if (y == 0 && next) {
            const int64_t k2 = np & (s2 - 1);
            left_next[p[i]] = (uint8_t)(k2 < h2);
            if (k2 == h2 - 1) T[((int64_t)1 << (d + 1)) - 1 + (np >> lg2)] = coord_of(xyz, n, p[i], an);
        }
    }
}

__global__ void k_inverse(const uint32_t *__restrict__ L, int64_t N, uint32_t *__restrict__ inv) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < N) inv[L[q]] = (uint32_t)q;
}

// The remaining levels d0 .. D-1 of one subtree of S0 = N >> d0 <= LMAX
// points, in LDS.  Lists hold local indices (positions in the axis-0 list of
// the subtree).
__global__ void __launch_bounds__(LTB) k_local_levels(const uint32_t *__restrict__ L0,
                                                     const uint32_t *__restrict__ L1,
                                                     const uint32_t *__restrict__ L2,
                                                     const uint32_t *__restrict__ inv,
                                                     const float *__restrict__ xyz, int64_t n,
                                                     int64_t N, int D, int d0, uint64_t axes,
                                                     float *__restrict__ T,
                                                     int32_t *__restrict__ rep) {
    __shared__ uint32_t ids[LMAX];
    __shared__ float cx[3][LMAX];
    __shared__ uint16_t lst[3][LMAX];
    __shared__ uint16_t tmp[LMAX];
    __shared__ uint16_t escan[LMAX];
    __shared__ uint8_t flag[LMAX];
    __shared__ uint32_t lw[LTB / WAVE];
    const int S0 = (int)(N >> d0);
    const int64_t seg = (int64_t)blockIdx.x * S0;
    for (int k = threadIdx.x; k < S0; k += LTB) {
        uint32_t id = L0[seg + k];
        ids[k] = id;
        for (int a = 0; a < 3; ++a) cx[a][k] = coord_of(xyz, n, id, a);
        lst[0][k] = (uint16_t)k;
        lst[1][k] = (uint16_t)(inv[L1[seg + k]] - (uint32_t)seg);
        lst[2][k] = (uint16_t)(inv[L2[seg + k]] - (uint32_t)seg);
    }
    __syncthreads();
    for (int d = d0; d < D; ++d) {
        const int s = (int)(N >> d), h = s >> 1, a = axis_at(axes, d);
        const int64_t node0 = ((int64_t)1 << d) - 1 + (int64_t)blockIdx.x * (S0 / s);
        for (int j = threadIdx.x; j < S0 / s; j += LTB) T[node0 + j] = cx[a][lst[a][j * s + h - 1]];
        for (int k = threadIdx.x; k < S0; k += LTB) flag[lst[a][k]] = (uint8_t)((k & (s - 1)) < h);
        __syncthreads();
        for (int b = 1; b <= 2; ++b) {
            uint16_t *lb = lst[(a + b) % 3];
            // exclusive scan of flags over the S0 positions (a run per thread)
            const int per = (S0 + LTB - 1) / LTB;
            const int k0 = threadIdx.x * per;
            uint32_t c = 0;
            for (int i = 0; i < per; ++i) {
                int k = k0 + i;
                if (k < S0) c += flag[lb[k]];
            }
            uint32_t tot;
            uint32_t e = block_excl_scan(c, lw, &tot);
            for (int i = 0; i < per; ++i) {
                int k = k0 + i;
                if (k < S0) {
                    escan[k] = (uint16_t)e;
                    e += flag[lb[k]];
                }
            }
            __syncthreads();
            for (int k = threadIdx.x; k < S0; k += LTB) {
                const int sg = k & ~(s - 1);
                const int lc = (int)escan[k] - (int)escan[sg];
                const uint16_t v = lb[k];
                const int np = flag[v] ? sg + lc : sg + h + (k - sg - lc);
                tmp[np] = v;
            }
            __syncthreads();
            for (int k = threadIdx.x; k < S0; k += LTB) lb[k] = tmp[k];
            __syncthreads();
        }
    }
    for (int k = threadIdx.x; k < S0; k += LTB) rep[seg + k] = (int32_t)ids[lst[0][k]];
}

// Leaf cells from the split values of the ancestors (Alg. 1: the left child
// takes hi = T_i, the right child lo = T_i on the node's axis).
// float64 helpers, every operation rounded on its own
__device__ __forceinline__ double dsub(double a, double b) { return __dsub_rn(a, b); }
__device__ __forceinline__ double dmul(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ double dadd(double a, double b) { return __dadd_rn(a, b); }

// Cell of every leaf from its ancestors' split values (upper bound from a
// left descent, lower bound from a right one, +-inf where unbounded), then the
// r_min pruning of the leaf (Sec. IV-B): a bounded cell whose farthest corner
// is within r_min of the representative (float64, margin 2^-18).  Pruned
// leaves are counted per block (prp[b]).  Only leaves in [l0, l1) (a shard's
// subtree) may be pruned; the others keep empty sets.
__global__ void __launch_bounds__(TB) k_cells_prune(const float *__restrict__ T, int64_t N, int D, uint64_t axes,
                                                    float *__restrict__ cells, const int32_t *__restrict__ rep,
                                                    const float *__restrict__ xyz, int64_t n, int prune, double thr,
                                                    int64_t l0, int64_t l1, uint8_t *__restrict__ pruned,
                                                    uint32_t *__restrict__ prp) {
    __shared__ uint32_t sc[TB / WAVE];
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool pr = false;
    if (l < N) {
        float c[6] = {-INFINITY, -INFINITY, -INFINITY, INFINITY, INFINITY, INFINITY};
        int64_t i = 0;
        for (int d = 0; d < D; ++d) {
            const int a = axis_at(axes, d);
            const int bit = (int)((l >> (D - 1 - d)) & 1);
            if (bit) c[a] = T[i];
            else c[3 + a] = T[i];
            i = 2 * i + 1 + bit;
        }
        for (int k = 0; k < 6; ++k) cells[6 * l + k] = c[k];
        const int64_t id = rep[l];
        pr = prune && id < n && l >= l0 && l < l1;
        for (int k = 0; k < 6 && pr; ++k) pr = isfinite(c[k]);
        if (pr) {
            double far2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double t = (double)xyz[3 * id + a];
                const double lo = dsub(t, (double)c[a]);
                const double hi = dsub((double)c[3 + a], t);
                const double l2 = dmul(lo, lo), h2 = dmul(hi, hi);
                far2 = dadd(far2, l2 > h2 ? l2 : h2);
            }
            pr = far2 <= thr;
        }
        pruned[l] = (uint8_t)pr;
    }
    const uint32_t cnt = (uint32_t)__popcll(__ballot(pr));
    if ((threadIdx.x & (WAVE - 1)) == 0) sc[threadIdx.x / WAVE] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < TB / WAVE; ++i) t += sc[i];
        prp[blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// Affordance sets through a uniform grid over the points
// ---------------------------------------------------------------------------
// Grid of cubic bins of side g (>= R) over the cloud's bounding box.  Points
// are sorted by bin with x fastest, so the bins of one (y, z) row are one
// contiguous run of points.  A leaf's candidates are the rows covering its
// cell grown by R (one extra bin on every side absorbs rounding); every
// candidate then takes the exact float64 "affords" test.
struct Grid {
    double origin[3];
    double g;
    double inv;             // 1 / g
    double lo[3], hi[3];    // bounding box of the points
    int32_t dims[3];
    int32_t pad;
    int64_t ncells;
};



// Reduce the bounding-box partials (one block), store the non-finite count in
// totals[3], and lay the grid over the box.
__global__ void __launch_bounds__(TB) k_grid_setup(const float *__restrict__ bbp, const uint32_t *__restrict__ badp,
                                                   int64_t nb, double R, int64_t cap, Grid *G,
                                                   unsigned long long *__restrict__ totals) {
    __shared__ float sl[TB / WAVE][6];
    __shared__ uint32_t sb[TB / WAVE];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    uint32_t bad = 0;
    for (int64_t b = threadIdx.x; b < nb; b += TB) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], bbp[6 * b + a]);
            hi[a] = fmaxf(hi[a], bbp[6 * b + 3 + a]);
        }
        bad += badp[b];
    }
    for (int off = WAVE / 2; off >= 1; off >>= 1) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], off, WAVE));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off, WAVE));
        }
        bad += (uint32_t)__shfl_xor((int)bad, off, WAVE);
    }
    const int w = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        for (int a = 0; a < 3; ++a) {
            sl[w][a] = lo[a];
            sl[w][3 + a] = hi[a];
        }
        sb[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int i = 1; i < TB / WAVE; ++i) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(sl[0][a], sl[i][a]);
            sl[0][a] = lo[a];
            hi[a] = fmaxf(sl[0][3 + a], sl[i][3 + a]);
            sl[0][3 + a] = hi[a];
        }
        sb[0] += sb[i];
    }
    for (int a = 0; a < 3; ++a) {
        lo[a] = sl[0][a];
        hi[a] = sl[0][3 + a];
    }
    totals[3] = sb[0];
    Grid g;
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = (double)lo[a];
        g.hi[a] = (double)hi[a];
        if (!(g.lo[a] <= g.hi[a]) || !isfinite(g.lo[a]) || !isfinite(g.hi[a])) g.lo[a] = g.hi[a] = 0.0;   // empty cloud
        g.origin[a] = g.lo[a];
        ext = fmax(ext, g.hi[a] - g.lo[a]);
    }
    double step = R * 0.5;   // bins of half the reach: fewer candidates per leaf
    if (ext / step > 1000.0) step = ext / 1000.0;
    int64_t total = 0;
    for (int it = 0; it < 64; ++it) {
        total = 1;
        for (int a = 0; a < 3; ++a) {
            g.dims[a] = (int32_t)floor((g.hi[a] - g.lo[a]) / step) + 1;
            total *= g.dims[a];
        }
        if (total <= cap) break;
        step *= 1.25;
    }
    g.g = step;
    g.inv = 1.0 / step;
    g.pad = 0;
    g.ncells = total;
    *G = g;
}

__device__ __forceinline__ int32_t bin_clamp(double t, int32_t dim) {
    if (!(t >= 0.0)) t = 0.0;   // also catches NaN (non-finite input is rejected after the build's sync)
    if (t > (double)(dim - 1)) t = (double)(dim - 1);
    return (int32_t)t;
}

__device__ __forceinline__ int32_t bin_of(double v, double origin, double g, int32_t dim) {
    return bin_clamp(floor((v - origin) / g), dim);
}

// Bounds on bin_of from a product with 1 / g: bin_lo(v) <= bin_of(v) <=
// bin_hi(v).  The product and the quotient differ by a few units in the last
// place, far inside the 2^-40 margins, and the clamp keeps the order.
__device__ __forceinline__ int32_t bin_lo(double v, double origin, double inv, int32_t dim) {
    return bin_clamp(floor((v - origin) * inv * (1.0 - 0x1p-40)), dim);
}
__device__ __forceinline__ int32_t bin_hi(double v, double origin, double inv, int32_t dim) {
    return bin_clamp(floor((v - origin) * inv * (1.0 + 0x1p-40)), dim);
}

__global__ void k_grid_keys(const float *__restrict__ xyz, int64_t n, const Grid *__restrict__ G,
                            uint32_t *__restrict__ key, uint32_t *__restrict__ val,
                            uint32_t *__restrict__ cellcnt) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const Grid g = *G;
    int32_t b[3];
    for (int a = 0; a < 3; ++a) b[a] = bin_of((double)xyz[3 * j + a], g.origin[a], g.g, g.dims[a]);
    const uint32_t c = (uint32_t)(((int64_t)b[2] * g.dims[1] + b[1]) * g.dims[0] + b[0]);
    key[j] = c;
    val[j] = (uint32_t)j;
    atomicAdd(&cellcnt[c], 1u);
}

__global__ void k_grid_gather(const float *__restrict__ xyz, const uint32_t *__restrict__ val, int64_t n,
                              float *__restrict__ sx, float *__restrict__ sy, float *__restrict__ sz) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t id = val[k];
    sx[k] = xyz[3 * id];
    sy[k] = xyz[3 * id + 1];
    sz[k] = xyz[3 * id + 2];
}

// Inclusive scan over the 64 lanes with DPP adds (row shifts, then the row
// totals through row_bcast:15 and row_bcast:31).
__device__ __forceinline__ uint32_t wave_incl_scan_b(uint32_t v, int) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
    return v;
}

struct AffArgs {
    const float *cells;
    const int32_t *rep;
    const uint8_t *pruned;
    const float *xyz;
    const Grid *grid;
    const uint32_t *cstart;    // [ncells + 1] first sorted point of every bin
    const float *sx, *sy, *sz; // points sorted by bin
    const uint32_t *sid;       // original index of each sorted point
    int64_t n, N;
    int64_t l0, l1;            // leaves that get sets (a shard's subtree); the others stay empty
    double R2;                 // (r_max (1 + 2^-20))^2
    double R;
    // float32 pre-test: a float32 squared distance at most R2lo is afforded and
    // one above R2hi is not (its relative error is below 6 * 2^-24, the band
    // is R2 (1 -+ 2^-21)); only candidates in between take the float64 test.
    float R2lo, R2hi;
    int pre32;                 // R2 within [1e-30, 1e30], where that bound holds
};

// LDS sync of one wave (lanes write what other lanes of the wave read).
__device__ __forceinline__ void wave_lds_sync_b() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive maximum over the 64 lanes (lanes that receive nothing take -1).
__device__ __forceinline__ int wave_incl_max_b(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x111, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x112, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x114, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x118, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x142, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x143, 0xc, 0xf, false));
    return v;
}

// Minimum / maximum over each row of 16 lanes, in every lane of the row: DPP
// swaps within quads (quad_perm [1,0,3,2], then [2,3,0,1]), then the
// half-row mirror (lane i <-> 7 - i of each 8) and the row mirror
// (i <-> 15 - i), each step fused into the min / max.
__device__ __forceinline__ float dpp_f(float v, int ctrl) {
    switch (ctrl) {   // the control must be a constant of the builtin
        case 0xB1: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xf, 0xf, false));
        case 0x4E: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xf, 0xf, false));
        case 0x141: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xf, 0xf, false));
        default: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xf, 0xf, false));
    }
}
__device__ __forceinline__ float row16_min(float v) {
    v = fminf(v, dpp_f(v, 0xB1));
    v = fminf(v, dpp_f(v, 0x4E));
    v = fminf(v, dpp_f(v, 0x141));
    return fminf(v, dpp_f(v, 0x140));
}
__device__ __forceinline__ float row16_max(float v) {
    v = fmaxf(v, dpp_f(v, 0xB1));
    v = fmaxf(v, dpp_f(v, 0x4E));
    v = fmaxf(v, dpp_f(v, 0x141));
    return fmaxf(v, dpp_f(v, 0x140));
}
// The same over float keys: ok(f) maps floats (no NaN) to int32 in the same
// order (-0 below +0), so the row reductions are integer min / max, which
// fold into one DPP instruction each.
__device__ __forceinline__ int32_t ok_of(float f) {
    const int32_t b = __float_as_int(f);
    return b ^ ((b >> 31) & 0x7FFFFFFF);
}
__device__ __forceinline__ float ok_float(int32_t k) { return __int_as_float(k ^ ((k >> 31) & 0x7FFFFFFF)); }
__device__ __forceinline__ int32_t row16_min_i(int32_t v) {
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0xB1, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x4E, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x141, 0xf, 0xf, false));
    return min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x140, 0xf, 0xf, false));
}
__device__ __forceinline__ int32_t row16_max_i(int32_t v) {
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0xB1, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x4E, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x141, 0xf, 0xf, false));
    return max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x140, 0xf, 0xf, false));
}
// ... and over the whole wave, uniform: the four row results by readlane.
__device__ __forceinline__ float wave_min_f(float v) {
    v = row16_min(v);
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return fminf(fminf(a, b), fminf(c, d));
}
__device__ __forceinline__ float wave_max_f(float v) {
    v = row16_max(v);
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return fmaxf(fmaxf(a, b), fmaxf(c, d));
}

// LPW consecutive leaves per wavefront, one after the other; the wave's lanes
// first set up those leaves side by side (the cell, the bins of its reach).
// COUNT: write the set size and the leaf record's bounding box of the set.
// FILL: write the set (rows in order, points in bin order), its padding, the
// leaf record's start and length, and the box of every 16-entry chunk.  The
// fill stages the accepted points in a per-wave LDS ring and encodes the chunk
// boxes from there, four chunks at a time, as they complete (their base, the
// set's box, is known from the count pass).
constexpr uint32_t RING = 256;   // staged set entries per wave (> (AU + 1) * WAVE)
constexpr int LPW = 4;           // leaves per wave (more leave a longer tail of slow waves)
template <bool FILL>
__global__ void __launch_bounds__(256) k_afford_grid(AffArgs A, uint32_t *__restrict__ count,
                                                     const uint32_t *__restrict__ pstart,
                                                     float *__restrict__ px, float *__restrict__ py,
                                                     float *__restrict__ pz, int32_t *__restrict__ pidx,
                                                     Leaf *__restrict__ leaf, uint4 *__restrict__ cbox) {
    __shared__ int8_t s_start[256 / WAVE][WAVE];   // per wave: the row whose candidates start at a slot
    __shared__ float s_ring[FILL ? 256 / WAVE : 1][3][FILL ? RING : 1];
    static_assert(LPW <= WAVE, "one lane sets up one leaf");
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t lw = ((int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE) * LPW;   // first leaf
    if (lw >= A.N) return;
    int8_t *S = s_start[threadIdx.x / WAVE];
    float *rx = s_ring[FILL ? threadIdx.x / WAVE : 0][0];
    float *ry = s_ring[FILL ? threadIdx.x / WAVE : 0][1];
    float *rz = s_ring[FILL ? threadIdx.x / WAVE : 0][2];
    const Grid g = *A.grid;
    // Set-up, lane i for leaf lw + i: the set the leaf gets (1: its
    // representative alone, a pruned leaf; 2: the grid gather; 0: none) and,
    // for the gather, its cell and the bins of its reach on every axis.
    int kind = 0;
    int32_t pb0[3] = {0, 0, 0}, pb1[3] = {-1, -1, -1};
    float pcl[3] = {0.f, 0.f, 0.f}, pch[3] = {0.f, 0.f, 0.f};
    {
        const int64_t lm = lw + lane;
        if (lane < LPW && lm < A.N) {
            if (A.pruned[lm]) {
                kind = 1;
            } else if (A.n > 0 && lm >= A.l0 && lm < A.l1) {
                const float *c = A.cells + 6 * lm;
                bool empty = false;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    pcl[a] = c[a];
                    pch[a] = c[3 + a];
                    const double cl = (double)pcl[a], ch = (double)pch[a];
                    // A point that passes the float64 test below lies within R
                    // of the cell on every axis up to rounding (about 1e-16
                    // relative); the slack covers that, and bin_of is
                    // monotone, so the bins from bin_of(lo_b) to bin_of(hi_b)
                    // hold every such point.  The range taken, bin_lo(lo_b) to
                    // bin_hi(hi_b), may add a bin on a side: its points lie
                    // outside [lo_b, hi_b] on that axis, fail the test and
                    // leave the set and its order as they are.
                    const double slack =
                        1e-9 * (A.R + 1.0 + (isfinite(cl) ? fabs(cl) : 0.0) + (isfinite(ch) ? fabs(ch) : 0.0));
                    const double lo_b = fmax(cl - A.R - slack, g.lo[a]);
                    const double hi_b = fmin(ch + A.R + slack, g.hi[a]);
                    if (!(lo_b <= hi_b)) {
                        empty = true;
                    } else {
                        pb0[a] = bin_lo(lo_b, g.origin[a], g.inv, g.dims[a]);
                        pb1[a] = bin_hi(hi_b, g.origin[a], g.inv, g.dims[a]);
                    }
                }
                if (!empty) kind = 2;
            }
        }
    }
    for (int li = 0; li < LPW; ++li) {
        const int64_t l = lw + li;
        if (l >= A.N) break;
        const uint32_t out0 = FILL ? pstart[l] : 0u;
        // FILL: the set's box corner, the chunk boxes' base (scalars: a lane picks
        // one by a lane-dependent choice, which must not become an indexed array)
        float bx = 0.f, by = 0.f, bz = 0.f;
        if (FILL) {
            const Leaf L0 = leaf[l];
            bx = L0.lo[0];
            by = L0.lo[1];
            bz = L0.lo[2];
        }
        uint32_t cnt = 0;
        uint32_t done = 0;   // FILL: entries whose chunk boxes are written
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        // chunk boxes of set positions [first, first + 64) from the ring, up to
        // `end` (later positions, padding, stay out of the boxes)
        auto boxes = [&](uint32_t first, uint32_t end) {
            static_assert(CHUNK == 16, "chunk boxes reduce over DPP rows of 16 lanes");
            wave_lds_sync_b();
            const uint32_t p = first + (uint32_t)lane;
            const bool real = p < cnt;
            const uint32_t q = p & (RING - 1);
            const float x = real ? rx[q] : 0.f, y = real ? ry[q] : 0.f, z = real ? rz[q] : 0.f;
            const int32_t kinf = ok_of(INFINITY), kninf = ok_of(-INFINITY);
            const int32_t lx = row16_min_i(real ? ok_of(x) : kinf), ly = row16_min_i(real ? ok_of(y) : kinf),
                          lz = row16_min_i(real ? ok_of(z) : kinf);
            const int32_t hx = row16_max_i(real ? ok_of(x) : kninf), hy = row16_max_i(real ? ok_of(y) : kninf),
                          hz = row16_max_i(real ? ok_of(z) : kninf);
            // lanes 0..5 of a chunk's row encode lo x, y, z, hi x, y, z (the
            // halves of hbox_encode, in its order), lanes 6 and 7 the zero pad
            const int j = lane & (CHUNK - 1);
            // (masks, not selects: the compiler turns a chain of lane-dependent
            // selects into a table in scratch memory)
            const int32_t m0 = -(int32_t)(j == 0), m1 = -(int32_t)(j == 1), m2 = -(int32_t)(j == 2);
            const int32_t m3 = -(int32_t)(j == 3), m4 = -(int32_t)(j == 4), m5 = -(int32_t)(j == 5);
            const int32_t kv = (lx & m0) | (ly & m1) | (lz & m2) | (hx & m3) | (hy & m4) | (hz & m5);
            const float b = __int_as_float((__float_as_int(bx) & (m0 | m3)) | (__float_as_int(by) & (m1 | m4)) |
                                           (__float_as_int(bz) & (m2 | m5)));
            const float v = ok_float(kv);
            const uint32_t h = j < 6 ? hbox_offset(b, v, j >= 3) : 0u;
            const uint32_t k = p / CHUNK;   // chunk of the set
            if (p - (uint32_t)j < end && j < 8)
                reinterpret_cast<uint16_t *>(cbox + (int64_t)out0 / CHUNK + k)[j] = (uint16_t)h;
            wave_lds_sync_b();   // the ring slots are free again
        };
        auto emit = [&](bool ok, float x, float y, float z, int32_t id) {
            const uint64_t m = __ballot(ok);
            if (ok) {
                if (FILL) {
                    const uint32_t rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                    const uint32_t pos = out0 + cnt + rank;
                    if (px) {   // not for indexed sets
                        const int64_t o = set_off(pos);
                        px[o] = x;
                        py[o] = y;
                        pz[o] = z;
                    }
                    pidx[pos] = id;
                    const uint32_t q = (cnt + rank) & (RING - 1);
                    rx[q] = x;
                    ry[q] = y;
                    rz[q] = z;
                } else {
                    lo[0] = fminf(lo[0], x); lo[1] = fminf(lo[1], y); lo[2] = fminf(lo[2], z);
                    hi[0] = fmaxf(hi[0], x); hi[1] = fmaxf(hi[1], y); hi[2] = fmaxf(hi[2], z);
                }
            }
            cnt += (uint32_t)__popcll(m);
        };
        const int kd = __builtin_amdgcn_readlane(kind, li);
        if (kd == 1) {
            const int64_t rid = A.rep[l];
            const float x = A.xyz[3 * rid], y = A.xyz[3 * rid + 1], z = A.xyz[3 * rid + 2];
            emit(lane == 0, x, y, z, (int32_t)rid);
        } else if (kd == 2) {
            double cl[3], ch[3];
            float clf[3], chf[3];
            int32_t b0[3], b1[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                clf[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pcl[a]), li));
                chf[a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pch[a]), li));
                cl[a] = (double)clf[a];
                ch[a] = (double)chf[a];
                b0[a] = __builtin_amdgcn_readlane(pb0[a], li);
                b1[a] = __builtin_amdgcn_readlane(pb1[a], li);
            }
            // (rows number at most the grid's cells, fewer than 2^32: the
            // row's place splits into y and z in 32-bit arithmetic)
            const uint32_t ny = (uint32_t)(b1[1] - b0[1] + 1);
            const int64_t nrows = (int64_t)ny * (int64_t)(b1[2] - b0[2] + 1);
            for (int64_t r0 = 0; r0 < nrows; r0 += WAVE) {
                const int64_t r = r0 + lane;
                uint32_t s = 0, e = 0;
                if (r < nrows) {
                    const uint32_t zr = (uint32_t)r / ny;
                    const int64_t y = b0[1] + (int64_t)((uint32_t)r - zr * ny), z = b0[2] + (int64_t)zr;
                    const int64_t row = (z * g.dims[1] + y) * g.dims[0];
                    s = A.cstart[row + b0[0]];
                    e = A.cstart[row + b1[0] + 1];
                }
                // the rows' candidates as one flattened list, AU steps of 64
                // in flight (all loads first, then tests and emits in order)
                const uint32_t rem = e - s;
                const uint32_t incl = wave_incl_scan_b(rem, lane);
                const uint32_t excl = incl - rem;
                const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
                const uint32_t base_l = s - excl;   // sorted index of list slot t of this row = base_l + t
                S[lane] = -1;
                int carry = -1;   // the row whose candidates cover the window's first slot
                for (uint32_t k0 = 0; k0 < total; k0 += AU * WAVE) {
                    float x[AU], y[AU], z[AU];
                    int32_t id[AU];
                    bool in[AU];
#pragma unroll
                    for (int u = 0; u < AU; ++u) {
                        const uint32_t w0 = k0 + (uint32_t)(u * WAVE);
                        const uint32_t slot = w0 + (uint32_t)lane;
                        in[u] = slot < total;
                        // the row of this slot: the last row starting at or before it
                        // (rows mark their first slot in LDS, then a prefix maximum)
                        if (rem > 0u && excl >= w0 && excl - w0 < (uint32_t)WAVE) S[excl - w0] = (int8_t)lane;
                        wave_lds_sync_b();
                        int sv = S[lane];
                        S[lane] = -1;
                        if (lane == 0) sv = max(sv, carry);
                        const int o = wave_incl_max_b(sv);
                        carry = __builtin_amdgcn_readlane(o, WAVE - 1);
                        const uint32_t k = __shfl(base_l, o, WAVE) + slot;
                        x[u] = y[u] = z[u] = 0.f;
                        id[u] = -1;
                        if (in[u]) {
                            x[u] = A.sx[k];
                            y[u] = A.sy[k];
                            z[u] = A.sz[k];
                            if (FILL) id[u] = (int32_t)A.sid[k];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < AU; ++u) {
                        bool ok = false;
                        bool open = in[u];
                        if (open && A.pre32) {
                            const float pf[3] = {x[u], y[u], z[u]};
                            float gs[3];
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                const float gg =
                                    fmaxf(fmaxf(__fsub_rn(clf[a], pf[a]), __fsub_rn(pf[a], chf[a])), 0.0f);
                                gs[a] = __fmul_rn(gg, gg);
                            }
                            const float d2f = __fadd_rn(__fadd_rn(gs[0], gs[1]), gs[2]);
                            if (d2f <= A.R2lo) {
                                ok = true;
                                open = false;
                            } else if (d2f > A.R2hi) {
                                open = false;
                            }
                        }
                        if (open) {
                            const double pp[3] = {(double)x[u], (double)y[u], (double)z[u]};
                            double d2 = 0.0;
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                const double below = dsub(cl[a], pp[a]);
                                const double above = dsub(pp[a], ch[a]);
                                double gg = below > above ? below : above;
                                if (gg < 0.0) gg = 0.0;
                                d2 = dadd(d2, dmul(gg, gg));
                            }
                            ok = d2 <= A.R2;
                        }
                        emit(ok, x[u], y[u], z[u], id[u]);
                    }
                    if (FILL) {
                        static_assert(RING > (AU + 1) * WAVE, "the ring holds the pending and the new entries");
                        while (cnt - done >= (uint32_t)WAVE) {   // four whole chunks are staged
                            boxes(done, done + WAVE);
                            done += WAVE;
                        }
                    }
                }
            }
        }
        if (!FILL) {
            for (int a = 0; a < 3; ++a) {
                lo[a] = wave_min_f(lo[a]);
                hi[a] = wave_max_f(hi[a]);
            }
            if (lane == 0) {
                count[l] = cnt;
                Leaf L;
                for (int a = 0; a < 3; ++a) {
                    L.lo[a] = lo[a];
                    L.hi[a] = hi[a];
                }
                L.start = 0;
                L.count = cnt;
                leaf[l] = L;
            }
            continue;
        }
        // padding, the chunk boxes still to write, the leaf record's placement
        const uint32_t padded = cnt ? ((cnt + SET_ALIGN - 1) / SET_ALIGN) * SET_ALIGN : 0u;
        for (uint32_t k = cnt + lane; k < padded; k += WAVE) {
            if (px) {
                const int64_t o = set_off(out0 + k);
                px[o] = INFINITY;
                py[o] = INFINITY;
                pz[o] = INFINITY;
            }
            pidx[out0 + k] = -1;
        }
        for (uint32_t first = done; first < padded; first += WAVE) boxes(first, padded);
        if (lane == 0) {
            leaf[l].start = out0;
            leaf[l].count = cnt;
        }
    }
}

// Padded set sizes, and per-block sums of the set sizes and padded sizes
// (pp[2 b], pp[2 b + 1]).
__global__ void __launch_bounds__(TB) k_pad_counts(const uint32_t *__restrict__ cnt, int64_t N,
                                                   uint32_t *__restrict__ out, unsigned long long *__restrict__ pp) {
    __shared__ unsigned long long sc[TB / WAVE][2];
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c = 0, p = 0;
    if (l < N) {
        const uint32_t v = cnt[l];
        const uint32_t q = v ? ((v + SET_ALIGN - 1) / SET_ALIGN) * SET_ALIGN : 0u;
        out[l] = q;
        c = v;
        p = q;
    }
    for (int off = WAVE / 2; off >= 1; off >>= 1) {
        c += __shfl_xor(c, off, WAVE);
        p += __shfl_xor(p, off, WAVE);
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        sc[threadIdx.x / WAVE][0] = c;
        sc[threadIdx.x / WAVE][1] = p;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tc = 0, tp = 0;
        for (int i = 0; i < TB / WAVE; ++i) {
            tc += sc[i][0];
            tp += sc[i][1];
        }
        pp[2 * blockIdx.x] = tc;
        pp[2 * blockIdx.x + 1] = tp;
    }
}

// totals[0..2] = set entries, padded entries, pruned leaves, from the
// per-block partials (one block).
__global__ void __launch_bounds__(TB) k_sum_partials(const unsigned long long *__restrict__ pp,
                                                     const uint32_t *__restrict__ prp, int64_t nb,
                                                     unsigned long long *__restrict__ totals) {
    __shared__ unsigned long long sc[TB / WAVE][3];
    unsigned long long c = 0, p = 0, r = 0;
    for (int64_t b = threadIdx.x; b < nb; b += TB) {
        c += pp[2 * b];
        p += pp[2 * b + 1];
        r += prp[b];
    }
    for (int off = WAVE / 2; off >= 1; off >>= 1) {
        c += __shfl_xor(c, off, WAVE);
        p += __shfl_xor(p, off, WAVE);
        r += __shfl_xor(r, off, WAVE);
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        sc[threadIdx.x / WAVE][0] = c;
        sc[threadIdx.x / WAVE][1] = p;
        sc[threadIdx.x / WAVE][2] = r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t[3] = {0, 0, 0};
        for (int i = 0; i < TB / WAVE; ++i)
            for (int k = 0; k < 3; ++k) t[k] += sc[i][k];
        for (int k = 0; k < 3; ++k) totals[k] = t[k];
    }
}

// A cloud's totals and its error word into the caller's pinned host words
// (one thread; every earlier kernel of the cloud has finished by then).
__global__ void k_publish(const unsigned long long *__restrict__ totals, const uint32_t *__restrict__ errw,
                          const uint32_t *__restrict__ errw2, unsigned long long *__restrict__ host) {
    if (threadIdx.x == 0) {
        for (int k = 0; k < 4; ++k) host[k] = totals[k];
        host[4] = *errw | *errw2;
    }
}

inline unsigned nblk(int64_t n, int tb = TB) { return (unsigned)((n + tb - 1) / tb); }

// One thread per block of the blocked tree copy (see tree_block_base).
__global__ void __launch_bounds__(TB) k_tree_blocks(const float *__restrict__ T, int D, int64_t nblocks,
                                                    float4 *__restrict__ tb) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblocks) return;
    int r = D & 3;
    while (r + 4 <= D - 4 && (uint64_t)b >= tree_block_base(r + 4, D)) r += 4;
    const int64_t i = ((int64_t)1 << r) - 1 + (b - (int64_t)tree_block_base(r, D));
    float v[16];
    v[0] = T[i];
    v[1] = T[2 * i + 1];
    v[2] = T[2 * i + 2];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[3 + k] = T[4 * i + 3 + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[7 + k] = T[8 * i + 7 + k];
    v[15] = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) tb[4 * b + k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Per-cloud scratch kept from the count phase to the fill phase.
struct CloudWork {
    Scratch scratch;
    uint32_t *rad = nullptr;       // radix sort scratch; rad[0] = error word
    uint32_t *rad_g = nullptr;     // the grid branch's radix scratch; rad_g[0] = its error word
    uint32_t *count = nullptr;     // entries per leaf
    uint32_t *pstart = nullptr;    // exclusive scan of padded counts
    uint32_t *scan_tmp = nullptr;
    unsigned long long *totals = nullptr;   // [0] entries [1] padded [2] pruned [3] non-finite
    AffArgs args{};
};

capt_status build_phase1(const float *xyz, int64_t n, float r_min, float r_max, uint32_t flags,
                         const uint8_t *axes, int shard_bits, int shard, hipStream_t s, CloudHost &C,
                         CloudWork &W, bool fork_grid) {
    int64_t N = 1;
    int D = 0;
    while (N < n) {
        N <<= 1;
        ++D;
    }
    if (D > 30) {
        set_error("cloud of %lld points exceeds 2^30", (long long)n);
        return CAPT_EUNSUPPORTED;
    }
    C.n = n;
    C.N = N;
    C.D = D;
    // fixed per-cloud block: T, leaves, points, rep, pruned flags
    const size_t oT = 0;
    const size_t oLeaf = align256(oT + sizeof(float) * (size_t)(N > 1 ? N - 1 : 1));
    const size_t oPts = align256(oLeaf + sizeof(Leaf) * (size_t)N);
    const size_t oRep = align256(oPts + sizeof(float) * 3 * (size_t)(n > 0 ? n : 1));
    const size_t oPr = align256(oRep + sizeof(int32_t) * (size_t)N);
    const size_t oTb = align256(oPr + (size_t)N);
    const size_t fixed_bytes = align256(oTb + sizeof(float4) * 4 * (size_t)tree_blocks_count(D));
    C.fixed = dev_alloc(fixed_bytes, s);
    if (!C.fixed) {
        set_error("device allocation of %zu bytes failed", fixed_bytes);
        return CAPT_ENOMEM;
    }
    C.fixed_bytes = fixed_bytes;
    char *F = static_cast<char *>(C.fixed);
    float *T = reinterpret_cast<float *>(F + oT);
    C.dev.T = T;
    C.dev.leaf = reinterpret_cast<Leaf *>(F + oLeaf);
    float *pts = reinterpret_cast<float *>(F + oPts);
    C.dev.pts = pts;
    C.rep = reinterpret_cast<int32_t *>(F + oRep);
    C.pruned_flag = reinterpret_cast<uint8_t *>(F + oPr);
    C.dev.tb = tree_blocks_count(D) > 0 ? reinterpret_cast<float4 *>(F + oTb) : nullptr;
    C.dev.n = n;
    C.dev.D = D;
    C.dev.flags = flags;
    C.dev.axes = axes_code(axes, D);
    C.dev.cyclic = C.dev.axes == axes_code(nullptr, D) ? 1 : 0;
    const uint64_t ax = C.dev.axes;

    // scratch
    const size_t wN = (size_t)N;
    const size_t wn = (size_t)std::max<int64_t>(n, 1);
    const int64_t cell_cap = std::max<int64_t>(4096, 4 * n);
    int cell_bits = 1;
    while (((int64_t)1 << cell_bits) < cell_cap) ++cell_bits;
    const size_t ntile = (size_t)((N + GTILE - 1) / GTILE);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t oL = take(sizeof(uint32_t) * 6 * wN);     // 3 lists x 2 buffers
    const size_t oK = take(sizeof(uint32_t) * 2 * 3 * wN);   // presort keys x 2
    const size_t oKg = take(sizeof(uint32_t) * 2 * wn);      // grid sort keys x 2
    const size_t oV = take(sizeof(uint32_t) * 2 * wn);       // grid sort values x 2
    const size_t oInv = take(sizeof(uint32_t) * wN);
    const size_t oLeft = take(2 * wN);   // "goes left" flags, two levels
    const int nglob = std::max(0, D - LMAX_LOG2);   // global levels (segments above LMAX)
    const size_t lvl_words = 2 * ntile + 64;          // per global level: two status lists, two counters
    const size_t oSums = take(sizeof(uint32_t) * (lvl_words * (size_t)std::max(nglob, 1) + 64));
    const size_t oRad = take(sizeof(uint32_t) * radix_tmp_words_seg(3, N));
    const size_t oRadG = take(sizeof(uint32_t) * radix_tmp_words(std::max<int64_t>(n, 1)));
    const size_t oCells = take(sizeof(float) * 6 * wN);
    const size_t oCnt = take(sizeof(uint32_t) * (wN + 1));
    const size_t oPs = take(sizeof(uint32_t) * (wN + 1));
    const size_t oTot = take(sizeof(unsigned long long) * 4);
    const int64_t nbN = (int64_t)nblk(N);   // blocks of the per-point / per-leaf kernels
    const size_t oPart = take((sizeof(float) * 6 + sizeof(uint32_t) * 2 + sizeof(unsigned long long) * 2) * nbN);
    const size_t nscan_cs = scan_lb_words(cell_cap + 1), nscan_ps = scan_lb_words(N);
    const size_t oScan = take(sizeof(uint32_t) * (nscan_cs + nscan_ps));   // look-back words of the two scans
    const size_t oGrid = take(sizeof(Grid) + 64);
    const size_t oCs = take(sizeof(uint32_t) * ((size_t)cell_cap + 1));
    const size_t oS = take(sizeof(float) * 3 * wn);
    if (!W.scratch.alloc(off, s)) {
        set_error("device allocation of %zu scratch bytes failed", off);
        return CAPT_ENOMEM;
    }
    char *Sb = W.scratch.as<char>();
    uint32_t *Lbuf = reinterpret_cast<uint32_t *>(Sb + oL);
    uint32_t *keys = reinterpret_cast<uint32_t *>(Sb + oK);
    uint32_t *gkeys = reinterpret_cast<uint32_t *>(Sb + oKg);
    uint32_t *gval = reinterpret_cast<uint32_t *>(Sb + oV);
    uint32_t *inv = reinterpret_cast<uint32_t *>(Sb + oInv);
    uint8_t *left = reinterpret_cast<uint8_t *>(Sb + oLeft);
    uint32_t *sums = reinterpret_cast<uint32_t *>(Sb + oSums);
    uint32_t *rad = reinterpret_cast<uint32_t *>(Sb + oRad);
    uint32_t *rad_g = reinterpret_cast<uint32_t *>(Sb + oRadG);
    W.rad = rad;
    W.rad_g = rad_g;
    float *cells = reinterpret_cast<float *>(Sb + oCells);
    W.count = reinterpret_cast<uint32_t *>(Sb + oCnt);
    W.pstart = reinterpret_cast<uint32_t *>(Sb + oPs);
    W.totals = reinterpret_cast<unsigned long long *>(Sb + oTot);
    W.scan_tmp = reinterpret_cast<uint32_t *>(Sb + oScan);
    Grid *grid = reinterpret_cast<Grid *>(Sb + oGrid);
    uint32_t *cstart = reinterpret_cast<uint32_t *>(Sb + oCs);
    float *sxyz = reinterpret_cast<float *>(Sb + oS);
    unsigned long long *pad_part = reinterpret_cast<unsigned long long *>(Sb + oPart);   // [nbN][2]
    float *bbp = reinterpret_cast<float *>(pad_part + 2 * nbN);                          // [nbN][6]
    uint32_t *badp = reinterpret_cast<uint32_t *>(bbp + 6 * nbN);                         // [nbN]
    uint32_t *prp = badp + nbN;                                                           // [nbN]
    // one clearing launch for the build's scratch: both sorts skip their own
    const int64_t clr_pre = radix_clear_words(3, N, 32), clr_grid = radix_clear_words(1, n, cell_bits);
    const int64_t clr_lvl = (N >> 0) > LMAX ? (int64_t)(lvl_words * (size_t)nglob) : 0;
    hipLaunchKernelGGL(k_binit, dim3((unsigned)std::min<int64_t>((cell_cap + TB) / TB + 1, 1024)), dim3(TB), 0, s,
                       W.totals, rad, rad_g, cstart, cell_cap + 1, W.scan_tmp, (int64_t)(nscan_cs + nscan_ps),
                       clr_pre, clr_grid, sums, clr_lvl);
    CAPT_LAUNCH_CHECK();

    // 1. presort: list a sorted by (coordinate a, id), the three lists in
    //    one segmented sort (buffer b holds the three lists back to back)
    uint32_t *L[3][2];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 2; ++b) L[a][b] = Lbuf + (size_t)(3 * b + a) * wN;
    int cur[3] = {0, 0, 0};
    hipLaunchKernelGGL(k_presort_keys, dim3(nblk(N)), dim3(TB), 0, s, xyz, n, N, keys, L[0][0], pts, bbp, badp);
    CAPT_LAUNCH_CHECK();

    // The grid of the points (step 4) needs only the points and the box
    // partials: it runs on a side stream while the splits run on s, and s
    // waits for it before the affordance sets.
    const double R = (double)r_max * (1.0 + 0x1p-20);
    // (A build of several clouds already runs clouds side by side on several
    // streams: there the branch stays on s, which saves its fork and join.)
    ForkJoin fj;
    if (fork_grid) {
        capt_status fs0 = fj.fork(s);
        if (fs0) return fs0;
    }
    const hipStream_t sg = fork_grid ? fj.side : s;
    capt_status fs = CAPT_OK;

    {
        int where = 0;
        capt_status st = radix_sort_u32_seg(keys, L[0][0], keys + 3 * wN, L[0][1], 3, N, 32, rad, s, &where, true);
        if (st) return st;
        cur[0] = cur[1] = cur[2] = where;
    }

    // the grid branch's launches follow the presort's, so the split chain starts first
    hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(TB), 0, sg, bbp, badp, nbN, R, cell_cap, grid, W.totals);
    CAPT_LAUNCH_CHECK();
    if (n > 0) {
        hipLaunchKernelGGL(k_grid_keys, dim3(nblk(n)), dim3(TB), 0, sg, xyz, n, grid, gkeys, gval, cstart);
        CAPT_LAUNCH_CHECK();
    }
    // bin starts: exclusive scan over the cap; cstart[ncells .. cap] = n
    fs = scan_exclusive_u32_lb(cstart, cstart, cell_cap + 1, W.scan_tmp, rad_g, sg);
    if (fs) return fs;
    int gwhere = 0;
    if (n > 1) {
        fs = radix_sort_u32(gkeys, gval, gkeys + wn, gval + wn, n, cell_bits, rad_g, sg, &gwhere, true);
        if (fs) return fs;
    }
    const uint32_t *sid = gwhere ? gval + wn : gval;
    if (n > 0) {
        hipLaunchKernelGGL(k_grid_gather, dim3(nblk(n)), dim3(TB), 0, sg, xyz, sid, n, sxyz, sxyz + wn,
                           sxyz + 2 * wn);
        CAPT_LAUNCH_CHECK();
    }


    // 2. splits: global levels while segments exceed LMAX, then LDS levels
    int d = 0;
    if ((N >> d) > LMAX) {   // (the level status words were cleared with the rest of the scratch)
        const int a0 = axis_at(ax, 0);
        hipLaunchKernelGGL(k_glevel_split, dim3(nblk(N)), dim3(TB), 0, s, L[a0][cur[a0]], xyz, n, N, 0, a0, T, left);
        CAPT_LAUNCH_CHECK();
    }
    uint8_t *lf_cur = left, *lf_next = left + wN;
    for (; d < D && (N >> d) > LMAX; ++d) {
        // the two lists off the split axis a are partitioned; the list on a
        // is in order for both halves already
        const int a = axis_at(ax, d);
        const int an = d + 1 < D ? axis_at(ax, d + 1) : (a + 1) % 3;
        const int b1 = an != a ? an : (a + 1) % 3;
        const int b2 = 3 - a - b1;
        const int64_t nt = N / GTILE;
        uint32_t *lv = sums + lvl_words * (size_t)d;
        const int next = (N >> (d + 1)) > LMAX ? 1 : 0;
        const int fused = next && an != a;   // level d + 1 written while scattering its list
        hipLaunchKernelGGL(k_glevel, dim3((unsigned)nt, 2), dim3(TB), 0, s, L[b1][cur[b1]], L[b2][cur[b2]],
                           L[b1][cur[b1] ^ 1], L[b2][cur[b2] ^ 1], lf_cur, lf_next, xyz, n, N, d, fused, an, T,
                           lv, lv + 2 * nt, nt, rad);
        CAPT_LAUNCH_CHECK();
        cur[b1] ^= 1;
        cur[b2] ^= 1;
        if (next && !fused) {   // level d + 1 splits on axis a again: from its list as it stands
            hipLaunchKernelGGL(k_glevel_split, dim3(nblk(N)), dim3(TB), 0, s, L[a][cur[a]], xyz, n, N, d + 1, a, T,
                               lf_next);
            CAPT_LAUNCH_CHECK();
        }
        std::swap(lf_cur, lf_next);
    }
    hipLaunchKernelGGL(k_inverse, dim3(nblk(N)), dim3(TB), 0, s, L[0][cur[0]], N, inv);
    CAPT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_local_levels, dim3(1u << d), dim3(LTB), 0, s, L[0][cur[0]], L[1][cur[1]], L[2][cur[2]],
                       inv, xyz, n, N, D, d, ax, T, C.rep);
    CAPT_LAUNCH_CHECK();
    {
        capt_status tbs = tree_blocks(T, D, const_cast<float4 *>(C.dev.tb), s);
        if (tbs) return tbs;
    }

    // 3. leaf cells and pruning
    const int prune = (!(flags & CAPT_NO_PRUNE) && r_min > 0.0f) ? 1 : 0;
    const double thr = ((double)r_min * (double)r_min) * (1.0 - 0x1p-18);
    // leaves of the shard: floor(l 2^bits / N) = shard
    const int64_t l0 = ((int64_t)shard * N + ((int64_t)1 << shard_bits) - 1) >> shard_bits;
    const int64_t l1 = ((int64_t)(shard + 1) * N + ((int64_t)1 << shard_bits) - 1) >> shard_bits;
    hipLaunchKernelGGL(k_cells_prune, dim3(nblk(N)), dim3(TB), 0, s, T, N, D, ax, cells, C.rep, xyz, n, prune, thr,
                       l0, l1, C.pruned_flag, prp);
    CAPT_LAUNCH_CHECK();

    // 4. join the grid branch (bins of side >= R / 2, points sorted by bin)
    fs = fj.join(s);
    if (fs) return fs;

    // 5. affordance counts and placement
    AffArgs &A = W.args;
    A.cells = cells;
    A.rep = C.rep;
    A.pruned = C.pruned_flag;
    A.xyz = xyz;
    A.grid = grid;
    A.cstart = cstart;
    A.sx = sxyz;
    A.sy = sxyz + wn;
    A.sz = sxyz + 2 * wn;
    A.sid = sid;
    A.n = n;
    A.N = N;
    A.l0 = l0;
    A.l1 = l1;
    A.R = R;
    A.R2 = R * R;
    {
        // the float32 pre-test's band, rounded outward to float
        const double lo = A.R2 * (1.0 - 0x1p-21), hi = A.R2 * (1.0 + 0x1p-21);
        float flo = (float)lo, fhi = (float)hi;
        if ((double)flo > lo) flo = std::nextafter(flo, 0.0f);
        if ((double)fhi < hi) fhi = std::nextafter(fhi, INFINITY);
        A.R2lo = flo;
        A.R2hi = fhi;
        A.pre32 = (A.R2 >= 1e-30 && A.R2 <= 1e30) ? 1 : 0;
    }
    hipLaunchKernelGGL((k_afford_grid<false>), dim3(nblk(N, 4 * LPW)), dim3(256), 0, s, A, W.count, nullptr, nullptr,
                       nullptr, nullptr, nullptr, const_cast<Leaf *>(C.dev.leaf), nullptr);
    CAPT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_pad_counts, dim3(nblk(N)), dim3(TB), 0, s, W.count, N, W.pstart, pad_part);
    CAPT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(TB), 0, s, pad_part, prp, nbN, W.totals);
    CAPT_LAUNCH_CHECK();
    return scan_exclusive_u32_lb(W.pstart, W.pstart, N, W.scan_tmp + nscan_cs, rad, s);
}

capt_status build_phase2(hipStream_t s, CloudHost &C, CloudWork &W, const unsigned long long tot[4]) {
    C.set_total = (int64_t)tot[0];
    C.set_padded = (int64_t)tot[1];
    C.pruned = (int64_t)tot[2];
    if (tot[1] >= MAX_SET_ENTRIES) {
        set_error("affordance sets hold %llu entries, more than 2^30", tot[1]);
        return CAPT_EUNSUPPORTED;
    }
    const size_t E = (size_t)(tot[1] > 0 ? tot[1] : CHUNK);
    const bool indexed = (C.dev.flags & CAPT_INDEXED_SETS) != 0;
    const size_t bytes = sets_bytes(E, indexed);
    C.sets = dev_alloc(bytes, s);
    if (!C.sets) {
        set_error("device allocation of %zu bytes for affordance sets failed", bytes);
        return CAPT_ENOMEM;
    }
    C.sets_bytes = bytes;
    float *px, *py, *pz;
    int32_t *pidx;
    uint4 *cbox;
    sets_layout(C.sets, E, indexed, &px, &py, &pz, &pidx, &cbox);
    C.dev.px = px;
    C.dev.py = py;
    C.dev.pz = pz;
    C.dev.pidx = pidx;
    C.dev.cbox = cbox;
    hipLaunchKernelGGL((k_afford_grid<true>), dim3(nblk(C.N, 4 * LPW)), dim3(256), 0, s, W.args, nullptr, W.pstart, px,
                       py, pz, pidx, const_cast<Leaf *>(C.dev.leaf), cbox);
    CAPT_LAUNCH_CHECK();
    return CAPT_OK;
}

}  // namespace

void free_cloud(CloudHost &c, hipStream_t s) {
    if (c.fixed) dev_free(c.fixed, s);
    if (c.sets) dev_free(c.sets, s);
    c.fixed = c.sets = nullptr;
}

capt_status upload_views(capt_forest_s *f, hipStream_t s) {
    const size_t bytes = sizeof(CloudDev) * f->clouds.size();
    f->d_clouds = static_cast<CloudDev *>(dev_alloc(bytes, s));
    if (!f->d_clouds) {
        set_error("device allocation of %zu bytes failed", bytes);
        return CAPT_ENOMEM;
    }
    std::vector<CloudDev> h(f->clouds.size());
    for (size_t c = 0; c < h.size(); ++c) h[c] = f->clouds[c].dev;
    CAPT_HIP(hipMemcpyAsync(f->d_clouds, h.data(), bytes, hipMemcpyHostToDevice, s));
    CAPT_HIP(hipStreamSynchronize(s));
    return CAPT_OK;
}

capt_status build_forest(const float *xyz, const int64_t *cloud_off, int32_t ncloud, float r_min,
                         float r_max, uint32_t flags, const uint8_t *axes, int shard_bits, int shard,
                         hipStream_t s, capt_forest_s *f) {
    f->clouds.resize(ncloud);
    f->r_min = r_min;
    f->r_max = r_max;
    f->flags = flags;
    std::vector<CloudWork> work(ncloud);
    // Several clouds are built on BUILD_STREAMS streams forked from the
    // caller's (cloud c on stream c % BUILD_STREAMS), so the many small kernels
    // of small clouds run side by side instead of one after the other.
    const int nst = std::max(1, std::min<int>(ncloud, BUILD_STREAMS));
    std::vector<ForkJoin> fj(nst);
    std::vector<hipStream_t> ws(nst, s);
    for (int i = 1; i < nst; ++i) {
        capt_status st = fj[i].fork(s);
        if (st) return st;
        ws[i] = fj[i].side;
    }
    // The clouds are issued by two host threads (cloud c by thread c % 2; the
    // launch chains of many small clouds are host-bound, and the runtime
    // serialises launches across threads, so more threads only contend),
    // unless the caller's allocator hooks are installed: those need not be
    // thread-safe.
    const int nth = default_allocator() ? std::min(nst, 2) : 1;
    std::vector<capt_status> th_st(nth, CAPT_OK);
    std::vector<std::string> th_msg(nth);
    int dev = 0;
    CAPT_HIP(hipGetDevice(&dev));
    auto issue = [&](int t, auto &&per_cloud) {
        if (t > 0 && hipSetDevice(dev) != hipSuccess) {
            th_st[t] = CAPT_EHIP;
            th_msg[t] = "hipSetDevice failed in a build thread";
            return;
        }
        for (int c = t; c < ncloud; c += nth) {
            const capt_status st = per_cloud(c);
            if (st) {
                th_st[t] = st;
                th_msg[t] = capt_last_error();
                return;
            }
        }
    };
    auto in_threads = [&](auto &&per_cloud) -> capt_status {
        std::vector<std::thread> th;
        for (int t = 1; t < nth; ++t) th.emplace_back([&, t] { issue(t, per_cloud); });
        issue(0, per_cloud);
        for (auto &x : th) x.join();
        for (int t = 0; t < nth; ++t)
            if (th_st[t]) {
                set_error("%s", th_msg[t].c_str());
                return th_st[t];
            }
        return CAPT_OK;
    };
    {
        capt_status st = in_threads([&](int c) {
            const int64_t n = cloud_off[c + 1] - cloud_off[c];
            return build_phase1(xyz + 3 * cloud_off[c], n, r_min, r_max, flags, axes, shard_bits, shard, ws[c % nst],
                                f->clouds[c], work[c], ncloud == 1);
        });
        if (st) return st;
    }
    // every cloud's totals and error word straight into pinned host memory,
    // then one wait
    Pinned res;
    if (!res.alloc(sizeof(unsigned long long) * 5 * (size_t)ncloud)) {
        set_error("pinned host allocation failed");
        return CAPT_ENOMEM;
    }
    unsigned long long *hw = res.as<unsigned long long>();
    for (int c = 0; c < ncloud; ++c) {
        hipLaunchKernelGGL(k_publish, dim3(1), dim3(WAVE), 0, ws[c % nst], work[c].totals, work[c].rad,
                           work[c].rad_g, hw + 5 * c);
        CAPT_LAUNCH_CHECK();
    }
    for (int i = 0; i < nst; ++i) {
        const hipError_t se = hipStreamSynchronize(ws[i]);
        if (se != hipSuccess) {
            res.p = nullptr;   // the kernels' state is unknown: never hand the block out again
            return hip_fail(se, "hipStreamSynchronize", __FILE__, __LINE__);
        }
    }
    std::vector<unsigned long long> tot(4 * (size_t)ncloud);
    std::vector<unsigned long long> sort_err((size_t)ncloud);
    for (int c = 0; c < ncloud; ++c) {
        for (int k = 0; k < 4; ++k) tot[4 * c + k] = hw[5 * c + k];
        sort_err[c] = hw[5 * c + 4];
    }
    for (int c = 0; c < ncloud; ++c)
        if (sort_err[c]) {
            set_error("internal: radix sort look-back bound exceeded while building cloud %d", c);
            return CAPT_EHIP;
        }
    for (int c = 0; c < ncloud; ++c) {
        const uint32_t bad = (uint32_t)(tot[4 * c + 3] & 0xFFFFFFFFull);
        if (bad) {
            set_error("cloud %d holds %u non-finite coordinates", c, bad);
            return CAPT_EINVAL;
        }
    }
    {
        capt_status st = in_threads([&](int c) { return build_phase2(ws[c % nst], f->clouds[c], work[c], &tot[4 * c]); });
        if (st) return st;
    }
    int64_t pruned = 0;
    for (int c = 0; c < ncloud; ++c) pruned += f->clouds[c].pruned;
    f->pruned_total = pruned;
    for (int i = 1; i < nst; ++i) {
        capt_status st = fj[i].join(s);
        if (st) return st;
    }
    return CAPT_OK;   // scratch is released stream-ordered; the forest is ready in stream order
}


size_t sets_bytes(size_t E, bool indexed) {
    return (indexed ? 0 : align256(sizeof(float) * 3 * E)) + align256(sizeof(int32_t) * E) +
           align256(sizeof(uint4) * (E / CHUNK + 1));
}

// E (a multiple of CHUNK) entries: the interleaved coordinate blocks (not for
// indexed sets), the indices, the chunk boxes.
void sets_layout(void *base, size_t E, bool indexed, float **px, float **py, float **pz, int32_t **pidx,
                 uint4 **cbox) {
    char *P = static_cast<char *>(base);
    const size_t a = indexed ? 0 : align256(sizeof(float) * 3 * E);
    float *b = indexed ? nullptr : reinterpret_cast<float *>(P);
    *px = b;
    *py = b ? b + CHUNK : nullptr;
    *pz = b ? b + 2 * CHUNK : nullptr;
    *pidx = reinterpret_cast<int32_t *>(P + a);
    *cbox = reinterpret_cast<uint4 *>(P + a + align256(sizeof(int32_t) * E));
}


capt_status tree_blocks(const float *T, int D, float4 *tb, hipStream_t s) {
    const int64_t nb = tree_blocks_count(D);
    if (nb <= 0 || !tb) return CAPT_OK;
    hipLaunchKernelGGL(k_tree_blocks, dim3(nblk(nb)), dim3(TB), 0, s, T, D, nb, tb);
    CAPT_LAUNCH_CHECK();
    return CAPT_OK;
}

capt_status ensure_views(capt_forest_s *f, hipStream_t s) {
    if (f->d_clouds) return CAPT_OK;
    return upload_views(f, s);
}

}  // namespace capt
