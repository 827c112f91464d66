// Morton-curve point-cloud filter (Alg. 2, Sec. IV-C) on the GPU.
//
// Six passes, one per axis permutation, each on the previous pass's
// survivors, in the order of a stable sort of the current list along the
// pass's Z-order curve (63-bit keys on a 2^21-per-axis grid over the input's
// cubic bounding box).  Two facts let every sort happen up front:
//  * every permutation's key is a bijection of the grid cell, so two points
//    tie under one permutation exactly when they tie under all of them; the
//    stable order of pass p is therefore "key_p, then original index" whatever
//    the earlier passes did;
//  * the survivors of a pass, taken in that order, are the full sorted list
//    with the dead points skipped.
// So one segmented radix sort orders all n points under all six keys, and
// pass p walks segment p with a liveness flag per point.
//
// A pass makes the sequential rule "keep j iff it is farther than r_filter
// from the last kept point" parallel: next[j] = the first live k > j farther
// than r_filter from j (for a dead j: the first live k > j), so the kept
// points are the live nodes of the chain 0 -> next[0] -> ...  One kernel
// resolves the chain in chunks of CC positions: a chunk builds the jump
// tables J_t = next^(2^t) of its positions in LDS, waits for the previous
// chunk to publish where the chain enters it, follows the tables to the
// chain's exit and publishes that for the next chunk; it then marks the
// chain's nodes inside the chunk top-down over the tables and writes the
// next pass's liveness flags.  The last pass also writes its survivors in
// order, at offsets found by decoupled look-back over earlier chunks' counts.
// Only the final count crosses to the host.
#include <algorithm>
#include <cmath>

#include "capt_internal.h"
#include "lookback.h"

namespace capt {

namespace {

constexpr int TB = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + TB - 1) / TB); }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct FState {
    float lo[3];
    float hi[3];
    double scale;
    int64_t mm[2];      // mm[0]: survivors of the last pass (n until it ends)
    unsigned int bad;   // non-finite coordinates
};

constexpr int BB_BLOCKS = 64;   // partial bounding boxes

// Scratch that must start at zero or one: the publication words of the six
// chain passes, the sort's error words, the liveness flags before pass 0.
__global__ void k_finit(uint32_t *__restrict__ pub, int64_t npub, uint32_t *__restrict__ errw,
                        uint8_t *__restrict__ live, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t; i < npub; i += stride) pub[i] = 0u;
    for (int64_t i = t; i < 64; i += stride) errw[i] = 0u;
    for (int64_t i = t; i < n; i += stride) live[i] = 1u;
}

// Per-block bounding box of the finite coordinates and count of non-finite
// ones; part[b] = {lo[3], hi[3]}, bad[b].
__global__ void k_bbox(const float *__restrict__ xyz, int64_t n, float *__restrict__ part,
                       unsigned int *__restrict__ badp) {
    __shared__ float sl[TB / WAVE][6];
    __shared__ unsigned int sb[TB / WAVE];
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
    for (int off = WAVE / 2; off >= 1; off >>= 1) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], off, WAVE));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off, WAVE));
        }
        bad += (unsigned int)__shfl_xor((int)bad, off, WAVE);
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
        part[6 * blockIdx.x + threadIdx.x] = v;
    }
    if (threadIdx.x == 0) {
        unsigned int t = 0;
        for (int i = 0; i < TB / WAVE; ++i) t += sb[i];
        badp[blockIdx.x] = t;
    }
}

// Reduce the partial boxes; set the grid (cell = largest extent / 2^21) and
// the rest of the state.  One wave.
__global__ void k_grid(const float *__restrict__ part, const unsigned int *__restrict__ badp, int nb, int64_t n,
                       FState *st) {
    const int lane = threadIdx.x;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    unsigned int bad = 0;
    if (lane < nb) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = part[6 * lane + a];
            hi[a] = part[6 * lane + 3 + a];
        }
        bad = badp[lane];
    }
    for (int off = WAVE / 2; off >= 1; off >>= 1) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], off, WAVE));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off, WAVE));
        }
        bad += (unsigned int)__shfl_xor((int)bad, off, WAVE);
    }
    if (lane != 0) return;
    double E = 0.0;
    for (int a = 0; a < 3; ++a) {
        st->lo[a] = lo[a];   // the sign of a zero minimum does not change any cell coordinate
        st->hi[a] = hi[a];
        const double e = __dsub_rn((double)hi[a], (double)lo[a]);
        if (e > E) E = e;
    }
    st->scale = E > 0.0 ? 2097152.0 / E : 0.0;
    st->mm[0] = n;
    st->mm[1] = 0;
    st->bad = bad;
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

// All six keys of every point: keys[p * n + id], vals[p * n + id] = id.
__global__ void k_morton6(const float *__restrict__ xyz, int64_t n, const FState *__restrict__ st,
                          uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    uint64_t sp[3];
    for (int a = 0; a < 3; ++a) sp[a] = spread3(cell_of(xyz[3 * j + a], st->lo[a], st->scale));
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        // axis X[i] of the permutation fills key bits 3b + (2 - i)
        keys[p * n + j] = (sp[c_perm[p][0]] << 2) | (sp[c_perm[p][1]] << 1) | sp[c_perm[p][2]];
        vals[p * n + j] = (uint32_t)j;
    }
}

// The chain kernel takes one position per thread; a chunk is CT positions
// (256, or 512 for large clouds, where fewer chunks shorten the look-back; at
// 1024 a block's LDS and waves let fewer chunks run at once).
constexpr int CI = 1;                // positions per thread
constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
// Positions past the chunk whose point is staged in LDS with the chunk's own:
// next-pointer searches rarely run further (beyond, they read global memory).
constexpr int STAGE_EXT = 64;
// dynamic LDS of the chain kernel: the staged positions' x, y, z (f32) and
// point id (u32) [CC + STAGE_EXT] each, J [CR][CC] u16, Nx [CC] u32, Ex [CC]
// u32, Cu [CC] u16, mark [CC] i8, the staged liveness flags [CC + STAGE_EXT] u8
constexpr size_t chain_lds(int CC) {
    return 4 * sizeof(uint32_t) * (CC + STAGE_EXT) + sizeof(uint16_t) * ilog2c(CC) * CC + 2 * sizeof(uint32_t) * CC +
           sizeof(uint16_t) * CC + CC + (CC + STAGE_EXT);
}
constexpr uint16_t OUTL = 0xFFFF;    // "leaves the chunk"
// A next pointer is searched for at most SCAN_BOUND positions ahead; beyond
// that it is left unresolved (UNRES) and found only if the chain reaches its
// position, by one wavefront scanning on from there.  Every position's own
// search is then bounded, and the scans for chain nodes cover disjoint ranges
// of the curve, so a pass stays linear in n whatever runs of coincident or
// near-coincident points the cloud holds.
constexpr int SCAN_BOUND = 1024;
constexpr uint32_t UNRES = 0xFFFFFFFFu;
constexpr uint32_t PUB = 0x80000000u;
constexpr uint32_t MX_AGG = 0x40000000u;   // farthest reach: this chunk's own (positions < 2^30)
constexpr uint32_t MX_PRE = 0x80000000u;   // farthest reach of chunks 0 .. c
constexpr uint32_t MX_FLAGS = 0xC0000000u;
constexpr uint32_t SPIN_LIMIT = 1u << 20;

__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The next pointer of position j by a wavefront scan from position `from`:
// the first live position k >= from farther than r_filter from j when j is
// live, the first live k >= from when j is dead; n when there is none.  All 64
// lanes of the wavefront call it together.
__device__ uint32_t scan_next(const float *__restrict__ xyz, const uint32_t *__restrict__ ord, int64_t n,
                              const uint8_t *__restrict__ live_in, float rf2, int64_t j, int64_t from) {
    const int lane = threadIdx.x & (WAVE - 1);
    const uint32_t a = ord[j];
    const bool lj = live_in[a] != 0;
    const float ax = xyz[3 * (int64_t)a], ay = xyz[3 * (int64_t)a + 1], az = xyz[3 * (int64_t)a + 2];
    for (int64_t base = from; base < n; base += WAVE) {
        const int64_t k = base + lane;
        bool ok = false;
        if (k < n) {
            const uint32_t b = ord[k];
            if (live_in[b])
                ok = !lj || sqdist(ax, ay, az, xyz[3 * (int64_t)b], xyz[3 * (int64_t)b + 1], xyz[3 * (int64_t)b + 2]) > rf2;
        }
        const uint64_t bal = __ballot(ok);
        if (bal) return (uint32_t)(base + __builtin_ctzll(bal));
    }
    return (uint32_t)n;
}

template <int CT>
__device__ __forceinline__ uint32_t block_excl_scan_c(uint32_t v, uint32_t *lw, uint32_t *total) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const uint32_t t = __shfl_up(inc, d, WAVE);
        if (lane >= d) inc += t;
    }
    if (lane == WAVE - 1) lw[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < CT / WAVE; ++i) {
        const uint32_t t = lw[i];
        off += (i < w) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// One filter pass (see the file comment).  ord: all n points in the pass's
// curve order (original ids); live_in / live_out: liveness per original id
// before / after the pass.  With `last`, the survivors also go to out in
// order and their count to st->mm[0].
template <int CT>
__global__ void __launch_bounds__(CT) k_filter_chain(const float *__restrict__ xyz, const uint32_t *__restrict__ ord,
                                                    int64_t n, const uint8_t *__restrict__ live_in,
                                                    uint8_t *__restrict__ live_out, FState *__restrict__ st,
                                                    float rf2, int last, uint32_t *__restrict__ exit_pub,
                                                    uint32_t *__restrict__ kept_st, uint32_t *__restrict__ max_pub,
                                                    uint32_t *__restrict__ chunk_ctr, uint32_t *__restrict__ out,
                                                    uint32_t *__restrict__ err) {
    constexpr int CC = CT * CI;          // chunk length
    constexpr int CR = ilog2c(CC);       // jump tables J_0 .. J_{CR-1}
    constexpr int SG = CC + STAGE_EXT;   // staged positions
    extern __shared__ uint32_t chain_mem[];
    float *Sx = reinterpret_cast<float *>(chain_mem);
    float *Sy = Sx + SG;
    float *Sz = Sy + SG;
    uint32_t *So = reinterpret_cast<uint32_t *>(Sz + SG);
    auto J = reinterpret_cast<uint16_t(*)[CC]>(So + SG);
    uint32_t *Nx = So + SG + CR * CC / 2;
    uint32_t *Ex = Nx + CC;
    uint16_t *Cu = reinterpret_cast<uint16_t *>(Ex + CC);
    int8_t *mark = reinterpret_cast<int8_t *>(Cu + CC);
    uint8_t *Sl = reinterpret_cast<uint8_t *>(mark + CC);
    __shared__ uint32_t s_chunk, s_entry, s_prefix, s_max;
    __shared__ uint32_t lw[CT / WAVE];
    if (threadIdx.x == 0) {
        s_chunk = atomicAdd(chunk_ctr, 1u);
        s_max = 0u;
    }
    __syncthreads();
    const int64_t c = s_chunk;
    const int64_t cs = c * CC;
    if (cs >= n) return;                      // uniform
    const int64_t ce = min(cs + (int64_t)CC, n);
    const int len = (int)(ce - cs);
    // 0. stage the point, id and liveness of positions [cs, cs + SG): one
    //    round of gathers instead of one per search step
    const int slen = (int)(min(cs + (int64_t)SG, n) - cs);
    for (int i = threadIdx.x; i < slen; i += CT) {
        const uint32_t b = ord[cs + i];
        So[i] = b;
        Sl[i] = live_in[b];
        Sx[i] = xyz[3 * (int64_t)b];
        Sy[i] = xyz[3 * (int64_t)b + 1];
        Sz[i] = xyz[3 * (int64_t)b + 2];
    }
    __syncthreads();
    // 1. next pointers (searched at most SCAN_BOUND positions ahead) and the
    //    first jump table
    for (int i = threadIdx.x; i < CC; i += CT) {
        if (i < len) {
            const int64_t j = cs + i;
            const int64_t kend = min(n, j + 1 + (int64_t)SCAN_BOUND);
            int64_t k = j + 1;
            if (Sl[i]) {
                const float ax = Sx[i], ay = Sy[i], az = Sz[i];
                for (; k < kend; ++k) {
                    const int64_t q = k - cs;
                    if (q < slen) {
                        if (Sl[q] && sqdist(ax, ay, az, Sx[q], Sy[q], Sz[q]) > rf2) break;
                    } else {
                        const uint32_t b = ord[k];
                        if (live_in[b] &&
                            sqdist(ax, ay, az, xyz[3 * (int64_t)b], xyz[3 * (int64_t)b + 1], xyz[3 * (int64_t)b + 2]) >
                                rf2)
                            break;
                    }
                }
            } else {
                while (k < kend && !(k - cs < slen ? Sl[k - cs] : live_in[ord[k]])) ++k;
            }
            const bool unres = k == kend && kend < n;
            Nx[i] = unres ? UNRES : (uint32_t)k;
            J[0][i] = k < ce ? (uint16_t)(k - cs) : OUTL;
            atomicMax(&s_max, unres ? (uint32_t)n : (uint32_t)k);   // an unresolved pointer reaches at most n
        } else {
            J[0][i] = OUTL;
        }
    }
    __syncthreads();
    // the farthest position a next pointer of this chunk reaches bounds where
    // the chain can enter later chunks: published at once as this chunk's own
    // value (MX_AGG), later as the running maximum over chunks 0 .. c (MX_PRE)
    const uint32_t own_max = s_max;
    if (threadIdx.x == 0) st_agent(&max_pub[c], (c == 0 ? MX_PRE : MX_AGG) | own_max);
    // 2. jump tables J_t = next^(2^t) inside the chunk
    for (int t = 1; t < CR; ++t) {
        for (int i = threadIdx.x; i < CC; i += CT) {
            const uint16_t v = J[t - 1][i];
            J[t][i] = v == OUTL ? OUTL : J[t - 1][v];
        }
        __syncthreads();
    }
    // 3. where the chain leaves the chunk from every entry position: its last
    //    node inside the chunk and that node's next pointer (maybe UNRES)
    for (int i = threadIdx.x; i < len; i += CT) {
        int cur = i;
        for (int t = CR - 1; t >= 0; --t)
            if (J[t][cur] != OUTL) cur = J[t][cur];
        Cu[i] = (uint16_t)cur;
        Ex[i] = Nx[cur];
    }
    // The chain enters this chunk at a position no later than M, the farthest
    // next pointer of the earlier chunks.  When every entry up to M leaves at
    // the same position (chains merge after a few nodes), that is the exit
    // whatever the earlier chunks do: publish it without waiting for them.
    // Otherwise wait for the previous chunk's exit.
    if (c > 0 && threadIdx.x < WAVE) {
        // decoupled look-back over the earlier chunks' maxima, 64 at a time
        const int lane = threadIdx.x;
        uint32_t m = 0;
        int64_t hi = c;   // chunks [0, hi) still to look at
        while (hi > 0) {
            const int64_t q = hi - 1 - lane;
            uint32_t v = MX_PRE;   // lanes past chunk 0: an empty inclusive maximum
            if (q >= 0) {
                uint32_t spins = 0;
                while (((v = ld_agent(&max_pub[q])) & MX_FLAGS) == 0) {
                    if (++spins > SPIN_LIMIT) {
                        atomicOr(err, 2u);
                        v = MX_PRE;
                        break;
                    }
                }
            }
            const uint64_t pre = __ballot((v & MX_FLAGS) == MX_PRE);
            const int stop = pre ? __builtin_ctzll(pre) : WAVE;   // nearest inclusive maximum
            if (lane <= stop) m = max(m, v & ~MX_FLAGS);
            if (pre) break;
            hi -= WAVE;
        }
        for (int off = WAVE / 2; off >= 1; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, WAVE));
        if (lane == 0) {
            st_agent(&max_pub[c], MX_PRE | max(m, own_max));
            s_max = m;
        }
    }
    __syncthreads();
    const int64_t M = c > 0 ? (int64_t)s_max : cs;
    bool same = M < ce && Ex[0] != UNRES;
    if (same)
        for (int i = threadIdx.x; i <= (int)(M - cs); i += CT) same = same && Ex[i] == Ex[0];
    const bool merged = __syncthreads_and(same) != 0;
    if (threadIdx.x < WAVE) {
        // the first wavefront waits for the entry and publishes the exit,
        // scanning on from the chunk's last chain node if its pointer is unresolved
        const int lane = threadIdx.x;
        if (merged && lane == 0) st_agent(&exit_pub[c], PUB | Ex[0]);
        uint32_t X = 0;
        if (c > 0 && lane == 0) {
            uint32_t v = 0, spins = 0;
            while (((v = ld_agent(&exit_pub[c - 1])) & PUB) == 0) {
                if (++spins > SPIN_LIMIT) {
                    atomicOr(err, 2u);
                    break;
                }
            }
            X = v & ~PUB;
        }
        X = (uint32_t)__shfl((int)X, 0, WAVE);
        if (!merged) {
            uint32_t E = (int64_t)X < ce ? Ex[X - cs] : X;
            if (E == UNRES) E = scan_next(xyz, ord, n, live_in, rf2, cs + Cu[X - cs], cs + Cu[X - cs] + 1);
            if (lane == 0) st_agent(&exit_pub[c], PUB | E);
        }
        if (lane == 0) s_entry = X;
    }
    for (int i = threadIdx.x; i < CC; i += CT) mark[i] = -1;
    __syncthreads();
    // 4. mark the chain inside the chunk, top-down over the tables
    const int64_t X = s_entry;
    if (X < ce) {
        if (threadIdx.x == 0) mark[X - cs] = (int8_t)CR;
        __syncthreads();
        for (int t = CR - 1; t >= 0; --t) {
            for (int i = threadIdx.x; i < len; i += CT)
                if (mark[i] > t) {
                    const uint16_t k = J[t][i];
                    if (k != OUTL) mark[k] = (int8_t)t;
                }
            __syncthreads();
        }
    }
    // 5. the pass's survivors: live chain nodes
    uint32_t f[CI];
    uint32_t cnt = 0;
#pragma unroll
    for (int u = 0; u < CI; ++u) {
        const int i = threadIdx.x * CI + u;
        f[u] = 0u;
        if (i < len) {
            f[u] = (mark[i] >= 0 && Sl[i]) ? 1u : 0u;
            live_out[So[i]] = (uint8_t)f[u];
        }
        cnt += f[u];
    }
    if (!last) return;
    uint32_t kept;
    uint32_t off = block_excl_scan_c<CT>(cnt, lw, &kept);
    // 6. offset of the chunk's survivors: look back over earlier chunks
    if (threadIdx.x < WAVE) {   // the first wavefront publishes and looks back
        uint32_t excl = 0;
        if (c == 0) {
            if (threadIdx.x == 0) st_agent(&kept_st[0], 0x80000000u | kept);
        } else {
            if (threadIdx.x == 0) st_agent(&kept_st[c], 0x40000000u | kept);
            excl = wave_lookback(kept_st, c, SPIN_LIMIT, err, 4u);
            if (threadIdx.x == 0) st_agent(&kept_st[c], 0x80000000u | (excl + kept));
        }
        if (threadIdx.x == 0) {
            s_prefix = excl;
            if (ce == n) st->mm[0] = (int64_t)(excl + kept);
        }
    }
    __syncthreads();
    off += s_prefix;
#pragma unroll
    for (int u = 0; u < CI; ++u) {
        const int i = threadIdx.x * CI + u;
        if (f[u]) out[off++] = So[i];
    }
}

// Gathers the survivors; the first thread also stores the survivor count,
// the non-finite count and the error word into the caller's pinned host
// words (every earlier kernel of the call has finished by then).
__global__ void k_output(const float *__restrict__ xyz, const uint32_t *__restrict__ cur, int64_t n,
                         const FState *__restrict__ st, const uint32_t *__restrict__ errw, float *__restrict__ out_xyz,
                         int32_t *__restrict__ out_index, const uint32_t *__restrict__ map,
                         unsigned long long *__restrict__ host) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) {
        host[0] = (unsigned long long)st->mm[0];
        host[1] = st->bad;
        host[2] = *errw;
    }
    if (j >= n || j >= st->mm[0]) return;
    const uint32_t id = cur[j];
    out_xyz[3 * j] = xyz[3 * (int64_t)id];
    out_xyz[3 * j + 1] = xyz[3 * (int64_t)id + 1];
    out_xyz[3 * j + 2] = xyz[3 * (int64_t)id + 2];
    if (out_index) out_index[j] = (int32_t)(map ? map[id] : id);
}

// Zero n words (the crop's counters and the scan's status words).
__global__ void k_zero_words(uint32_t *__restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

// Reach crop: flag[j] = 1 iff point j is finite and its float32 squared
// distance to the base is at most reach2; non-finite coordinates are counted
// into *bad (zeroed beforehand).
__global__ void k_crop_flag(const float *__restrict__ xyz, int64_t n, float bx, float by, float bz, float reach2,
                            uint32_t *__restrict__ flag, unsigned int *__restrict__ bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t j = t; j < n; j += stride) {
        const float x = xyz[3 * j], y = xyz[3 * j + 1], z = xyz[3 * j + 2];
        const unsigned int nb = (unsigned int)!isfinite(x) + (unsigned int)!isfinite(y) + (unsigned int)!isfinite(z);
        if (nb) atomicAdd(bad, nb);
        flag[j] = (nb == 0 && sqdist(x, y, z, bx, by, bz) <= reach2) ? 1u : 0u;
    }
}

// Stable compaction of the cropped points (pos = exclusive scan of flag);
// map[k] = input index of compacted point k.  The last thread stores the
// count, the non-finite count and the scan's error word into the caller's
// pinned host words.
__global__ void k_crop_compact(const float *__restrict__ xyz, int64_t n, const uint32_t *__restrict__ flag,
                               const uint32_t *__restrict__ pos, float *__restrict__ cxyz, uint32_t *__restrict__ map,
                               const unsigned int *__restrict__ bad, const uint32_t *__restrict__ errw,
                               unsigned long long *__restrict__ host) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t k = pos[j];
    if (flag[j]) {
        cxyz[3 * (int64_t)k] = xyz[3 * j];
        cxyz[3 * (int64_t)k + 1] = xyz[3 * j + 1];
        cxyz[3 * (int64_t)k + 2] = xyz[3 * j + 2];
        map[k] = (uint32_t)j;
    }
    if (j == n - 1) {
        host[0] = (unsigned long long)(k + flag[j]);
        host[1] = *bad;
        host[2] = *errw;
    }
}

}  // namespace

namespace {

capt_status filter_core(const float *xyz, int64_t n, float r_filter, const uint32_t *map, float *out_xyz,
                        int32_t *out_index, int64_t *n_out, hipStream_t s) {
    if (n == 0) {
        *n_out = 0;
        return CAPT_OK;
    }
    constexpr int NP = 6;
    const size_t wn = (size_t)n;
    // chunk length: 256 positions, or 512 once that would make more than 256 chunks
    const int CT = (n + 255) / 256 > 256 ? 512 : 256;
    const int64_t nchunk = (n + CT - 1) / CT;
    const int64_t npub = NP * (3 * nchunk + 64);   // per pass: exits, survivor counts, farthest reaches, counter
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t oSt = take(sizeof(FState));
    const size_t oCur = take(sizeof(uint32_t) * wn);
    const size_t oK0 = take(sizeof(uint64_t) * wn * NP);
    const size_t oK1 = take(sizeof(uint64_t) * wn * NP);
    const size_t oV0 = take(sizeof(uint32_t) * wn * NP);
    const size_t oV1 = take(sizeof(uint32_t) * wn * NP);
    const size_t oLive = take(wn * (NP + 1));
    const size_t oPub = take(sizeof(uint32_t) * (size_t)npub);
    const size_t oRad = take(sizeof(uint32_t) * radix_tmp_words_seg(NP, n));
    const size_t oBB = take(sizeof(float) * 6 * BB_BLOCKS + sizeof(unsigned int) * BB_BLOCKS);
    Scratch sc;
    if (!sc.alloc(off, s)) {
        set_error("device allocation of %zu filter scratch bytes failed", off);
        return CAPT_ENOMEM;
    }
    Pinned res;
    if (!res.alloc(3 * sizeof(unsigned long long))) {
        set_error("pinned host allocation failed");
        return CAPT_ENOMEM;
    }
    char *B = sc.as<char>();
    FState *st = reinterpret_cast<FState *>(B + oSt);
    uint32_t *cur = reinterpret_cast<uint32_t *>(B + oCur);
    uint64_t *k0 = reinterpret_cast<uint64_t *>(B + oK0);
    uint64_t *k1 = reinterpret_cast<uint64_t *>(B + oK1);
    uint32_t *v0 = reinterpret_cast<uint32_t *>(B + oV0);
    uint32_t *v1 = reinterpret_cast<uint32_t *>(B + oV1);
    uint8_t *live = reinterpret_cast<uint8_t *>(B + oLive);
    uint32_t *pub = reinterpret_cast<uint32_t *>(B + oPub);
    uint32_t *rad = reinterpret_cast<uint32_t *>(B + oRad);
    float *bbp = reinterpret_cast<float *>(B + oBB);
    unsigned int *bbbad = reinterpret_cast<unsigned int *>(bbp + 6 * BB_BLOCKS);

    const float rf2 = r_filter * r_filter;
    hipLaunchKernelGGL(k_finit, dim3((unsigned)std::min<int64_t>(std::max<int64_t>(npub, n) / TB + 1, 1024)), dim3(TB),
                       0, s, pub, npub, rad, live, n);
    CAPT_LAUNCH_CHECK();
    const int nbb = (int)std::min<int64_t>(nblk(n), BB_BLOCKS);
    hipLaunchKernelGGL(k_bbox, dim3((unsigned)nbb), dim3(TB), 0, s, xyz, n, bbp, bbbad);
    CAPT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_grid, dim3(1), dim3(WAVE), 0, s, bbp, bbbad, nbb, n, st);
    CAPT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_morton6, dim3(nblk(n)), dim3(TB), 0, s, xyz, n, st, k0, v0);
    CAPT_LAUNCH_CHECK();
    int where = 0;
    capt_status e = radix_sort_u64_seg(k0, v0, k1, v1, NP, n, 63, rad, s, &where);
    if (e) return e;
    const uint32_t *ord = where ? v1 : v0;
    for (int p = 0; p < NP; ++p) {
        uint32_t *pp = pub + (size_t)p * (3 * nchunk + 64);
        if (CT == 512)
            hipLaunchKernelGGL(k_filter_chain<512>, dim3((unsigned)nchunk), dim3(512), chain_lds(512), s, xyz,
                               ord + (size_t)p * wn, n, live + (size_t)p * wn, live + (size_t)(p + 1) * wn, st, rf2,
                               (int)(p == NP - 1), pp, pp + nchunk, pp + 2 * nchunk, pp + 3 * nchunk, cur, rad);
        else
            hipLaunchKernelGGL(k_filter_chain<256>, dim3((unsigned)nchunk), dim3(256), chain_lds(256), s, xyz,
                               ord + (size_t)p * wn, n, live + (size_t)p * wn, live + (size_t)(p + 1) * wn, st, rf2,
                               (int)(p == NP - 1), pp, pp + nchunk, pp + 2 * nchunk, pp + 3 * nchunk, cur, rad);
        CAPT_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_output, dim3(nblk(n)), dim3(TB), 0, s, xyz, cur, n, st, rad, out_xyz, out_index, map,
                       res.as<unsigned long long>());
    CAPT_LAUNCH_CHECK();
    const hipError_t se = hipStreamSynchronize(s);
    if (se != hipSuccess) {
        res.p = nullptr;   // the kernel's state is unknown: never hand the block out again
        return hip_fail(se, "hipStreamSynchronize", __FILE__, __LINE__);
    }
    const unsigned long long *h = res.as<unsigned long long>();
    if (h[2]) {
        set_error("internal: a look-back wait bound was exceeded in the filter (code %llu)", h[2]);
        return CAPT_EHIP;
    }
    if (h[1]) {
        set_error("input holds %llu non-finite coordinates", h[1]);
        return CAPT_EINVAL;
    }
    *n_out = (int64_t)h[0];
    return CAPT_OK;
}

}  // namespace

capt_status filter(const float *xyz, int64_t n, float r_filter, const float *crop, float *out_xyz,
                   int32_t *out_index, int64_t *n_out, hipStream_t s) {
    if (!crop || n == 0) return filter_core(xyz, n, r_filter, nullptr, out_xyz, out_index, n_out, s);
    // the crop first: stable compaction of the points inside the reach ball,
    // then the filter on them with their input indices as the index map
    const size_t wn = (size_t)n;
    const size_t nst = scan_lb_words(n) + 64;
    const size_t oC = 0;
    const size_t oMap = align256(oC + sizeof(float) * 3 * wn);
    const size_t oFlag = align256(oMap + sizeof(uint32_t) * wn);
    const size_t oPos = align256(oFlag + sizeof(uint32_t) * wn);
    const size_t oSt = align256(oPos + sizeof(uint32_t) * wn);
    const size_t bytes = align256(oSt + sizeof(uint32_t) * nst);
    Scratch sc;
    if (!sc.alloc(bytes, s)) {
        set_error("device allocation of %zu crop scratch bytes failed", bytes);
        return CAPT_ENOMEM;
    }
    Pinned res;
    if (!res.alloc(3 * sizeof(unsigned long long))) {
        set_error("pinned host allocation failed");
        return CAPT_ENOMEM;
    }
    char *B = sc.as<char>();
    float *cxyz = reinterpret_cast<float *>(B + oC);
    uint32_t *map = reinterpret_cast<uint32_t *>(B + oMap);
    uint32_t *flag = reinterpret_cast<uint32_t *>(B + oFlag);
    uint32_t *pos = reinterpret_cast<uint32_t *>(B + oPos);
    uint32_t *status = reinterpret_cast<uint32_t *>(B + oSt);   // [0, 64): bad count and error word
    const float reach2 = crop[3] * crop[3];   // one float32 product (contraction is off)
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min<int64_t>((int64_t)(nst + TB - 1) / TB, 1024)), dim3(TB),
                       0, s, status, (int64_t)nst);
    CAPT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_crop_flag, dim3((unsigned)std::min<int64_t>(nblk(n), 4096)), dim3(TB), 0, s, xyz, n, crop[0],
                       crop[1], crop[2], reach2, flag, reinterpret_cast<unsigned int *>(status));
    CAPT_LAUNCH_CHECK();
    capt_status e = scan_exclusive_u32_lb(flag, pos, n, status + 64, status + 1, s);
    if (e) return e;
    hipLaunchKernelGGL(k_crop_compact, dim3(nblk(n)), dim3(TB), 0, s, xyz, n, flag, pos, cxyz, map,
                       reinterpret_cast<const unsigned int *>(status), status + 1, res.as<unsigned long long>());
    CAPT_LAUNCH_CHECK();
    const hipError_t se = hipStreamSynchronize(s);
    if (se != hipSuccess) {
        res.p = nullptr;   // the kernels' state is unknown: never hand the block out again
        return hip_fail(se, "hipStreamSynchronize", __FILE__, __LINE__);
    }
    const unsigned long long *h = res.as<unsigned long long>();
    if (h[2]) {
        set_error("internal: a look-back wait bound was exceeded in the crop (code %llu)", h[2]);
        return CAPT_EHIP;
    }
    if (h[1]) {
        set_error("input holds %llu non-finite coordinates", h[1]);
        return CAPT_EINVAL;
    }
    return filter_core(cxyz, (int64_t)h[0], r_filter, map, out_xyz, out_index, n_out, s);
}

}  // namespace capt
