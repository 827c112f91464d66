// Collision queries against CAPTs (Alg. 3, Sec. IV-D) on wave64 CDNA4.
//
// Mapping.  A wavefront holds up to 64 spheres, one per lane: 64 / g whole
// configurations of g <= 16 spheres (k_collide_cloud), or four 16-lane slots,
// each holding the next 16 spheres of one larger configuration
// (k_collide_slots; a slot moves on to the configuration's next 16 spheres
// only if the current ones missed, so a configuration stops at its first
// colliding piece, as Alg. 3's sequential loop stops at its first colliding
// sphere).  Each lane descends the tree branch-free (the top levels of T sit
// in LDS) and tests its leaf's AABB.  The surviving spheres' sets are stored
// as 16-entry chunks with a float32 box each and are scanned in two levels:
// the (sphere, chunk) pairs of all surviving spheres form one flattened list
// (an exclusive wave scan of the chunk counts places each sphere's pairs;
// every lane takes one pair per step), chunks whose box lies within reach go
// to a per-wave ring in LDS, and the entries of four ring chunks are tested
// per 64-lane step.  A ballot after every step marks the configurations that
// were hit; their spheres drop out (early exit, Sec. I and IV-D).  Every lane
// stays busy whatever the mix of set sizes, which the paper's CPU layout
// (lanes across one set at a time) does not give.
//
// Kernels: k_collide_cloud / k_collide_slots (one cloud, persistent, per-XCD
// work queues), k_collide_batched (many clouds, persistent, tiles popped from a
// queue sorted by descending cost), k_brute (baseline), k_query_stats and
// k_chunk_stats (work accounting).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>

#include "capt_internal.h"

namespace capt {

namespace {

// Inclusive scan over the 64 lanes with DPP adds: shifts inside each row of
// 16 lanes, then row 0's total into row 1 and row 2's into row 3 (row_bcast:15),
// then lane 31's running total into rows 2 and 3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);   // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return v;
}

// Inclusive maximum over the 64 lanes with the same DPP pattern (lanes that
// receive nothing take -1, below every lane index).
__device__ __forceinline__ int wave_incl_max(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x111, 0xf, 0xf, false));   // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x112, 0xf, 0xf, false));   // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x114, 0xf, 0xf, false));   // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x118, 0xf, 0xf, false));   // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x142, 0xa, 0xf, false));   // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return v;
}

// Load at a 32-bit byte offset from a wave-uniform base: the address stays a
// scalar base plus one 32-bit lane offset (no 64-bit per-lane address math).
// Used for arrays under 4 GiB: T (fewer than 2^30 nodes), the set arrays and
// chunk boxes (fewer than 2^30 entries).
template <class T> __device__ __forceinline__ T ld32(const T *base, uint32_t byte_off) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

__device__ __forceinline__ float axis_of(const float4 &q, int a) {
    return a == 0 ? q.x : (a == 1 ? q.y : q.z);
}

// Branch-free descent: i <- 2i + 1 + (x_d > T_i), ties go left.  The first
// `L` levels read T from LDS.
// The split axis of depth lv comes from the forest's axis code.
__device__ __forceinline__ uint32_t descend(const float4 &q, const float *Tl, int L,
                                            const float *__restrict__ Tg, int D, uint64_t axes) {
    uint32_t i = 0;
    int lv = 0;
    for (; lv < L; ++lv) {
        const float t = Tl[i];
        i = 2 * i + 1 + (axis_of(q, axis_at(axes, lv)) > t ? 1u : 0u);
    }
    for (; lv < D; ++lv) {
        const float t = Tg[i];
        i = 2 * i + 1 + (axis_of(q, axis_at(axes, lv)) > t ? 1u : 0u);
    }
    return i;
}

// descend_leaf for a forest whose split axes do not follow d mod 3: one level
// per step.
__device__ __forceinline__ Leaf descend_leaf_any(const float4 &q, const float *Tl, int L,
                                                 const float *__restrict__ Tg, const Leaf *__restrict__ leaves,
                                                 int D, uint64_t axes, uint32_t *lf) {
    uint32_t i = 0;
    int lv = 0;
    for (; lv < L; ++lv) i = 2 * i + 1 + (axis_of(q, axis_at(axes, lv)) > Tl[i] ? 1u : 0u);
    for (; lv < D; ++lv) i = 2 * i + 1 + (axis_of(q, axis_at(axes, lv)) > ld32(Tg, 4u * i) ? 1u : 0u);
    *lf = i - ((1u << D) - 1u);
    return leaves[*lf];
}

// The same descent, shaped for latency: the LDS levels are taken three per
// round trip (the node, both children and all four grandchildren are read
// together, then three comparisons pick the path), and so are the global
// levels down to the first root level of the tree's blocked copy (TB, when the
// forest has one); from there every four levels are one 64-byte block, one
// cache line per round trip.  Returns the leaf record; *lf gets its index.
__device__ __forceinline__ Leaf descend_leaf(const float4 &q, const float *Tl, int L, const float *__restrict__ Tg,
                                             const float4 *__restrict__ TB, const Leaf *__restrict__ leaves, int D,
                                             uint32_t *lf) {
    const float xs[3] = {q.x, q.y, q.z};
    uint32_t i = 0;
    int lv = 0;
    for (; lv + 3 <= L; lv += 3) {   // levels lv, lv+1, lv+2 split axes 0, 1, 2 (lv is a multiple of 3)
        const float t0 = Tl[i];
        const float t1a = Tl[2 * i + 1], t1b = Tl[2 * i + 2];
        const float t2a = Tl[4 * i + 3], t2b = Tl[4 * i + 4], t2c = Tl[4 * i + 5], t2d = Tl[4 * i + 6];
        const uint32_t b0 = xs[0] > t0 ? 1u : 0u;
        const uint32_t b1 = xs[1] > (b0 ? t1b : t1a) ? 1u : 0u;
        const float t2 = b0 ? (b1 ? t2d : t2c) : (b1 ? t2b : t2a);
        const uint32_t b2 = xs[2] > t2 ? 1u : 0u;
        i = 8 * i + 7 + 4 * b0 + 2 * b1 + b2;
    }
    int a = lv % 3;
    for (; lv < L; ++lv) {
        i = 2 * i + 1 + (xs[a] > Tl[i] ? 1u : 0u);
        a = (a == 2) ? 0 : a + 1;
    }
    // Eytzinger levels lv .. gend - 1 (all the rest without a blocked copy)
    const int gend = TB ? D - 4 * ((D - lv) / 4) : D;
    const int a1 = (a == 2) ? 0 : a + 1;
    const int a2 = (a1 == 2) ? 0 : a1 + 1;
    for (; lv + 3 <= gend; lv += 3) {   // after three levels the cyclic axis is back to `a`
        const float t0 = ld32(Tg, 4u * i);
        const float t1a = ld32(Tg, 8u * i + 4u), t1b = ld32(Tg, 8u * i + 8u);
        const float t2a = ld32(Tg, 16u * i + 12u), t2b = ld32(Tg, 16u * i + 16u);
        const float t2c = ld32(Tg, 16u * i + 20u), t2d = ld32(Tg, 16u * i + 24u);
        const uint32_t b0 = xs[a] > t0 ? 1u : 0u;
        const uint32_t b1 = xs[a1] > (b0 ? t1b : t1a) ? 1u : 0u;
        const float t2 = b0 ? (b1 ? t2d : t2c) : (b1 ? t2b : t2a);
        const uint32_t b2 = xs[a2] > t2 ? 1u : 0u;
        i = 8 * i + 7 + 4 * b0 + 2 * b1 + b2;
    }
    if (gend - lv == 2) {
        const float t0 = ld32(Tg, 4u * i), t1a = ld32(Tg, 8u * i + 4u), t1b = ld32(Tg, 8u * i + 8u);
        const uint32_t b0 = xs[a] > t0 ? 1u : 0u;
        const uint32_t b1 = xs[a1] > (b0 ? t1b : t1a) ? 1u : 0u;
        i = 4 * i + 3 + 2 * b0 + b1;
    } else if (gend - lv == 1) {
        i = 2 * i + 1 + (xs[a] > ld32(Tg, 4u * i) ? 1u : 0u);
    }
    if (TB) {
        // 4-level blocks from root level gend: levels r .. r+3 split on axes
        // c0, c1, c2, c0 (cyclic), and the next block's root on c1
        int c0 = gend % 3;
        for (int r = gend; r < D; r += 4) {
            const int c1 = (c0 == 2) ? 0 : c0 + 1;
            const int c2 = (c1 == 2) ? 0 : c1 + 1;
            const uint32_t off = 64u * (tree_block_base(r, D) + (i - ((1u << r) - 1u)));
            const float4 v0 = ld32(TB, off), v1 = ld32(TB, off + 16u), v2 = ld32(TB, off + 32u),
                         v3 = ld32(TB, off + 48u);
            // v0 = (n0, n1, n2, n3), v1 = (n4, n5, n6, n7), v2 = (n8 .. n11), v3 = (n12, n13, n14, pad)
            const uint32_t b0 = xs[c0] > v0.x ? 1u : 0u;
            const uint32_t b1 = xs[c1] > (b0 ? v0.z : v0.y) ? 1u : 0u;
            const float t2 = b0 ? (b1 ? v1.z : v1.y) : (b1 ? v1.x : v0.w);
            const uint32_t b2 = xs[c2] > t2 ? 1u : 0u;
            const float p0 = b2 ? v2.x : v1.w, p1 = b2 ? v2.z : v2.y;
            const float p2 = b2 ? v3.x : v2.w, p3 = b2 ? v3.z : v3.y;
            const float t3 = b0 ? (b1 ? p3 : p2) : (b1 ? p1 : p0);
            const uint32_t b3 = xs[c0] > t3 ? 1u : 0u;
            i = 16 * i + 15 + 8 * b0 + 4 * b1 + 2 * b2 + b3;
            c0 = c1;
        }
    }
    *lf = i - ((1u << D) - 1u);
    return leaves[*lf];
}

// Lanes per configuration slot of the slot kernels (four slots per wave).
constexpr int SLOT = 16;

// Per-wave LDS scratch of the two-level set scan.
constexpr uint32_t RING = 128;                 // chunks awaiting the entry scan (power of two)
constexpr uint32_t CPS = WAVE / CHUNK;         // chunks covered by one 64-lane step
struct WaveLds {
    float4 sph[WAVE];        // the tile's spheres, w = fl(r*r)
    uint32_t chunk[RING];    // surviving chunk (global chunk index)
    uint8_t owner[RING];     // lane of the sphere it belongs to
    float4 base[WAVE];       // lower corner of each sphere's set box (chunk boxes are relative to it)
    int8_t start[WAVE];      // box step: the lane whose pairs start at this slot, or -1
    uint8_t hitf[WAVE];      // entry round: 1 for a sphere hit in this round
    uint8_t pad[32];
};
static_assert(sizeof(WaveLds) % 16 == 0, "per-wave LDS blocks stay 16-byte aligned");

// LDS written by some lanes of a wave and read by others: the LDS unit serves
// one wave's requests in order, so only compiler reordering must be stopped.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Process one tile of up to 64 spheres against one cloud.  Lane l holds a
// sphere if `valid`; the lanes form groups of gg (lanes c*gg .. c*gg+gg-1),
// each group a part of one configuration, or the whole wave is one
// configuration (`single`).  Returns, per lane, whether a sphere of its group
// (its configuration when single) was hit.
//
// A surviving sphere's set is stored as 16-entry chunks, each with a float32
// bounding box.  Level 1 box-tests the (sphere, chunk) pairs of all surviving
// spheres as one flattened list (an exclusive wave scan of the chunk counts
// places each sphere's pairs; lane j of a step finds its sphere by binary
// search over the scan) and appends the chunks whose box is within r to a
// per-wave ring in LDS.  Level 2 tests the entries of 4 ring chunks per
// 64-lane step (lane j: entry j % 16 of chunk j / 16), U steps in flight.  A
// chunk box never lies farther than any of its points under the same rounding
// order, so a skipped chunk holds no hit and the answer equals a scan of every
// entry.  A hit retires its configuration: its spheres' ring chunks are
// skipped and the level-1 prefix is rebuilt over the spheres still open.
template <int U, bool IDX, bool SLOTS, bool AXES = true>
__device__ __forceinline__ bool wave_tile(const CloudDev &C, const float *Tl, int L, float4 q, bool valid, int gg,
                                          bool single, WaveLds &W) {
    const int lane = lane_id();
    const float r2 = __fmul_rn(q.w, q.w);
    Leaf leaf;
    uint32_t lf;
    if (AXES && !C.cyclic)   // uniform; the batched kernel takes cyclic forests only
        leaf = descend_leaf_any(q, Tl, L, C.T, C.leaf, C.D, C.axes, &lf);
    else
        leaf = descend_leaf(q, Tl, L, C.T, C.tb, C.leaf, C.D, &lf);
    if (!valid) leaf.count = 0;
    bool alive = leaf.count > 0;
    if (alive) alive = box_sqdist(q.x, q.y, q.z, leaf.lo, leaf.hi) <= r2;
    wave_lds_sync();   // the previous tile's readers of W are done
    W.sph[lane] = make_float4(q.x, q.y, q.z, r2);
    W.base[lane] = make_float4(leaf.lo[0], leaf.lo[1], leaf.lo[2], 0.0f);
    W.start[lane] = -1;
    W.hitf[lane] = 0;
    const int cfg = lane / gg;
    const uint64_t gmask = gg >= WAVE ? ~0ull : ((1ull << gg) - 1);
    bool done = false;
    uint64_t dead = 0;                                    // lanes whose configuration is hit
    uint32_t rem = alive ? (leaf.count + CHUNK - 1) / CHUNK : 0u;   // chunks not yet box-tested
    uint32_t cpos = leaf.start / CHUNK;                   // the first of them
    // A one-chunk set's chunk box is its leaf AABB, already passed: straight
    // to the entry scan.
    const bool direct = rem == 1u;
    const uint64_t dm = __ballot(direct);
    if (direct) {
        const uint32_t at = lanes_below(dm);
        W.chunk[at] = cpos;
        W.owner[at] = (uint8_t)lane;
        rem = 0u;
    }
    uint32_t head = 0, tail = (uint32_t)__popcll(dm);     // ring [head, tail), wave-uniform
    const uint4 *__restrict__ CB = C.cbox;
    const float *__restrict__ PX = C.px;
    const int32_t *__restrict__ PI = C.pidx;
    const float *__restrict__ PT = C.pts;
    constexpr bool indexed = IDX;   // sets of point indices (CAPT_INDEXED_SETS)

    // Entry scan of the next `nproc` <= U*CPS ring chunks; true if a hit retired
    // a configuration (then `done` and `dead` are up to date).
    auto entry_round = [&](uint32_t nproc) -> bool {
        float4 s[U];
        float px[U], py[U], pz[U];
        int own[U];
        bool in[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t k = (uint32_t)u * CPS + (uint32_t)lane / CHUNK;
            in[u] = k < nproc;
            const uint32_t slot = (head + k) & (RING - 1);
            uint32_t ch = 0;
            int o = 0;
            if (in[u]) {
                ch = W.chunk[slot];
                o = W.owner[slot];
            }
            in[u] = in[u] && !((dead >> o) & 1ull);
            own[u] = o;
            s[u] = W.sph[o];
            const uint32_t e = ch * CHUNK + ((uint32_t)lane & (CHUNK - 1));
            if (indexed) {
                // the entry's point index, then its coordinates in the point
                // table; padding entries (index -1) are skipped
                const int32_t id = in[u] ? ld32(PI, 4u * e) : -1;
                in[u] = id >= 0;
                const int64_t p3 = 3 * (int64_t)(id >= 0 ? id : 0);
                px[u] = in[u] ? PT[p3] : 0.f;
                py[u] = in[u] ? PT[p3 + 1] : 0.f;
                pz[u] = in[u] ? PT[p3 + 2] : 0.f;
            } else {
                // the chunk's x, y and z blocks from one 64-bit address
                const float *cp = PX + 48 * (size_t)ch + ((uint32_t)lane & (CHUNK - 1));
                px[u] = in[u] ? cp[0] : 0.f;
                py[u] = in[u] ? cp[CHUNK] : 0.f;
                pz[u] = in[u] ? cp[2 * CHUNK] : 0.f;
            }
        }
        bool hit[U];
        bool any = false;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            hit[u] = in[u] && sqdist(s[u].x, s[u].y, s[u].z, px[u], py[u], pz[u]) <= s[u].w;
            any = any || hit[u];
        }
        head += nproc;
        if (__ballot(any) == 0) return false;
        if (single) {
            done = valid;
            return true;
        }
        if (SLOTS) {
            // four groups of SLOT lanes (gg == SLOT): one ballot per group
            uint32_t gm = 0;
#pragma unroll
            for (int c = 0; c < WAVE / SLOT; ++c) {
                bool h = false;
#pragma unroll
                for (int u = 0; u < U; ++u) h = h || (hit[u] && own[u] / SLOT == c);
                if (__ballot(h) != 0) gm |= 1u << c;
            }
            if (valid) done = done || ((gm >> cfg) & 1u) != 0;
        } else {
            // the spheres hit in this round, flagged in LDS by the lanes that
            // found the hits, then read back one flag per lane
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (hit[u]) W.hitf[own[u]] = 1;
            wave_lds_sync();
            const uint64_t hm = __ballot(W.hitf[lane] != 0);
            W.hitf[lane] = 0;
            if (valid) done = done || (((hm >> (cfg * gg)) & gmask) != 0);
        }
        dead = __ballot(done);
        return true;
    };

    wave_lds_sync();
    while (tail - head >= (uint32_t)U * CPS) {
        if (entry_round((uint32_t)U * CPS) && single) return done;
    }
    while (true) {
        if (done) rem = 0;
        const uint32_t incl = wave_incl_scan(rem, lane);
        const uint32_t excl = incl - rem;
        const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
        if (total == 0) break;
        const uint32_t base_l = cpos - excl;   // chunk of pair slot t of this lane = base_l + t
        bool rescan = false;
        uint32_t end = 0;
        int carry = -1;   // the lane whose pairs cover slot k0 (from the previous step)
        for (uint32_t k0 = 0; k0 < total && !rescan; k0 += WAVE) {
            const uint32_t slot = k0 + (uint32_t)lane;
            // owner of this lane's slot: the last lane whose pairs start at or
            // before it (lanes mark their first slot in LDS, then a prefix maximum)
            if (rem > 0u && excl >= k0 && excl - k0 < (uint32_t)WAVE) W.start[excl - k0] = (int8_t)lane;
            wave_lds_sync();
            int sv = W.start[lane];
            W.start[lane] = -1;
            if (lane == 0) sv = max(sv, carry);
            const int o = wave_incl_max(sv);
            carry = __builtin_amdgcn_readlane(o, WAVE - 1);
            const uint32_t ch = __shfl(base_l, o, WAVE) + slot;
            const bool in = slot < total && !((dead >> o) & 1ull);
            const float4 so = W.sph[o];
            bool surv = false;
            if (in) {
                const float4 bo = W.base[o];
                float lo[3], hi[3];
                hbox_decode(ld32(CB, 16u * ch), bo.x, bo.y, bo.z, lo, hi);
                surv = box_sqdist(so.x, so.y, so.z, lo, hi) <= so.w;
            }
            const uint64_t m = __ballot(surv);
            if (surv) {
                const uint32_t at = (tail + lanes_below(m)) & (RING - 1);
                W.chunk[at] = ch;
                W.owner[at] = (uint8_t)o;
            }
            tail += (uint32_t)__popcll(m);
            end = k0 + WAVE;
            wave_lds_sync();
            // full rounds only; fewer than U*CPS chunks stay for the next batch,
            // so the ring never holds more than U*CPS + 63 < RING chunks
            while (tail - head >= (uint32_t)U * CPS) {
                if (entry_round((uint32_t)U * CPS)) {
                    if (single) return done;
                    rescan = true;
                }
            }
        }
        if (!rescan) break;   // every chunk has been box-tested
        const uint32_t used = end <= excl ? 0u : min(rem, end - excl);
        rem -= used;
        cpos += used;
    }
    while (head != tail) {
        if (entry_round(min(tail - head, (uint32_t)U * CPS)) && single) break;
    }
    return done;
}

// Per-XCD work queues: blocks are dispatched round-robin over the XCDs, so
// block b takes tiles from the range and counter of XCD b % NXCD, keeping the
// queue atomics in that XCD's L2.
constexpr int NXCD = 8;
constexpr int CTR_STRIDE = 16;   // one 64-byte line per counter

template <int U, bool IDX>
__global__ void k_collide_cloud(CloudDev C, const float4 *__restrict__ sph, int64_t nsph, int g,
                                uint8_t *__restrict__ out, int L, unsigned int *__restrict__ ctr, int chunk) {
    extern __shared__ float4 lds4[];
    WaveLds &W = reinterpret_cast<WaveLds *>(lds4)[threadIdx.x / WAVE];
    float *Tl = reinterpret_cast<float *>(reinterpret_cast<WaveLds *>(lds4) + blockDim.x / WAVE);
    const int nT = (1 << L) - 1;
    for (int i = threadIdx.x; i < nT; i += blockDim.x) Tl[i] = C.T[i];
    __syncthreads();
    const int lane = lane_id();
    const int64_t ncfg = nsph / g;
    const int cpt = g <= WAVE ? WAVE / g : 1;       // configurations per tile
    const int64_t ntiles = (ncfg + cpt - 1) / cpt;
    const int nq = (int)min<int64_t>(NXCD, (int64_t)gridDim.x);
    const int xq = (int)(blockIdx.x % (unsigned)nq);
    const int64_t t0 = ntiles * xq / nq, t1 = ntiles * (xq + 1) / nq;
    while (true) {
        unsigned int c = 0;
        if (lane == 0) c = atomicAdd(&ctr[xq * CTR_STRIDE], (unsigned int)chunk);
        c = __shfl(c, 0, WAVE);
        const int64_t ta = t0 + (int64_t)c;
        if (ta >= t1) break;
        const int64_t tb = min<int64_t>(ta + chunk, t1);
        if (g <= WAVE) {
            // the next tile's spheres are loaded while this one is processed
            auto load = [&](int64_t t) {
                const int64_t c0 = t * cpt;
                const int nc = (int)min<int64_t>(cpt, ncfg - c0);
                return lane < nc * g ? sph[c0 * g + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
            };
            float4 qn = load(ta);
            for (int64_t t = ta; t < tb; ++t) {
                const float4 q = qn;
                if (t + 1 < tb) qn = load(t + 1);
                const int64_t c0 = t * cpt;
                const int nc = (int)min<int64_t>(cpt, ncfg - c0);
                const bool hit = wave_tile<U, IDX, false>(C, Tl, L, q, lane < nc * g, g, 2 * g > nc * g, W);
                if (lane < nc * g && lane % g == 0) out[c0 + lane / g] = (uint8_t)hit;
            }
        } else {
            for (int64_t t = ta; t < tb; ++t) {
                bool hit = false;
                for (int s0 = 0; s0 < g && !hit; s0 += WAVE) {
                    const int ns = min(WAVE, g - s0);
                    const float4 q = lane < ns ? sph[t * g + s0 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
                    hit = wave_tile<U, IDX, false>(C, Tl, L, q, lane < ns, WAVE, true, W);
                    hit = __shfl(hit, 0, WAVE);
                }
                if (lane == 0) out[t] = (uint8_t)hit;
            }
        }
    }
}


// Sphere sources of the slot kernel: item i has `len` spheres in test order.
// Materialised spheres: item = configuration, sphere k = spheres[i * g + k].
struct SphereSrc {
    const float4 *sph;
    __device__ __forceinline__ float4 operator()(int64_t item, int k, int len) const {
        return sph[item * len + k];
    }
};
// Posed template: item = edge of `edge` configurations, each a rigid pose
// (row-major rotation R, then translation t: 12 floats) of the g template
// spheres; sphere k is template sphere k % g under pose item * edge + k / g:
// centre ((R0 x + R1 y) + R2 z) + t0 (and likewise), every operation rounded
// to float32 on its own, radius unchanged.
struct PosedSrc {
    const float *poses;
    const float4 *tmpl;
    int g;
    __device__ __forceinline__ float4 operator()(int64_t item, int k, int len) const {
        const int edge = len / g;
        const int c = k / g;
        const float4 t = tmpl[k - c * g];
        const float *P = poses + 12 * (item * edge + c);
        const float4 a = *reinterpret_cast<const float4 *>(P);       // R0 R1 R2 R3
        const float4 b = *reinterpret_cast<const float4 *>(P + 4);   // R4 R5 R6 R7
        const float4 d = *reinterpret_cast<const float4 *>(P + 8);   // R8 t0 t1 t2
        float4 q;
        q.x = __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(a.x, t.x), __fmul_rn(a.y, t.y)), __fmul_rn(a.z, t.z)), d.y);
        q.y = __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(a.w, t.x), __fmul_rn(b.x, t.y)), __fmul_rn(b.y, t.z)), d.z);
        q.z = __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(b.z, t.x), __fmul_rn(b.w, t.y)), __fmul_rn(d.x, t.z)), d.w);
        q.w = t.w;
        return q;
    }
};

// Padded spheres (query padding, Sec. V-B): radius r + pad, one float32
// addition, so that a filtered cloud answers conservatively.
struct PaddedSrc {
    const float4 *sph;
    float pad;
    __device__ __forceinline__ float4 operator()(int64_t item, int k, int len) const {
        float4 q = sph[item * len + k];
        q.w = __fadd_rn(q.w, pad);
        return q;
    }
};

// Items (configurations, or edges of posed configurations) of `len` spheres,
// with early exit inside an item: the wave's 64 lanes form four slots of
// SLOT lanes; a slot holds one item and tests its spheres SLOT at a time, in
// order, stopping at the first piece with a hit (as a sequential scan of the
// item would); a slot that finishes takes the next item from the wave's
// popped range (per-XCD queues as above).  The slots of a wave run together
// through the two-level scan, each slot a group.
// U <= 2 is held to 64 VGPRs, so that eight waves fit per SIMD (32 per CU):
// the kernel is bound by memory latency and more resident waves hide more
// of it; U = 4 would spill at that budget.
template <int U, class Src, bool IDX>
__global__ void __attribute__((amdgpu_waves_per_eu(U <= 2 ? 8 : 1, 8))) k_collide_slots(CloudDev C, Src src, int64_t ncfg, int g,
                                uint8_t *__restrict__ out, int L, unsigned int *__restrict__ ctr, int chunk) {
    extern __shared__ float4 lds4[];
    WaveLds &W = reinterpret_cast<WaveLds *>(lds4)[threadIdx.x / WAVE];
    float *Tl = reinterpret_cast<float *>(reinterpret_cast<WaveLds *>(lds4) + blockDim.x / WAVE);
    const int nT = (1 << L) - 1;
    for (int i = threadIdx.x; i < nT; i += blockDim.x) Tl[i] = C.T[i];
    __syncthreads();
    const int lane = lane_id();
    const int j = lane & (SLOT - 1);
    const int lead = lane & ~(SLOT - 1);   // first lane of this lane's slot
    const int nq = (int)min<int64_t>(NXCD, (int64_t)gridDim.x);
    const int xq = (int)(blockIdx.x % (unsigned)nq);
    const int64_t t0 = ncfg * xq / nq, t1 = ncfg * (xq + 1) / nq;
    int64_t ra = 0, rb = 0;   // popped configurations not yet started (wave-uniform)
    bool drained = false;
    int64_t cfg = -1;         // the configuration in this lane's slot, -1 = free
    int s0 = 0;               // its next piece starts at sphere s0
    while (true) {
        // fill free slots in slot order, popping more configurations as needed
        while (true) {
            const uint64_t freem = __ballot(j == 0 && cfg < 0);
            if (freem == 0) break;
            if (ra >= rb) {
                if (drained) break;
                unsigned int c = 0;
                if (lane == 0) c = atomicAdd(&ctr[xq * CTR_STRIDE], (unsigned int)chunk);
                c = __shfl(c, 0, WAVE);
                const int64_t a = t0 + (int64_t)c;
                if (a >= t1) {
                    drained = true;
                    break;
                }
                ra = a;
                rb = min<int64_t>(a + chunk, t1);
            }
            const bool myfree = (freem >> lead) & 1ull;
            const int64_t rank = __popcll(freem & ((1ull << lead) - 1ull));   // free slots before this one
            if (myfree && rank < rb - ra) {
                cfg = ra + rank;
                s0 = 0;
            }
            ra = min<int64_t>(ra + __popcll(freem), rb);
        }
        const bool active = cfg >= 0;
        if (__ballot(active) == 0) break;   // range drained and every slot finished
        const int si = s0 + j;
        const bool valid = active && si < g;
        const float4 q = valid ? src(cfg, si, g) : make_float4(0.f, 0.f, 0.f, 0.f);
        bool hit = wave_tile<U, IDX, true>(C, Tl, L, q, valid, SLOT, false, W);
        hit = __shfl(hit, lead, WAVE);   // the slot's first lane always holds a sphere
        if (active) {
            if (hit || s0 + SLOT >= g) {
                if (j == 0) out[cfg] = (uint8_t)hit;
                cfg = -1;
            } else {
                s0 += SLOT;
            }
        }
    }
}

__global__ void k_zero_u32(unsigned int *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// One queue entry of the batched launch.
struct Tile {
    int32_t cloud;
    int32_t ncfg;
    int64_t cfg0;   // global configuration index (= output index)
};

__global__ void k_reset_counter(unsigned int *ctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr = 0u;
}

// The slot scheme of k_collide_slots over one fixed range of configurations
// [c0, c1) of one cloud (no LDS tree levels); returns when all are answered.
template <int U, bool IDX>
__device__ void slots_over_range(const CloudDev &C, const float *Tl, int L, const float4 *__restrict__ sph, int g,
                                 int64_t c0, int64_t c1, uint8_t *__restrict__ out, int32_t *__restrict__ visits,
                                 WaveLds &W) {
    const int lane = lane_id();
    const int j = lane & (SLOT - 1);
    const int lead = lane & ~(SLOT - 1);
    int64_t ra = c0;
    int64_t cfg = -1;
    int s0 = 0;
    while (true) {
        const uint64_t freem = __ballot(j == 0 && cfg < 0);
        if (freem != 0 && ra < c1) {
            const bool myfree = (freem >> lead) & 1ull;
            const int64_t rank = __popcll(freem & ((1ull << lead) - 1ull));
            if (myfree && rank < c1 - ra) {
                cfg = ra + rank;
                s0 = 0;
            }
            ra = min<int64_t>(ra + __popcll(freem), c1);
        }
        const bool active = cfg >= 0;
        if (__ballot(active) == 0) break;
        const int si = s0 + j;
        const bool valid = active && si < g;
        const float4 q = valid ? sph[cfg * g + si] : make_float4(0.f, 0.f, 0.f, 0.f);
        bool hit = wave_tile<U, IDX, true, false>(C, Tl, L, q, valid, SLOT, false, W);
        hit = __shfl(hit, lead, WAVE);
        if (active) {
            if (hit || s0 + SLOT >= g) {
                if (j == 0) {
                    out[cfg] = (uint8_t)hit;
                    if (visits) atomicAdd(&visits[cfg], 1);
                }
                cfg = -1;
            } else {
                s0 += SLOT;
            }
        }
    }
}

// Tree levels of the batched kernel's per-wave LDS copy (2^9 - 1 = 511 split
// values).
constexpr int BATCH_TOP = 9;

template <int U, bool IDX>
__global__ void k_collide_batched(const CloudDev *__restrict__ clouds, const Tile *__restrict__ tiles,
                                  int64_t ntiles, unsigned int *__restrict__ ctr,
                                  const float4 *__restrict__ sph, int g, uint8_t *__restrict__ out,
                                  int32_t *__restrict__ visits) {
    extern __shared__ float4 lds4[];
    WaveLds &W = reinterpret_cast<WaveLds *>(lds4)[threadIdx.x / WAVE];
    // the top BATCH_TOP levels of the current tile's tree, one copy per wave,
    // reloaded when a tile of another cloud comes
    float *Tl = reinterpret_cast<float *>(reinterpret_cast<WaveLds *>(lds4) + blockDim.x / WAVE) +
                (threadIdx.x / WAVE) * (1 << BATCH_TOP);
    const int lane = lane_id();
    int cur = -1, L = 0;
    while (true) {
        unsigned int t = 0;
        if (lane == 0) t = atomicAdd(ctr, 1u);
        t = __shfl(t, 0, WAVE);
        if ((int64_t)t >= ntiles) break;
        const Tile tile = tiles[t];
        const CloudDev C = clouds[tile.cloud];
        if (tile.cloud != cur) {
            cur = tile.cloud;
            L = min(C.D, BATCH_TOP);
            wave_lds_sync();   // the last tile's descents are done with the old copy
            for (int k = lane; k < (1 << L) - 1; k += WAVE) Tl[k] = C.T[k];
            wave_lds_sync();
        }
        if (g > SLOT) {
            slots_over_range<U, IDX>(C, Tl, L, sph, g, tile.cfg0, tile.cfg0 + tile.ncfg, out, visits, W);
        } else {
            const int cpt = WAVE / g;
            for (int c = 0; c < tile.ncfg; c += cpt) {
                const int64_t c0 = tile.cfg0 + c;
                const int nc = min(cpt, tile.ncfg - c);
                const float4 q = lane < nc * g ? sph[c0 * g + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
                const bool hit = wave_tile<U, IDX, false, false>(C, Tl, L, q, lane < nc * g, g, 2 * g > nc * g, W);
                if (lane < nc * g && lane % g == 0) {
                    out[c0 + lane / g] = (uint8_t)hit;
                    if (visits) atomicAdd(&visits[c0 + lane / g], 1);
                }
            }
        }
    }
}

// GPU brute force: one wave per tile of spheres (as above); the cloud is
// streamed in index order, 64 points per step (one per lane, broadcast with
// readlane), same predicate; after every step a ballot retires the tile once
// every configuration in it has been hit.
__global__ void k_brute(const float *__restrict__ pts, int64_t n, const float4 *__restrict__ sph,
                        int64_t nsph, int g, uint8_t *__restrict__ out) {
    const int lane = lane_id();
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int64_t ncfg = nsph / g;
    const int gg = g > WAVE ? WAVE : g;
    const uint64_t gmask = gg >= WAVE ? ~0ull : ((1ull << gg) - 1);
    const int cpt = g > WAVE ? 1 : WAVE / g;
    const int64_t ntiles = (ncfg + cpt - 1) / cpt;
    for (int64_t t = wid; t < ntiles; t += waves) {
        const int64_t c0 = t * cpt;
        const int nc = (int)min<int64_t>(cpt, ncfg - c0);
        bool any_slice = false;                   // g > 64: configuration hit so far
        const int nslice = g > WAVE ? (g + WAVE - 1) / WAVE : 1;
        bool done = false;
        for (int sl = 0; sl < nslice && !any_slice; ++sl) {
            const int ns = g > WAVE ? min(WAVE, g - sl * WAVE) : nc * g;
            const bool valid = lane < ns;
            const int64_t s0 = c0 * g + (int64_t)sl * WAVE;
            const float4 q = valid ? sph[s0 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
            const float r2 = __fmul_rn(q.w, q.w);
            const int cfg = g > WAVE ? 0 : lane / gg;
            bool hit = false;
            for (int64_t j0 = 0; j0 < n; j0 += WAVE) {
                const int64_t j = j0 + lane;
                float x = INFINITY, y = INFINITY, z = INFINITY;
                if (j < n) {
                    x = pts[3 * j];
                    y = pts[3 * j + 1];
                    z = pts[3 * j + 2];
                }
                const int cnt = (int)min<int64_t>(WAVE, n - j0);
                for (int k = 0; k < cnt; ++k) {
                    const float bx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), k));
                    const float by = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(y), k));
                    const float bz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(z), k));
                    hit = hit || (valid && sqdist(q.x, q.y, q.z, bx, by, bz) <= r2);
                }
                const uint64_t hm = __ballot(hit);
                const bool cdone = valid && (((hm >> (cfg * gg)) & gmask) != 0);
                if (__ballot(valid && !cdone) == 0) break;
            }
            const uint64_t hm = __ballot(hit);
            done = valid && (((hm >> (cfg * gg)) & gmask) != 0);
            any_slice = hm != 0;
        }
        if (g <= WAVE) {
            if (lane < nc * g && lane % g == 0) out[c0 + lane / g] = (uint8_t)done;
        } else if (lane == 0) {
            out[c0] = (uint8_t)any_slice;
        }
    }
}

// Per-sphere work accounting (thread per sphere, not tuned).
__global__ void k_query_stats(CloudDev C, const float4 *__restrict__ sph, int64_t nsph,
                              int32_t *__restrict__ leaf_out, uint8_t *__restrict__ rej_out,
                              int32_t *__restrict__ scanned_out, uint8_t *__restrict__ hit_out) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsph) return;
    const float4 q = sph[s];
    const float r2 = __fmul_rn(q.w, q.w);
    const int64_t N = (int64_t)1 << C.D;
    const uint32_t node = descend(q, nullptr, 0, C.T, C.D, C.axes);
    const uint32_t lf = node - (uint32_t)(N - 1);
    const Leaf L = C.leaf[lf];
    const bool rej = L.count == 0 || box_sqdist(q.x, q.y, q.z, L.lo, L.hi) > r2;
    int32_t m = 0;
    bool hit = false;
    if (!rej) {
        for (uint32_t k = 0; k < L.count && !hit; ++k) {
            ++m;
            const uint32_t e = L.start + k;
            float x, y, z;
            set_point(C, e, x, y, z);
            hit = sqdist(q.x, q.y, q.z, x, y, z) <= r2;
        }
    }
    if (leaf_out) leaf_out[s] = (int32_t)lf;
    if (rej_out) rej_out[s] = (uint8_t)rej;
    if (scanned_out) scanned_out[s] = m;
    if (hit_out) hit_out[s] = (uint8_t)hit;
}

// The two-level scan's work per sphere, in stored order, up to and including
// the chunk that holds the first hit: chunk boxes tested and chunks whose
// entries were scanned (thread per sphere, not tuned).
__global__ void k_chunk_stats(CloudDev C, const float4 *__restrict__ sph, int64_t nsph, int32_t *__restrict__ boxes,
                              int32_t *__restrict__ chunks) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsph) return;
    const float4 q = sph[s];
    const float r2 = __fmul_rn(q.w, q.w);
    const int64_t N = (int64_t)1 << C.D;
    const uint32_t lf = descend(q, nullptr, 0, C.T, C.D, C.axes) - (uint32_t)(N - 1);
    const Leaf L = C.leaf[lf];
    int32_t nb = 0, nc = 0;
    if (L.count > 0 && box_sqdist(q.x, q.y, q.z, L.lo, L.hi) <= r2) {
        bool hit = false;
        const uint32_t c0 = L.start / CHUNK, c1 = c0 + (L.count + CHUNK - 1) / CHUNK;
        for (uint32_t c = c0; c < c1 && !hit; ++c) {
            ++nb;
            float lo[3], hi[3];
            hbox_decode(C.cbox[c], L.lo[0], L.lo[1], L.lo[2], lo, hi);
            if (box_sqdist(q.x, q.y, q.z, lo, hi) > r2) continue;
            ++nc;
            for (uint32_t e = c * CHUNK; e < (c + 1) * CHUNK && !hit; ++e) {
                float x, y, z;
                set_point(C, e, x, y, z);
                hit = sqdist(q.x, q.y, q.z, x, y, z) <= r2;
            }
        }
    }
    if (boxes) boxes[s] = nb;
    if (chunks) chunks[s] = nc;
}

__global__ void k_check_radii(const float4 *__restrict__ sph, int64_t m, float r_min, float r_max, float pad,
                              unsigned int *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned int b = 0;
    for (; i < m; i += stride) {
        const float r = __fadd_rn(sph[i].w, pad);
        b += !(r >= r_min && r <= r_max);
    }
    if (b) atomicAdd(bad, b);
}

}  // namespace

capt_tuning &tuning() {
    static capt_tuning t = {12, 2, 16, 13, 2};
    return t;
}

struct BatchPlan {
    const float *spheres = nullptr;
    uint8_t *out = nullptr;
    int32_t group = 0;
    std::vector<int64_t> qoff;
    capt_tuning tun{};
    Tile *d_tiles = nullptr;
    unsigned int *d_ctr = nullptr;
    int64_t ntiles = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    int32_t *visits = nullptr;   // diagnostic decision counts, or null
};

void free_plan(BatchPlan *p) {
    if (!p) return;
    (void)hipDeviceSynchronize();   // a replay may still read the tile queue
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->d_tiles) dev_free(p->d_tiles, nullptr);
    if (p->d_ctr) dev_free(p->d_ctr, nullptr);
    delete p;
}

namespace {

// Tree levels kept in LDS beside `extra` bytes of per-wave scratch.
int lds_levels_for(int D, size_t extra) {
    int L = std::min(D, std::max(0, std::min(15, (int)tuning().lds_levels)));
    const size_t cap = (size_t)device_info().lds_per_block;
    while (L > 0 && extra + sizeof(float) * (size_t)((1 << L) - 1) > cap) --L;
    return L;
}

// Kernels whose dynamic LDS may exceed 64 KB declare the device maximum once.
template <class K> capt_status allow_lds(K kernel) {
    CAPT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                 device_info().lds_per_block));
    return CAPT_OK;
}

// Launch shape shared by the single-cloud kernels.
struct CloudShape {
    int threads = 0, L = 0;
    int64_t blocks = 0;
    size_t lds = 0;
};

CloudShape cloud_shape(const CloudDev &C, int64_t units) {
    const capt_tuning &t = tuning();
    CloudShape sh;
    sh.threads = WAVE * std::max(1, std::min(16, (int)t.waves_per_group));
    const size_t wl = sizeof(WaveLds) * (size_t)(sh.threads / WAVE);
    sh.L = lds_levels_for(C.D, wl);
    const int64_t wpb = sh.threads / WAVE;
    sh.blocks = (int64_t)device_info().cus * std::max(1, (int)t.groups_per_cu);
    sh.blocks = std::max<int64_t>(1, std::min(sh.blocks, (units + wpb - 1) / wpb));
    sh.lds = wl + sizeof(float) * (size_t)((1 << sh.L) - 1);
    return sh;
}

// queue chunk: about 8 pops per wave over the whole launch, 1 .. 64 units
int queue_chunk(const CloudShape &sh, int64_t units) {
    const int64_t per_wave = units / std::max<int64_t>(1, sh.blocks * (sh.threads / WAVE));
    return (int)std::max<int64_t>(1, std::min<int64_t>(64, per_wave / 8));
}

template <class K> bool allow_lds_once(K k) {
    return allow_lds(k) == CAPT_OK;
}

// Slot kernel over `nitem` items of `len` spheres each.
template <class Src, bool IDX>
capt_status launch_slots_t(const CloudDev &C, Src src, int64_t nitem, int len, uint8_t *out, unsigned int *ctr,
                         hipStream_t s) {
    if (nitem <= 0) return CAPT_OK;
    static const bool lds_ok = allow_lds_once(k_collide_slots<4, Src, IDX>) && allow_lds_once(k_collide_slots<2, Src, IDX>) &&
                               allow_lds_once(k_collide_slots<1, Src, IDX>);
    if (!lds_ok) {
        set_error("raising the dynamic LDS limit of the collision kernel failed");
        return CAPT_EHIP;
    }
    const CloudShape sh = cloud_shape(C, nitem);
    const int chunk = queue_chunk(sh, nitem);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(NXCD * CTR_STRIDE), 0, s, ctr, NXCD * CTR_STRIDE);
    CAPT_LAUNCH_CHECK();
    const dim3 grid((unsigned)sh.blocks), block(sh.threads);
    switch (tuning().scan_unroll) {
        case 4:
            hipLaunchKernelGGL((k_collide_slots<4, Src, IDX>), grid, block, sh.lds, s, C, src, nitem, len, out, sh.L, ctr,
                               chunk);
            break;
        case 2:
            hipLaunchKernelGGL((k_collide_slots<2, Src, IDX>), grid, block, sh.lds, s, C, src, nitem, len, out, sh.L, ctr,
                               chunk);
            break;
        default:
            hipLaunchKernelGGL((k_collide_slots<1, Src, IDX>), grid, block, sh.lds, s, C, src, nitem, len, out, sh.L, ctr,
                               chunk);
            break;
    }
    CAPT_LAUNCH_CHECK();
    return CAPT_OK;
}

template <class Src>
capt_status launch_slots(const CloudDev &C, Src src, int64_t nitem, int len, uint8_t *out, unsigned int *ctr,
                         hipStream_t s) {
    if (C.flags & CAPT_INDEXED_SETS) return launch_slots_t<Src, true>(C, src, nitem, len, out, ctr, s);
    return launch_slots_t<Src, false>(C, src, nitem, len, out, ctr, s);
}

template <bool IDX>
capt_status launch_cloud_t(const CloudDev &C, const float *spheres, int64_t nsph, int32_t g, uint8_t *out,
                         unsigned int *ctr, hipStream_t s) {
    if (nsph <= 0) return CAPT_OK;
    const int64_t ncfg = nsph / g;
    const float4 *sp = reinterpret_cast<const float4 *>(spheres);
    if (g > SLOT) return launch_slots(C, SphereSrc{sp}, ncfg, g, out, ctr, s);   // slots: the queue holds configurations
    static const bool lds_ok = allow_lds_once(k_collide_cloud<4, IDX>) && allow_lds_once(k_collide_cloud<2, IDX>) &&
                               allow_lds_once(k_collide_cloud<1, IDX>);
    if (!lds_ok) {
        set_error("raising the dynamic LDS limit of the collision kernel failed");
        return CAPT_EHIP;
    }
    const int cpt = WAVE / g;
    const int64_t ntiles = (ncfg + cpt - 1) / cpt;
    const CloudShape sh = cloud_shape(C, ntiles);
    const int chunk = queue_chunk(sh, ntiles);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(NXCD * CTR_STRIDE), 0, s, ctr, NXCD * CTR_STRIDE);
    CAPT_LAUNCH_CHECK();
    const dim3 grid((unsigned)sh.blocks), block(sh.threads);
    switch (tuning().scan_unroll) {
        case 4:
            hipLaunchKernelGGL((k_collide_cloud<4, IDX>), grid, block, sh.lds, s, C, sp, nsph, g, out, sh.L, ctr, chunk);
            break;
        case 2:
            hipLaunchKernelGGL((k_collide_cloud<2, IDX>), grid, block, sh.lds, s, C, sp, nsph, g, out, sh.L, ctr, chunk);
            break;
        default:
            hipLaunchKernelGGL((k_collide_cloud<1, IDX>), grid, block, sh.lds, s, C, sp, nsph, g, out, sh.L, ctr, chunk);
            break;
    }
    CAPT_LAUNCH_CHECK();
    return CAPT_OK;
}

capt_status launch_cloud(const CloudDev &C, const float *spheres, int64_t nsph, int32_t g, uint8_t *out,
                         unsigned int *ctr, hipStream_t s) {
    if (C.flags & CAPT_INDEXED_SETS) return launch_cloud_t<true>(C, spheres, nsph, g, out, ctr, s);
    return launch_cloud_t<false>(C, spheres, nsph, g, out, ctr, s);
}

capt_status make_plan(capt_forest_s *f, const float *spheres, const int64_t *qoff, int32_t g, uint8_t *out,
                      BatchPlan *p) {
    const int nc = (int)f->clouds.size();
    const capt_tuning &t = tuning();
    const int tile_cfgs = std::max(1, (int)t.tile_cfgs);
    std::vector<Tile> tiles;
    std::vector<double> cost;
    for (int c = 0; c < nc; ++c) {
        const int64_t c0 = qoff[c] / g, c1 = qoff[c + 1] / g;
        const CloudHost &H = f->clouds[c];
        // per-configuration cost estimate: descent plus a mean set scan
        const double per = (double)H.D + (double)H.set_total / (double)H.N;
        for (int64_t k = c0; k < c1; k += tile_cfgs) {
            Tile tl;
            tl.cloud = c;
            tl.cfg0 = k;
            tl.ncfg = (int32_t)std::min<int64_t>(tile_cfgs, c1 - k);
            tiles.push_back(tl);
            cost.push_back(per * tl.ncfg);
        }
    }
    std::vector<size_t> order(tiles.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    std::vector<Tile> sorted(tiles.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = tiles[order[i]];
    p->ntiles = (int64_t)sorted.size();
    const size_t tb = sizeof(Tile) * std::max<size_t>(1, sorted.size());
    p->d_tiles = static_cast<Tile *>(dev_alloc(tb, nullptr));
    p->d_ctr = static_cast<unsigned int *>(dev_alloc(256, nullptr));
    if (!p->d_tiles || !p->d_ctr) {
        set_error("device allocation for the tile queue failed");
        return CAPT_ENOMEM;
    }
    if (!sorted.empty()) CAPT_HIP(hipMemcpy(p->d_tiles, sorted.data(), sizeof(Tile) * sorted.size(), hipMemcpyHostToDevice));
    p->spheres = spheres;
    p->out = out;
    p->group = g;
    p->qoff.assign(qoff, qoff + nc + 1);
    p->tun = t;
    return CAPT_OK;
}

template <bool IDX>
capt_status enqueue_batched_t(capt_forest_s *f, BatchPlan *p, hipStream_t s) {
    const capt_tuning &t = tuning();
    const int threads = WAVE * std::max(1, std::min(16, (int)t.waves_per_group));
    int64_t blocks = (int64_t)device_info().cus * std::max(1, (int)t.groups_per_cu);
    const int64_t wpb = threads / WAVE;
    blocks = std::max<int64_t>(1, std::min(blocks, (p->ntiles + wpb - 1) / wpb));
    const size_t lds = (sizeof(WaveLds) + sizeof(float) * ((size_t)1 << BATCH_TOP)) * (size_t)wpb;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, p->d_ctr);
    CAPT_LAUNCH_CHECK();
    if (p->ntiles > 0) {
        const float4 *sp = reinterpret_cast<const float4 *>(p->spheres);
        switch (t.scan_unroll) {
            case 4:
                hipLaunchKernelGGL((k_collide_batched<4, IDX>), dim3((unsigned)blocks), dim3(threads), lds, s, f->d_clouds,
                                   p->d_tiles, p->ntiles, p->d_ctr, sp, p->group, p->out, p->visits);
                break;
            case 2:
                hipLaunchKernelGGL((k_collide_batched<2, IDX>), dim3((unsigned)blocks), dim3(threads), lds, s, f->d_clouds,
                                   p->d_tiles, p->ntiles, p->d_ctr, sp, p->group, p->out, p->visits);
                break;
            default:
                hipLaunchKernelGGL((k_collide_batched<1, IDX>), dim3((unsigned)blocks), dim3(threads), lds, s, f->d_clouds,
                                   p->d_tiles, p->ntiles, p->d_ctr, sp, p->group, p->out, p->visits);
                break;
        }
        CAPT_LAUNCH_CHECK();
    }
    return CAPT_OK;
}

capt_status enqueue_batched(capt_forest_s *f, BatchPlan *p, hipStream_t s) {
    if (f->flags & CAPT_INDEXED_SETS) return enqueue_batched_t<true>(f, p, s);
    return enqueue_batched_t<false>(f, p, s);
}

bool same_tuning(const capt_tuning &a, const capt_tuning &b) {
    return a.waves_per_group == b.waves_per_group && a.groups_per_cu == b.groups_per_cu &&
           a.tile_cfgs == b.tile_cfgs && a.lds_levels == b.lds_levels && a.scan_unroll == b.scan_unroll;
}

}  // namespace

capt_status check_radii(const float *spheres, int64_t m, float r_min, float r_max, hipStream_t s, float pad) {
    if (m <= 0) return CAPT_OK;
    Scratch sc;
    if (!sc.alloc(256, s)) {
        set_error("device allocation failed");
        return CAPT_ENOMEM;
    }
    CAPT_HIP(hipMemsetAsync(sc.p, 0, 4, s));
    const int64_t blocks = std::min<int64_t>((m + 255) / 256, 4096);
    hipLaunchKernelGGL(k_check_radii, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<const float4 *>(spheres), m, r_min, r_max, pad, sc.as<unsigned int>());
    CAPT_LAUNCH_CHECK();
    unsigned int bad = 0;
    CAPT_HIP(hipMemcpyAsync(&bad, sc.p, 4, hipMemcpyDeviceToHost, s));
    CAPT_HIP(hipStreamSynchronize(s));
    if (bad) {
        set_error("%u query radii (after padding by %g) lie outside [r_min, r_max] = [%g, %g]", bad, (double)pad,
                  (double)r_min, (double)r_max);
        return CAPT_ERADIUS;
    }
    return CAPT_OK;
}

capt_status collides(capt_forest_s *f, const float *spheres, const int64_t *qoff, int32_t g, uint8_t *out,
                     uint32_t flags, hipStream_t s) {
    const int nc = (int)f->clouds.size();
    if (flags & CAPT_CHECK_RADII) {
        capt_status st = check_radii(spheres, qoff[nc], f->r_min, f->r_max, s);
        if (st) return st;
    }
    bool cyclic = true;   // the batched kernel takes forests with the cyclic split axes only
    for (int c = 0; c < nc; ++c) cyclic = cyclic && f->clouds[c].dev.cyclic;
    if (nc == 1 || (flags & CAPT_PER_CLOUD) || !cyclic) {
        // queue counters, one set per cloud so launches on the stream never share them
        Scratch ctr;
        if (!ctr.alloc(sizeof(unsigned int) * NXCD * CTR_STRIDE * (size_t)nc, s)) {
            set_error("device allocation for queue counters failed");
            return CAPT_ENOMEM;
        }
        for (int c = 0; c < nc; ++c) {
            const int64_t m = qoff[c + 1] - qoff[c];
            capt_status st = launch_cloud(f->clouds[c].dev, spheres + 4 * qoff[c], m, g, out + qoff[c] / g,
                                          ctr.as<unsigned int>() + (size_t)c * NXCD * CTR_STRIDE, s);
            if (st) return st;
        }
        return CAPT_OK;
    }
    capt_status vs = ensure_views(f, s);
    if (vs) return vs;
    BatchPlan *p = f->plan;
    const bool reuse = p && p->spheres == spheres && p->out == out && p->group == g &&
                       std::equal(p->qoff.begin(), p->qoff.end(), qoff) && same_tuning(p->tun, tuning());
    if (!reuse) {
        free_plan(f->plan);
        f->plan = nullptr;
        p = new BatchPlan();
        capt_status st = make_plan(f, spheres, qoff, g, out, p);
        if (st) {
            free_plan(p);
            return st;
        }
        f->plan = p;
    }
    if (flags & CAPT_NO_GRAPH) return enqueue_batched(f, p, s);
    if (!p->exec) {
        CAPT_HIP(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
        CAPT_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
        capt_status st = enqueue_batched(f, p, p->cap);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(p->cap, &graph);
        if (st) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        CAPT_HIP(e);
        p->graph = graph;
        CAPT_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    }
    CAPT_HIP(hipGraphLaunch(p->exec, s));
    return CAPT_OK;
}

// The batched launch of capt_collides on a plan of its own (no graph, not
// cached) whose kernel also counts, per configuration, how often it decides it.
capt_status collides_visits(capt_forest_s *f, const float *spheres, const int64_t *qoff, int32_t g, uint8_t *out,
                            int32_t *visits, hipStream_t s) {
    for (const CloudHost &H : f->clouds) {
        if (!H.dev.cyclic) {
            set_error("the batched query takes forests with the cyclic split axes only");
            return CAPT_EUNSUPPORTED;
        }
    }
    capt_status st = ensure_views(f, s);
    if (st) return st;
    BatchPlan *p = new BatchPlan();
    st = make_plan(f, spheres, qoff, g, out, p);
    if (!st) {
        p->visits = visits;
        st = enqueue_batched(f, p, s);
    }
    if (!st) CAPT_HIP(hipStreamSynchronize(s));
    free_plan(p);
    return st;
}

// Queue counters of capt_collides_noalloc: one set of NXCD counters (a
// 64-byte line each) per cloud.  Host code never passes this array's name to a
// kernel (on the host it is only a stand-in for the symbol); the launches take
// the device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned int scratch[CAPT_NOALLOC_MAX_CLOUDS * NXCD * CTR_STRIDE];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned int *g_scratch_dev[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per device.
capt_status scratch_address(unsigned int **out) {
    int dev = 0;
    CAPT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("device ordinal %d beyond the %d the library tracks", dev, MAX_DEVICES);
        return CAPT_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            set_error("hipGetSymbolAddress of the query counters failed: %s", hipGetErrorString(e));
            return CAPT_EHIP;
        }
        g_scratch_dev[dev] = static_cast<unsigned int *>(ptr);
    }
    *out = g_scratch_dev[dev];
    return CAPT_OK;
}
}  // namespace

capt_status collides_noalloc(capt_forest_s *f, const float *spheres, const int64_t *qoff, int32_t g, uint8_t *out,
                             hipStream_t s) {
    const int nc = (int)f->clouds.size();
    if (nc > CAPT_NOALLOC_MAX_CLOUDS) {
        set_error("forest of %d clouds: the allocation-free query takes at most %d", nc, CAPT_NOALLOC_MAX_CLOUDS);
        return CAPT_EUNSUPPORTED;
    }
    unsigned int *ctr = nullptr;
    capt_status st = scratch_address(&ctr);
    if (st) return st;
    for (int c = 0; c < nc; ++c) {
        const int64_t m = qoff[c + 1] - qoff[c];
        st = launch_cloud(f->clouds[c].dev, spheres + 4 * qoff[c], m, g, out + qoff[c] / g,
                          ctr + (size_t)c * NXCD * CTR_STRIDE, s);
        if (st) return st;
    }
    return CAPT_OK;
}

capt_status collides_posed(capt_forest_s *f, const float *tmpl, int32_t g, const float *poses, const int64_t *poff,
                           int32_t edge, uint8_t *out, uint32_t flags, hipStream_t s) {
    const int nc = (int)f->clouds.size();
    if (flags & CAPT_CHECK_RADII) {
        capt_status st = check_radii(tmpl, g, f->r_min, f->r_max, s);
        if (st) return st;
    }
    Scratch ctr;
    if (!ctr.alloc(sizeof(unsigned int) * NXCD * CTR_STRIDE * (size_t)nc, s)) {
        set_error("device allocation for queue counters failed");
        return CAPT_ENOMEM;
    }
    for (int c = 0; c < nc; ++c) {
        const int64_t np = poff[c + 1] - poff[c];
        if (np <= 0) continue;
        PosedSrc src{poses + 12 * poff[c], reinterpret_cast<const float4 *>(tmpl), g};
        capt_status st = launch_slots(f->clouds[c].dev, src, np / edge, edge * g, out + poff[c] / edge,
                                      ctr.as<unsigned int>() + (size_t)c * NXCD * CTR_STRIDE, s);
        if (st) return st;
    }
    return CAPT_OK;
}

capt_status collides_padded(capt_forest_s *f, const float *spheres, const int64_t *qoff, int32_t g, float pad,
                            uint8_t *out, uint32_t flags, hipStream_t s) {
    const int nc = (int)f->clouds.size();
    if (flags & CAPT_CHECK_RADII) {
        capt_status st = check_radii(spheres, qoff[nc], f->r_min, f->r_max, s, pad);
        if (st) return st;
    }
    Scratch ctr;
    if (!ctr.alloc(sizeof(unsigned int) * NXCD * CTR_STRIDE * (size_t)nc, s)) {
        set_error("device allocation for queue counters failed");
        return CAPT_ENOMEM;
    }
    // every group size goes through the slot kernel (one cloud per launch)
    for (int c = 0; c < nc; ++c) {
        const int64_t m = qoff[c + 1] - qoff[c];
        if (m <= 0) continue;
        PaddedSrc src{reinterpret_cast<const float4 *>(spheres) + qoff[c], pad};
        capt_status st = launch_slots(f->clouds[c].dev, src, m / g, g, out + qoff[c] / g,
                                      ctr.as<unsigned int>() + (size_t)c * NXCD * CTR_STRIDE, s);
        if (st) return st;
    }
    return CAPT_OK;
}

capt_status query_stats(capt_forest_s *f, const float *spheres, const int64_t *qoff, int32_t *leaf,
                        uint8_t *rejected, int32_t *scanned, uint8_t *hit, hipStream_t s) {
    const int nc = (int)f->clouds.size();
    for (int c = 0; c < nc; ++c) {
        const int64_t m = qoff[c + 1] - qoff[c];
        if (m <= 0) continue;
        const int64_t o = qoff[c];
        hipLaunchKernelGGL(k_query_stats, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, f->clouds[c].dev,
                           reinterpret_cast<const float4 *>(spheres + 4 * o), m, leaf ? leaf + o : nullptr,
                           rejected ? rejected + o : nullptr, scanned ? scanned + o : nullptr,
                           hit ? hit + o : nullptr);
        CAPT_LAUNCH_CHECK();
    }
    return CAPT_OK;
}

capt_status chunk_stats(capt_forest_s *f, const float *spheres, const int64_t *qoff, int32_t *boxes, int32_t *chunks,
                        hipStream_t s) {
    const int nc = (int)f->clouds.size();
    for (int c = 0; c < nc; ++c) {
        const int64_t m = qoff[c + 1] - qoff[c];
        if (m <= 0) continue;
        const int64_t o = qoff[c];
        hipLaunchKernelGGL(k_chunk_stats, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, f->clouds[c].dev,
                           reinterpret_cast<const float4 *>(spheres + 4 * o), m, boxes ? boxes + o : nullptr,
                           chunks ? chunks + o : nullptr);
        CAPT_LAUNCH_CHECK();
    }
    return CAPT_OK;
}

capt_status bruteforce(const float *xyz, const int64_t *cloud_off, int32_t ncloud, const float *spheres,
                       const int64_t *qoff, int32_t g, uint8_t *out, hipStream_t s) {
    for (int c = 0; c < ncloud; ++c) {
        const int64_t m = qoff[c + 1] - qoff[c];
        if (m <= 0) continue;
        const int64_t n = cloud_off[c + 1] - cloud_off[c];
        const int64_t ncfg = m / g;
        const int cpt = g <= WAVE ? WAVE / g : 1;
        const int64_t ntiles = (ncfg + cpt - 1) / cpt;
        const int threads = 256;
        int64_t blocks = std::min<int64_t>((ntiles + 3) / 4, (int64_t)device_info().cus * 8);
        blocks = std::max<int64_t>(blocks, 1);
        hipLaunchKernelGGL(k_brute, dim3((unsigned)blocks), dim3(threads), 0, s, xyz + 3 * cloud_off[c], n,
                           reinterpret_cast<const float4 *>(spheres + 4 * qoff[c]), m, g, out + qoff[c] / g);
        CAPT_LAUNCH_CHECK();
    }
    return CAPT_OK;
}

}  // namespace capt
