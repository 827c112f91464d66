// Internal declarations of the CAPT HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/capt.h"

namespace capt {

constexpr int WAVE = 64;

// One leaf record: float32 bounding box of the stored set, then the set's
// first entry and length in the per-cloud SoA arrays.  32 bytes, so one leaf
// is two 16-byte loads.
struct alignas(16) Leaf {
    float lo[3];
    float hi[3];
    uint32_t start;
    uint32_t count;
};
static_assert(sizeof(Leaf) == 32, "leaf record is 32 bytes");

// Per-cloud view of a forest, resident in device memory for the batched
// kernel and passed by value to the single-cloud kernels.
struct CloudDev {
    const float *T;        // [N-1] split values, Eytzinger order
    const float4 *tb;      // 4-level blocks of the lower levels (tree_blocks), or NULL
    const Leaf *leaf;      // [N]
    const float *px;       // set entries: x, y, z blocks of every 16-entry chunk (set_off)
    const float *py;       // px + 16
    const float *pz;       // px + 32
    const int32_t *pidx;   // original index of each set entry (-1 = padding)
    const uint4 *cbox;     // per 16-entry chunk of the sets: its box, half-precision (hbox_encode)
    const float *pts;      // [n][3] the cloud as built
    int64_t n;
    int32_t D;
    uint32_t flags;
    uint64_t axes;         // split axis of depth d in bits 2d, 2d+1
    int32_t cyclic;        // axes follow d mod 3 (the kernels' fast descent)
};

// Split-axis code of a forest: bits 2d, 2d+1 hold the axis of depth d.
// axes == NULL gives the cyclic rule d mod 3.
inline uint64_t axes_code(const uint8_t *axes, int D) {
    uint64_t c = 0;
    for (int d = 0; d < D && d < 32; ++d) c |= (uint64_t)(axes ? axes[d] : (uint8_t)(d % 3)) << (2 * d);
    return c;
}
__host__ __device__ __forceinline__ int axis_at(uint64_t code, int d) { return (int)((code >> (2 * d)) & 3u); }

// Blocked copy of a tree's lower levels: for every node i at a root level
// r = D - 4k (k >= 1), the 15 split values of its 4-level subtree in
// breadth-first order (i; 2i+1, 2i+2; 4i+3 .. 4i+6; 8i+7 .. 8i+14) and one
// pad, 64 bytes, so a descent reads four levels from one cache line.  Blocks
// go by root level, shallowest first, then by node; those of root level r
// start at block tree_block_base(r, D).  Built for 4 <= D <= 29 (the query
// addresses them with 32-bit byte offsets).
__host__ __device__ __forceinline__ uint32_t tree_block_base(int r, int D) {
    return (uint32_t)((((uint64_t)1 << r) - ((uint64_t)1 << (D & 3))) / 15u);
}
inline int64_t tree_blocks_count(int D) {
    return (D >= 4 && D <= 29) ? (int64_t)tree_block_base(D, D) : 0;
}

// Stored-set alignment: every set starts at a multiple of this many entries
// and is padded with +inf entries up to one.  A chunk of SET_ALIGN entries is
// also the unit of the second-level bounding boxes the query scan tests.
constexpr uint32_t SET_ALIGN = 16;
constexpr uint32_t CHUNK = SET_ALIGN;
// Set entries are stored per chunk of CHUNK entries as structure of arrays:
// chunk k holds its 16 x values, then its 16 y, then its 16 z (192 bytes), so
// the coordinates of one chunk sit in two 128-byte cache lines.  With px the x
// block of chunk 0, py = px + 16 and pz = px + 32, the coordinate of entry e
// is at float offset set_off(e) from each.
__host__ __device__ __forceinline__ int64_t set_off(int64_t e) { return 48 * (e >> 4) + (e & 15); }

// The box of every 16-entry chunk is stored in 16 bytes: per axis, the lower
// and upper bound as half-precision offsets from the lower corner of the
// set's own box (the leaf AABB), rounded outward so that the box decoded in
// float32, base + (float)offset, contains every point of the chunk.  A decoded
// box may only be larger than the exact one, so the scan's test on it never
// skips a chunk that holds a hit.  Layout: offsets lo x, y, z, hi x, y, z, two
// unused halves.
__host__ __device__ __forceinline__ float h2f(uint32_t h) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}
// Offset of v >= base: the nearest half, then moved down (up) one half at a
// time until base + offset <= v (>= v) holds in float32.
__host__ __device__ inline uint32_t hbox_offset(float base, float v, bool up) {
    const float d = v - base;
    uint32_t h = __builtin_bit_cast(uint16_t, (_Float16)d);   // d >= 0: 0 .. 0x7C00 (+inf)
    if (up) {
        for (int it = 0; it < 8 && base + h2f(h) < v; ++it) h = h < 0x7C00u ? h + 1u : h;
        if (base + h2f(h) < v) h = 0x7C00u;
    } else {
        for (int it = 0; it < 8 && base + h2f(h) > v; ++it) h = h > 0u ? h - 1u : 0u;
        if (base + h2f(h) > v) h = 0u;
    }
    return h;
}
__host__ __device__ inline uint4 hbox_encode(const float base[3], const float lo[3], const float hi[3]) {
    uint32_t o[6];
    for (int a = 0; a < 3; ++a) {
        o[a] = hbox_offset(base[a], lo[a], false);
        o[3 + a] = hbox_offset(base[a], hi[a], true);
    }
    return make_uint4(o[0] | (o[1] << 16), o[2] | (o[3] << 16), o[4] | (o[5] << 16), 0u);
}
__device__ __forceinline__ void hbox_decode(uint4 b, float bx, float by, float bz, float lo[3], float hi[3]) {
    lo[0] = bx + h2f(b.x & 0xFFFFu);
    lo[1] = by + h2f(b.x >> 16);
    lo[2] = bz + h2f(b.y & 0xFFFFu);
    hi[0] = bx + h2f(b.y >> 16);
    hi[1] = by + h2f(b.z & 0xFFFFu);
    hi[2] = bz + h2f(b.z >> 16);
}

// Stored set entries per cloud (with padding) stay below this, so the query
// kernels address the set arrays with 32-bit byte offsets.
constexpr unsigned long long MAX_SET_ENTRIES = 1ull << 30;
// Largest configuration (spheres per group) a query accepts.
constexpr int32_t MAX_GROUP = 1 << 20;

// ---------------------------------------------------------------------------
// Host-side error state and helpers (api.hip)
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
capt_status hip_fail(hipError_t e, const char *what, const char *file, int line);
void *dev_alloc(size_t bytes, hipStream_t s);
bool default_allocator();   // no caller hooks installed (the pool is safe to use from several threads)
void dev_free(void *p, hipStream_t s);

#define CAPT_HIP(call)                                                          \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) return ::capt::hip_fail(e_, #call, __FILE__, __LINE__); \
    } while (0)

#define CAPT_LAUNCH_CHECK() CAPT_HIP(hipGetLastError())

// RAII scratch buffer from the configured allocator.
struct Scratch {
    void *p = nullptr;
    hipStream_t s = nullptr;
    Scratch() = default;
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
    ~Scratch() { release(); }
    bool alloc(size_t bytes, hipStream_t st) {
        release();
        s = st;
        p = dev_alloc(bytes ? bytes : 16, st);
        return p != nullptr;
    }
    void release() {
        if (p) dev_free(p, s);
        p = nullptr;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Pinned host memory for the few words a call reads back before it returns:
// the last kernel of the call stores them straight into this memory and the
// host waits on the stream, with no copy.  Blocks come from a process-wide
// cache (allocated once, kept until the process ends).
void *pinned_acquire(size_t bytes);
void pinned_release(void *p, size_t bytes);
struct Pinned {
    void *p = nullptr;
    size_t n = 0;
    Pinned() = default;
    Pinned(const Pinned &) = delete;
    Pinned &operator=(const Pinned &) = delete;
    ~Pinned() {
        if (p) pinned_release(p, n);
    }
    bool alloc(size_t bytes) {
        n = bytes;
        p = pinned_acquire(bytes);
        return p != nullptr;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Fork-join of a library-owned side stream inside one call: fork() makes the
// side stream wait for the work queued on s so far, join() makes s wait for
// the side stream's work.  A ForkJoin that is still forked joins on
// destruction (so stream-ordered releases on s come after the side work).
// Side streams and events come from a process-wide pool, one context per
// concurrent user.
struct ForkJoin {
    hipStream_t side = nullptr;
    hipStream_t main = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int dev = -1;
    bool forked = false;
    ForkJoin() = default;
    ForkJoin(const ForkJoin &) = delete;
    ForkJoin &operator=(const ForkJoin &) = delete;
    ~ForkJoin();
    capt_status fork(hipStream_t s);
    capt_status join(hipStream_t s);
};

// Device properties used for launch planning.
struct DeviceInfo {
    int cus = 256;
    int lds_per_block = 65536;
};
const DeviceInfo &device_info();

// ---------------------------------------------------------------------------
// Primitives (primitives.hip)
// ---------------------------------------------------------------------------
// Exclusive prefix sum of n uint32 values (n may be given on the device
// through n_dev, in which case `n` is only the capacity).  out may alias in.
// total (device, may be NULL) receives the sum.  tmp must hold
// scan_tmp_words(n) uint32 words.
size_t scan_tmp_words(int64_t n);
capt_status scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n,
                               const int64_t *n_dev, uint32_t *total, uint32_t *tmp,
                               hipStream_t s);

// One-pass exclusive scan by decoupled look-back (sums below 2^30): status
// holds scan_lb_words(n) words the caller zeroed; err is an error word (bit 16
// set if an internal wait bound was hit).
size_t scan_lb_words(int64_t n);
capt_status scan_exclusive_u32_lb(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *status, uint32_t *err,
                                  hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by the low `bits` bits of the
// key (n < 2^30).  Keys/values ping-pong between the two buffers; *where tells
// whether the result is in (k0, v0) (0) or (k1, v1) (1).  tmp must hold
// radix_tmp_words(n) words; tmp[0] is an error word the caller clears before
// and checks after (non-zero: an internal wait bound was hit).
size_t radix_tmp_words(int64_t n);
capt_status radix_sort_u64(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n,
                           int bits, uint32_t *tmp, hipStream_t s, int *where);
// Segmented form: nseg (<= 8) lists of len keys each, sorted independently in
// the same launches; tmp holds radix_tmp_words_seg(nseg, len) words.
size_t radix_tmp_words_seg(int nseg, int64_t len);
capt_status radix_sort_u64_seg(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int nseg, int64_t len,
                               int bits, uint32_t *tmp, hipStream_t s, int *where);
// cleared: words tmp[64 .. 64 + radix_clear_words(nseg, len, bits)) are zero
// already (the caller cleared them in a kernel of its own), so the sort skips
// its clearing launch.
capt_status radix_sort_u32_seg(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int nseg, int64_t len,
                               int bits, uint32_t *tmp, hipStream_t s, int *where, bool cleared = false);
capt_status radix_sort_u32(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n,
                           int bits, uint32_t *tmp, hipStream_t s, int *where, bool cleared = false);
int64_t radix_clear_words(int nseg, int64_t len, int bits);

// ---------------------------------------------------------------------------
// Forest (api.hip / build.hip)
// ---------------------------------------------------------------------------
struct CloudHost {
    int64_t n = 0;
    int64_t N = 1;
    int32_t D = 0;
    int64_t set_total = 0;     // stored entries without padding
    int64_t set_padded = 0;    // stored entries with padding
    int64_t pruned = 0;
    void *fixed = nullptr;     // T, leaves, pts, rep, pruned flags
    void *sets = nullptr;      // px, py, pz, pidx, chunk boxes
    size_t fixed_bytes = 0;
    size_t sets_bytes = 0;
    CloudDev dev{};
    int32_t *rep = nullptr;    // device [N]
    uint8_t *pruned_flag = nullptr;  // device [N]
};

struct BatchPlan;

}  // namespace capt

struct capt_forest_s {
    std::vector<capt::CloudHost> clouds;
    capt::CloudDev *d_clouds = nullptr;   // device copy of every cloud's view
    float r_min = 0.f, r_max = 0.f;
    uint32_t flags = 0;
    int64_t pruned_total = 0;
    capt::BatchPlan *plan = nullptr;      // cached batched launch (query.hip)
};

namespace capt {

// build.hip
// axes: host [D] split axis per depth (0, 1, 2) or NULL for d mod 3.
// shard_bits, shard: only the leaves l with floor(l 2^shard_bits / N) = shard
// get affordance sets (0, 0: every leaf).
capt_status build_forest(const float *xyz, const int64_t *cloud_off, int32_t ncloud,
                         float r_min, float r_max, uint32_t flags, const uint8_t *axes, int shard_bits,
                         int shard, hipStream_t s, capt_forest_s *f);
void free_cloud(CloudHost &c, hipStream_t s);
capt_status upload_views(capt_forest_s *f, hipStream_t s);
capt_status ensure_views(capt_forest_s *f, hipStream_t s);   // per-cloud views on the device (batched kernel)
// Bytes of the sets block for `entries` padded entries and its sub-arrays.
// indexed: no coordinate arrays (px, py, pz come back NULL).
size_t sets_bytes(size_t entries, bool indexed);
void sets_layout(void *base, size_t entries, bool indexed, float **px, float **py, float **pz, int32_t **pidx,
                 uint4 **cbox);

// query.hip
capt_status collides(capt_forest_s *f, const float *spheres, const int64_t *query_off,
                     int32_t group, uint8_t *out, uint32_t flags, hipStream_t s);
// the same answers with the queue counters in the library's static device array
capt_status collides_noalloc(capt_forest_s *f, const float *spheres, const int64_t *query_off, int32_t group,
                             uint8_t *out, hipStream_t s);
// the batched launch with per-configuration decision counts (diagnostic)
capt_status collides_visits(capt_forest_s *f, const float *spheres, const int64_t *query_off, int32_t group,
                            uint8_t *out, int32_t *visits, hipStream_t s);
capt_status collides_posed(capt_forest_s *f, const float *tmpl, int32_t g, const float *poses, const int64_t *pose_off,
                           int32_t edge, uint8_t *out, uint32_t flags, hipStream_t s);
capt_status query_stats(capt_forest_s *f, const float *spheres, const int64_t *query_off,
                        int32_t *leaf, uint8_t *rejected, int32_t *scanned, uint8_t *hit, hipStream_t s);
capt_status chunk_stats(capt_forest_s *f, const float *spheres, const int64_t *query_off, int32_t *boxes,
                        int32_t *chunks, hipStream_t s);
capt_status bruteforce(const float *xyz, const int64_t *cloud_off, int32_t ncloud,
                       const float *spheres, const int64_t *query_off, int32_t group,
                       uint8_t *out, hipStream_t s);
capt_status check_radii(const float *spheres, int64_t m, float r_min, float r_max, hipStream_t s, float pad = 0.0f);
capt_status collides_padded(capt_forest_s *f, const float *spheres, const int64_t *query_off, int32_t group, float pad,
                            uint8_t *out, uint32_t flags, hipStream_t s);
void free_plan(BatchPlan *p);
capt_tuning &tuning();

// probe.hip
capt_status probe_read(const void *buf, size_t bytes, int32_t passes, int32_t blocks_per_cu, float *sink,
                       hipStream_t s);
capt_status probe_gather(const int32_t *items, int64_t m, const void *leaves, int64_t nleaf, const float *x,
                         const float *y, const float *z, int64_t entries, int32_t lanes_per_item, uint8_t *out,
                         hipStream_t s);

// build.hip: the blocked copy of T's lower levels (tree_blocks_count(D) blocks)
capt_status tree_blocks(const float *T, int D, float4 *tb, hipStream_t s);

// clearance.hip
capt_status clearance_fwd(capt_forest_s *f, const float *spheres, const int64_t *query_off,
                          float *clr, int32_t *witness, hipStream_t s);
capt_status clearance_bwd(capt_forest_s *f, const float *spheres, const int64_t *query_off,
                          const int32_t *witness, const float *grad, float *grad_center, float *grad_radius,
                          hipStream_t s);

// filter.hip
// crop: host [4] (base x, y, z, reach) or NULL
capt_status filter(const float *xyz, int64_t n, float r_filter, const float *crop, float *out_xyz,
                   int32_t *out_index, int64_t *n_out, hipStream_t s);

// ---------------------------------------------------------------------------
// Device helpers shared by the kernels of this library
// ---------------------------------------------------------------------------
// The float32 sphere-point predicate: ((dx*dx + dy*dy) + dz*dz) <= r*r,
// every operation rounded on its own (the library is compiled with
// -ffp-contract=off; the explicit _rn intrinsics make the intent visible).
__device__ __forceinline__ float sqdist(float ax, float ay, float az, float bx, float by,
                                        float bz) {
    float dx = __fsub_rn(ax, bx);
    float dy = __fsub_rn(ay, by);
    float dz = __fsub_rn(az, bz);
    float s = __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy));
    return __fadd_rn(s, __fmul_rn(dz, dz));
}

// Squared distance from a point to a float32 box, with the same rounding
// order as sqdist (so it never exceeds sqdist to any point inside the box).
__device__ __forceinline__ float box_sqdist(float x, float y, float z, const float lo[3],
                                            const float hi[3]) {
    float gx = fmaxf(fmaxf(__fsub_rn(lo[0], x), __fsub_rn(x, hi[0])), 0.0f);
    float gy = fmaxf(fmaxf(__fsub_rn(lo[1], y), __fsub_rn(y, hi[1])), 0.0f);
    float gz = fmaxf(fmaxf(__fsub_rn(lo[2], z), __fsub_rn(z, hi[2])), 0.0f);
    float s = __fadd_rn(__fmul_rn(gx, gx), __fmul_rn(gy, gy));
    return __fadd_rn(s, __fmul_rn(gz, gz));
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Coordinates of set entry e: from the set arrays, or (indexed sets) from the
// forest's point table; padding entries read as +inf either way.
__device__ __forceinline__ void set_point(const CloudDev &C, int64_t e, float &x, float &y, float &z) {
    if (C.flags & CAPT_INDEXED_SETS) {
        const int32_t id = C.pidx[e];
        if (id < 0) {
            x = y = z = INFINITY;
        } else {
            x = C.pts[3 * (int64_t)id];
            y = C.pts[3 * (int64_t)id + 1];
            z = C.pts[3 * (int64_t)id + 2];
        }
    } else {
        const int64_t o = set_off(e);
        x = C.px[o];
        y = C.py[o];
        z = C.pz[o];
    }
}

}  // namespace capt
