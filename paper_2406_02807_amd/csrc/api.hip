// C ABI of the CAPT library: argument checks, error state, allocator hooks,
// forest lifetime, import/export, and dispatch to the kernels.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "capt_internal.h"

namespace capt {

namespace {
thread_local char g_err[512] = "";

struct Allocator {
    void *(*alloc)(size_t, void *, void *) = nullptr;
    void (*release)(void *, void *, void *) = nullptr;
    void *ctx = nullptr;
};
Allocator g_alloc;

struct ApiGuard {
    ApiGuard() { g_err[0] = 0; }
};
}  // namespace

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

capt_status hip_fail(hipError_t e, const char *what, const char *file, int line) {
    set_error("%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    return e == hipErrorOutOfMemory ? CAPT_ENOMEM : CAPT_EHIP;
}

namespace {
// The default allocator is the device's stream-ordered pool; its release
// threshold is raised once per device so freed blocks stay cached for the
// next build instead of going back to the driver.
void keep_pool_cached() {
    static std::mutex mu;
    static bool done[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
    std::lock_guard<std::mutex> lock(mu);
    if (done[dev]) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        // never reuse a block whose free on another stream has not completed
        // yet: the pool would make this allocation's stream wait for that
        // stream's work (a frame's build behind the previous frame's query)
        int no = 0;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolReuseAllowInternalDependencies, &no);
    }
    (void)hipGetLastError();
    done[dev] = true;
}
}  // namespace

void *dev_alloc(size_t bytes, hipStream_t s) {
    if (g_alloc.alloc) return g_alloc.alloc(bytes, s, g_alloc.ctx);
    keep_pool_cached();
    void *p = nullptr;
    if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

bool default_allocator() { return g_alloc.alloc == nullptr; }

void dev_free(void *p, hipStream_t s) {
    if (!p) return;
    if (g_alloc.release) {
        g_alloc.release(p, s, g_alloc.ctx);
        return;
    }
    (void)hipFreeAsync(p, s);
}

namespace {
std::mutex g_pinned_mu;
std::vector<std::pair<size_t, void *>> g_pinned_free;   // (size class, block)
size_t pinned_class(size_t b) {
    size_t c = 256;
    while (c < b) c <<= 1;
    return c;
}
}  // namespace

void *pinned_acquire(size_t bytes) {
    const size_t c = pinned_class(bytes);
    {
        std::lock_guard<std::mutex> lock(g_pinned_mu);
        for (size_t i = 0; i < g_pinned_free.size(); ++i)
            if (g_pinned_free[i].first == c) {
                void *p = g_pinned_free[i].second;
                g_pinned_free[i] = g_pinned_free.back();
                g_pinned_free.pop_back();
                return p;
            }
    }
    // coherent: kernel stores reach host memory without a cache flush
    void *p = nullptr;
    if (hipHostMalloc(&p, c, hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void pinned_release(void *p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_pinned_mu);
    g_pinned_free.emplace_back(pinned_class(bytes), p);
}

namespace {
struct SideCtx {
    int dev;
    hipStream_t side;
    hipEvent_t e1, e2;
};
std::mutex g_side_mu;
std::vector<SideCtx> g_side_free;
}  // namespace

capt_status ForkJoin::fork(hipStream_t s) {
    CAPT_HIP(hipGetDevice(&dev));
    bool have = false;
    {
        std::lock_guard<std::mutex> lock(g_side_mu);
        for (size_t i = 0; i < g_side_free.size(); ++i)
            if (g_side_free[i].dev == dev) {
                side = g_side_free[i].side;
                ev_fork = g_side_free[i].e1;
                ev_join = g_side_free[i].e2;
                g_side_free[i] = g_side_free.back();
                g_side_free.pop_back();
                have = true;
                break;
            }
    }
    if (!have) {
        // default priority, no implicit ordering with the null stream
        CAPT_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
        CAPT_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
        CAPT_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
    }
    main = s;
    CAPT_HIP(hipEventRecord(ev_fork, s));
    CAPT_HIP(hipStreamWaitEvent(side, ev_fork, 0));
    forked = true;
    return CAPT_OK;
}

capt_status ForkJoin::join(hipStream_t s) {
    if (!forked) return CAPT_OK;
    forked = false;
    CAPT_HIP(hipEventRecord(ev_join, side));
    CAPT_HIP(hipStreamWaitEvent(s, ev_join, 0));
    return CAPT_OK;
}

ForkJoin::~ForkJoin() {
    if (!side) return;
    if (forked && (join(main) != CAPT_OK)) (void)hipStreamSynchronize(side);
    std::lock_guard<std::mutex> lock(g_side_mu);
    g_side_free.push_back({dev, side, ev_fork, ev_join});
}

const DeviceInfo &device_info() {
    static DeviceInfo info;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return;
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) return;
        info.cus = p.multiProcessorCount > 0 ? p.multiProcessorCount : 256;
        info.lds_per_block = p.sharedMemPerBlock > 0 ? (int)p.sharedMemPerBlock : 65536;
        if (info.lds_per_block > 163840) info.lds_per_block = 163840;
    });
    return info;
}

}  // namespace capt

using namespace capt;

namespace {

bool finite_f(float v) { return std::isfinite(v); }

capt_status check_offsets(const int64_t *off, int32_t count, const char *name) {
    if (!off) {
        set_error("%s is NULL", name);
        return CAPT_EINVAL;
    }
    if (off[0] != 0) {
        set_error("%s[0] = %lld, expected 0", name, (long long)off[0]);
        return CAPT_EINVAL;
    }
    for (int32_t c = 0; c < count; ++c)
        if (off[c + 1] < off[c]) {
            set_error("%s decreases at %d", name, c);
            return CAPT_EINVAL;
        }
    return CAPT_OK;
}

capt_status check_queries(capt_forest f, const float *spheres, const int64_t *qoff, int32_t group) {
    if (!f) {
        set_error("forest is NULL");
        return CAPT_EINVAL;
    }
    const int32_t nc = (int32_t)f->clouds.size();
    capt_status st = check_offsets(qoff, nc, "query_off");
    if (st) return st;
    if (group < 1 || group > MAX_GROUP) {
        set_error("group = %d outside 1 .. 2^20", group);
        return CAPT_EINVAL;
    }
    for (int32_t c = 0; c < nc; ++c)
        if ((qoff[c + 1] - qoff[c]) % group) {
            set_error("query range of cloud %d (%lld spheres) is not a multiple of group %d", c,
                      (long long)(qoff[c + 1] - qoff[c]), group);
            return CAPT_EINVAL;
        }
    if (qoff[nc] > 0 && !spheres) {
        set_error("spheres is NULL");
        return CAPT_EINVAL;
    }
    if (qoff[nc] >= ((int64_t)1 << 40)) {
        set_error("too many spheres");
        return CAPT_EUNSUPPORTED;
    }
    return CAPT_OK;
}

void destroy_forest(capt_forest_s *f) {
    if (!f) return;
    (void)hipDeviceSynchronize();
    free_plan(f->plan);
    for (auto &c : f->clouds) free_cloud(c, nullptr);
    if (f->d_clouds) dev_free(f->d_clouds, nullptr);
    delete f;
}

// Stream-ordered release: the memory returns to the allocator behind the
// work already queued on s, so the host does not wait.
void destroy_forest_async(capt_forest_s *f, hipStream_t s) {
    if (!f) return;
    if (f->plan) {
        destroy_forest(f);
        return;
    }
    for (auto &c : f->clouds) free_cloud(c, s);
    if (f->d_clouds) dev_free(f->d_clouds, s);
    delete f;
}

// ---- blob layout --------------------------------------------------------
constexpr uint32_t BLOB_MAGIC = 0x54504143u;   // "CAPT"
constexpr uint32_t BLOB_VERSION = 2;

struct BlobHeader {
    uint32_t magic;
    uint32_t version;
    int64_t n;
    int64_t N;
    int32_t D;
    uint32_t flags;
    float r_min;
    float r_max;
    int64_t set_total;
};
static_assert(sizeof(BlobHeader) == 48, "blob header is 48 bytes");

inline size_t a8(size_t x) { return (x + 7) & ~(size_t)7; }

// Version 2 (a forest with a non-cyclic split axis per depth) carries the
// 8-byte axis code right after the header.
struct BlobLayout {
    size_t pts, T, rep, aabb, pruned, off, idx, total;
    BlobLayout(int64_t n, int64_t N, int64_t S, uint32_t version) {
        size_t o = a8(sizeof(BlobHeader) + (version >= 2 ? sizeof(uint64_t) : 0));
        pts = o;    o = a8(o + sizeof(float) * 3 * (size_t)n);
        T = o;      o = a8(o + sizeof(float) * (size_t)(N - 1));
        rep = o;    o = a8(o + sizeof(int32_t) * (size_t)N);
        aabb = o;   o = a8(o + sizeof(float) * 6 * (size_t)N);
        pruned = o; o = a8(o + (size_t)N);
        off = o;    o = a8(o + sizeof(int64_t) * (size_t)(N + 1));
        idx = o;    o = a8(o + sizeof(int32_t) * (size_t)S);
        total = o;
    }
};

}  // namespace

extern "C" {

const char *capt_last_error(void) { return g_err; }

capt_status capt_set_allocator(void *(*alloc)(size_t, void *, void *), void (*release)(void *, void *, void *),
                               void *ctx) {
    ApiGuard g;
    if ((alloc == nullptr) != (release == nullptr)) {
        set_error("alloc and release must both be set or both be NULL");
        return CAPT_EINVAL;
    }
    g_alloc.alloc = alloc;
    g_alloc.release = release;
    g_alloc.ctx = ctx;
    return CAPT_OK;
}

capt_status capt_set_tuning(const capt_tuning *t) {
    ApiGuard g;
    if (!t) {
        set_error("tuning is NULL");
        return CAPT_EINVAL;
    }
    if (t->waves_per_group < 0 || t->waves_per_group > 16 || t->groups_per_cu < 0 || t->groups_per_cu > 16 ||
        t->tile_cfgs < 0 || t->tile_cfgs > 4096 || t->lds_levels < 0 || t->lds_levels > 15 ||
        !(t->scan_unroll == 0 || t->scan_unroll == 1 || t->scan_unroll == 2 || t->scan_unroll == 4)) {
        set_error("tuning value out of range");
        return CAPT_EINVAL;
    }
    capt_tuning &cur = tuning();
    if (t->waves_per_group) cur.waves_per_group = t->waves_per_group;
    if (t->groups_per_cu) cur.groups_per_cu = t->groups_per_cu;
    if (t->tile_cfgs) cur.tile_cfgs = t->tile_cfgs;
    if (t->lds_levels) cur.lds_levels = t->lds_levels;
    if (t->scan_unroll) cur.scan_unroll = t->scan_unroll;
    return CAPT_OK;
}

capt_status capt_get_tuning(capt_tuning *t) {
    ApiGuard g;
    if (!t) {
        set_error("tuning is NULL");
        return CAPT_EINVAL;
    }
    *t = tuning();
    return CAPT_OK;
}

capt_status capt_filter(const float *xyz, int64_t n, float r_filter, float *out_xyz, int32_t *out_index,
                        int64_t *n_out, void *stream) {
    ApiGuard g;
    if (!n_out) {
        set_error("n_out is NULL");
        return CAPT_EINVAL;
    }
    if (n < 0 || (n > 0 && (!xyz || !out_xyz))) {
        set_error("bad cloud arguments (n = %lld)", (long long)n);
        return CAPT_EINVAL;
    }
    if (!finite_f(r_filter) || !(r_filter >= 0.0f)) {
        set_error("r_filter = %g must be finite and >= 0", (double)r_filter);
        return CAPT_EINVAL;
    }
    if (n >= ((int64_t)1 << 30)) {
        set_error("cloud of %lld points reaches 2^30", (long long)n);
        return CAPT_EUNSUPPORTED;
    }
    return filter(xyz, n, r_filter, nullptr, out_xyz, out_index, n_out, (hipStream_t)stream);
}

namespace {
capt_status check_crop(const float *crop) {
    if (!crop) {
        set_error("crop is NULL");
        return CAPT_EINVAL;
    }
    if (!finite_f(crop[0]) || !finite_f(crop[1]) || !finite_f(crop[2]) || std::isnan(crop[3]) || !(crop[3] >= 0.0f)) {
        set_error("crop base (%g, %g, %g) must be finite and reach %g >= 0", (double)crop[0], (double)crop[1],
                  (double)crop[2], (double)crop[3]);
        return CAPT_EINVAL;
    }
    return CAPT_OK;
}
}  // namespace

capt_status capt_filter_crop(const float *xyz, int64_t n, float r_filter, const float *crop, float *out_xyz,
                             int32_t *out_index, int64_t *n_out, void *stream) {
    ApiGuard g;
    if (!n_out) {
        set_error("n_out is NULL");
        return CAPT_EINVAL;
    }
    if (n < 0 || (n > 0 && (!xyz || !out_xyz))) {
        set_error("bad cloud arguments (n = %lld)", (long long)n);
        return CAPT_EINVAL;
    }
    if (!finite_f(r_filter) || !(r_filter >= 0.0f)) {
        set_error("r_filter = %g must be finite and >= 0", (double)r_filter);
        return CAPT_EINVAL;
    }
    capt_status st = check_crop(crop);
    if (st) return st;
    if (n >= ((int64_t)1 << 30)) {
        set_error("cropped filter of %lld points exceeds 2^30", (long long)n);
        return CAPT_EUNSUPPORTED;
    }
    return filter(xyz, n, r_filter, crop, out_xyz, out_index, n_out, (hipStream_t)stream);
}

namespace {
capt_status build_entry(const float *xyz, const int64_t *cloud_off, int32_t ncloud, float r_min, float r_max,
                        uint32_t flags, const uint8_t *axes, int shard_bits, int shard, void *stream,
                        capt_forest *out);
}  // namespace

capt_status capt_build(const float *xyz, const int64_t *cloud_off, int32_t ncloud, float r_min, float r_max,
                       uint32_t flags, void *stream, capt_forest *out) {
    ApiGuard g;
    return build_entry(xyz, cloud_off, ncloud, r_min, r_max, flags, nullptr, 0, 0, stream, out);
}

capt_status capt_build_axes(const float *xyz, const int64_t *cloud_off, int32_t ncloud, float r_min, float r_max,
                            uint32_t flags, const uint8_t *axes, void *stream, capt_forest *out) {
    ApiGuard g;
    if (!axes) {
        set_error("axes is NULL");
        return CAPT_EINVAL;
    }
    for (int d = 0; d < 30; ++d)
        if (axes[d] > 2) {
            set_error("axes[%d] = %u is not an axis (0, 1, 2)", d, (unsigned)axes[d]);
            return CAPT_EINVAL;
        }
    return build_entry(xyz, cloud_off, ncloud, r_min, r_max, flags, axes, 0, 0, stream, out);
}

capt_status capt_build_shard(const float *xyz, const int64_t *cloud_off, int32_t ncloud, float r_min, float r_max,
                             uint32_t flags, int32_t shard_bits, int32_t shard, void *stream, capt_forest *out) {
    ApiGuard g;
    if (out) *out = nullptr;
    if (shard_bits < 0 || shard_bits > CAPT_MAX_SHARD_BITS) {
        set_error("shard_bits = %d must lie in [0, %d]", shard_bits, CAPT_MAX_SHARD_BITS);
        return CAPT_EINVAL;
    }
    if (shard < 0 || shard >= (1 << shard_bits)) {
        set_error("shard = %d must lie in [0, 2^%d)", shard, shard_bits);
        return CAPT_EINVAL;
    }
    return build_entry(xyz, cloud_off, ncloud, r_min, r_max, flags, nullptr, shard_bits, shard, stream, out);
}

namespace {
capt_status build_entry(const float *xyz, const int64_t *cloud_off, int32_t ncloud, float r_min, float r_max,
                        uint32_t flags, const uint8_t *axes, int shard_bits, int shard, void *stream,
                        capt_forest *out) {
    if (!out) {
        set_error("out is NULL");
        return CAPT_EINVAL;
    }
    *out = nullptr;
    if (ncloud < 1) {
        set_error("ncloud = %d must be >= 1", ncloud);
        return CAPT_EINVAL;
    }
    capt_status st = check_offsets(cloud_off, ncloud, "cloud_off");
    if (st) return st;
    if (cloud_off[ncloud] > 0 && !xyz) {
        set_error("xyz is NULL");
        return CAPT_EINVAL;
    }
    if (!finite_f(r_min) || !finite_f(r_max) || !(r_min >= 0.0f) || !(r_max > 0.0f) || r_min > r_max) {
        set_error("radii r_min = %g, r_max = %g must satisfy 0 <= r_min <= r_max, r_max > 0", (double)r_min,
                  (double)r_max);
        return CAPT_EINVAL;
    }
    if (flags & ~(CAPT_NO_PRUNE | CAPT_INDEXED_SETS)) {
        set_error("unknown build flags 0x%x", flags);
        return CAPT_EINVAL;
    }
    capt_forest_s *f = new (std::nothrow) capt_forest_s();
    if (!f) {
        set_error("host allocation failed");
        return CAPT_ENOMEM;
    }
    st = build_forest(xyz, cloud_off, ncloud, r_min, r_max, flags, axes, shard_bits, shard, (hipStream_t)stream, f);
    if (st) {
        destroy_forest(f);
        return st;
    }
    *out = f;
    return CAPT_OK;
}
}  // namespace

capt_status capt_build_filtered(const float *xyz, int64_t n, float r_filter, const float *crop, float r_min,
                                float r_max, uint32_t flags, int32_t *kept_index, int64_t *n_kept, void *stream,
                                capt_forest *out) {
    ApiGuard g;
    if (!out) {
        set_error("out is NULL");
        return CAPT_EINVAL;
    }
    *out = nullptr;
    if (n < 0 || (n > 0 && !xyz)) {
        set_error("bad cloud arguments (n = %lld)", (long long)n);
        return CAPT_EINVAL;
    }
    if (!finite_f(r_filter) || !(r_filter >= 0.0f)) {
        set_error("r_filter = %g must be finite and >= 0", (double)r_filter);
        return CAPT_EINVAL;
    }
    if (crop) {
        capt_status cs = check_crop(crop);
        if (cs) return cs;
    }
    if (n >= ((int64_t)1 << 30)) {
        set_error("cloud of %lld points exceeds the filter's limit", (long long)n);
        return CAPT_EUNSUPPORTED;
    }
    if (!finite_f(r_min) || !finite_f(r_max) || !(r_min >= 0.0f) || !(r_max > 0.0f) || r_min > r_max) {
        set_error("radii r_min = %g, r_max = %g must satisfy 0 <= r_min <= r_max, r_max > 0", (double)r_min,
                  (double)r_max);
        return CAPT_EINVAL;
    }
    if (flags & ~(CAPT_NO_PRUNE | CAPT_INDEXED_SETS)) {
        set_error("unknown build flags 0x%x", flags);
        return CAPT_EINVAL;
    }
    const hipStream_t s = (hipStream_t)stream;
    // the kept points live in stream-ordered scratch: the build copies them
    Scratch kept;
    if (!kept.alloc(sizeof(float) * 3 * (size_t)std::max<int64_t>(n, 1), s)) {
        set_error("device allocation of the kept points failed");
        return CAPT_ENOMEM;
    }
    int64_t m = 0;
    capt_status st = filter(xyz, n, r_filter, crop, kept.as<float>(), kept_index, &m, s);
    if (st) return st;
    if (n_kept) *n_kept = m;
    capt_forest_s *f = new (std::nothrow) capt_forest_s();
    if (!f) {
        set_error("host allocation failed");
        return CAPT_ENOMEM;
    }
    const int64_t off[2] = {0, m};
    st = build_forest(kept.as<float>(), off, 1, r_min, r_max, flags, nullptr, 0, 0, s, f);
    if (st) {
        destroy_forest(f);
        return st;
    }
    *out = f;
    return CAPT_OK;
}

capt_status capt_collides(capt_forest f, const float *spheres, const int64_t *query_off, int32_t group,
                          uint8_t *out, uint32_t flags, void *stream) {
    ApiGuard g;
    capt_status st = check_queries(f, spheres, query_off, group);
    if (st) return st;
    if (flags & ~(CAPT_CHECK_RADII | CAPT_PER_CLOUD | CAPT_NO_GRAPH)) {
        set_error("unknown query flags 0x%x", flags);
        return CAPT_EINVAL;
    }
    const int64_t M = query_off[f->clouds.size()];
    if (M > 0 && !out) {
        set_error("out is NULL");
        return CAPT_EINVAL;
    }
    if (M == 0) return CAPT_OK;
    return collides(f, spheres, query_off, group, out, flags, (hipStream_t)stream);
}

capt_status capt_collides_noalloc(capt_forest f, const float *spheres, const int64_t *query_off, int32_t group,
                                  uint8_t *out, uint32_t flags, void *stream) {
    ApiGuard g;
    capt_status st = check_queries(f, spheres, query_off, group);
    if (st) return st;
    if (flags != 0) {
        set_error("capt_collides_noalloc takes flags 0 (got 0x%x)", flags);
        return CAPT_EINVAL;
    }
    const int64_t M = query_off[f->clouds.size()];
    if (M > 0 && !out) {
        set_error("out is NULL");
        return CAPT_EINVAL;
    }
    if (M == 0) return CAPT_OK;
    return collides_noalloc(f, spheres, query_off, group, out, (hipStream_t)stream);
}

capt_status capt_collides_visits(capt_forest f, const float *spheres, const int64_t *query_off, int32_t group,
                                 uint8_t *out, int32_t *visits, void *stream) {
    ApiGuard g;
    capt_status st = check_queries(f, spheres, query_off, group);
    if (st) return st;
    const int64_t M = query_off[f->clouds.size()];
    if (M > 0 && (!out || !visits)) {
        set_error("out or visits is NULL");
        return CAPT_EINVAL;
    }
    if (M == 0) return CAPT_OK;
    return collides_visits(f, spheres, query_off, group, out, visits, (hipStream_t)stream);
}

capt_status capt_collides_padded(capt_forest f, const float *spheres, const int64_t *query_off, int32_t group,
                                 float pad, uint8_t *out, uint32_t flags, void *stream) {
    ApiGuard g;
    capt_status st = check_queries(f, spheres, query_off, group);
    if (st) return st;
    if (flags & ~CAPT_CHECK_RADII) {
        set_error("unknown padded query flags 0x%x", flags);
        return CAPT_EINVAL;
    }
    if (!finite_f(pad) || !(pad >= 0.0f)) {
        set_error("pad = %g must be finite and >= 0", (double)pad);
        return CAPT_EINVAL;
    }
    const int64_t M = query_off[f->clouds.size()];
    if (M > 0 && !out) {
        set_error("out is NULL");
        return CAPT_EINVAL;
    }
    if (M == 0) return CAPT_OK;
    return collides_padded(f, spheres, query_off, group, pad, out, flags, (hipStream_t)stream);
}

capt_status capt_collides_posed(capt_forest f, const float *tmpl, int32_t g, const float *poses,
                                const int64_t *pose_off, int32_t edge, uint8_t *out, uint32_t flags, void *stream) {
    ApiGuard guard;
    if (g < 1 || g > 1024) {
        set_error("template size g = %d outside 1 .. 1024", g);
        return CAPT_EINVAL;
    }
    if (!tmpl) {
        set_error("template is NULL");
        return CAPT_EINVAL;
    }
    if (edge < 1 || (int64_t)edge * g > MAX_GROUP) {
        set_error("edge = %d outside 1 .. 2^20 / g", edge);
        return CAPT_EINVAL;
    }
    capt_status st = check_queries(f, poses, pose_off, edge);   // pose ranges in whole edges
    if (st) return st;
    if (flags & ~CAPT_CHECK_RADII) {
        set_error("unknown posed query flags 0x%x", flags);
        return CAPT_EINVAL;
    }
    const int64_t P = pose_off[f->clouds.size()];
    if (P > 0 && !out) {
        set_error("out is NULL");
        return CAPT_EINVAL;
    }
    if (P == 0) return CAPT_OK;
    return collides_posed(f, tmpl, g, poses, pose_off, edge, out, flags, (hipStream_t)stream);
}

capt_status capt_clearance(capt_forest f, const float *spheres, const int64_t *query_off, float *clearance,
                           int32_t *witness, void *stream) {
    ApiGuard g;
    capt_status st = check_queries(f, spheres, query_off, 1);
    if (st) return st;
    const int64_t M = query_off[f->clouds.size()];
    if (M > 0 && (!clearance || !witness)) {
        set_error("clearance or witness is NULL");
        return CAPT_EINVAL;
    }
    if (f->pruned_total > 0) {
        set_error("forest has %lld pruned leaves; build with CAPT_NO_PRUNE or r_min = 0 for clearance",
                  (long long)f->pruned_total);
        return CAPT_EPRUNED;
    }
    if (M == 0) return CAPT_OK;
    return clearance_fwd(f, spheres, query_off, clearance, witness, (hipStream_t)stream);
}

capt_status capt_clearance_backward(capt_forest f, const float *spheres, const int64_t *query_off,
                                    const int32_t *witness, const float *grad_clearance, float *grad_center,
                                    float *grad_radius, void *stream) {
    ApiGuard g;
    capt_status st = check_queries(f, spheres, query_off, 1);
    if (st) return st;
    const int64_t M = query_off[f->clouds.size()];
    if (M > 0 && (!witness || !grad_clearance || !grad_center)) {
        set_error("witness, grad_clearance or grad_center is NULL");
        return CAPT_EINVAL;
    }
    if (f->pruned_total > 0) {
        set_error("forest has pruned leaves");
        return CAPT_EPRUNED;
    }
    if (M == 0) return CAPT_OK;
    return clearance_bwd(f, spheres, query_off, witness, grad_clearance, grad_center, grad_radius,
                         (hipStream_t)stream);
}

void capt_destroy(capt_forest f) { destroy_forest(f); }

void capt_destroy_async(capt_forest f, void *stream) { destroy_forest_async(f, static_cast<hipStream_t>(stream)); }

capt_status capt_forest_info(capt_forest f, int32_t cloud, int64_t *n, int32_t *D, int64_t *set_total,
                             int64_t *pruned, int64_t *bytes) {
    ApiGuard g;
    if (!f || cloud < 0 || cloud >= (int32_t)f->clouds.size()) {
        set_error("bad forest or cloud index");
        return CAPT_EINVAL;
    }
    const CloudHost &c = f->clouds[cloud];
    if (n) *n = c.n;
    if (D) *D = c.D;
    if (set_total) *set_total = c.set_total;
    if (pruned) *pruned = c.pruned;
    if (bytes) *bytes = (int64_t)(c.fixed_bytes + c.sets_bytes);
    return CAPT_OK;
}

capt_status capt_export(capt_forest f, int32_t cloud, void *host_blob, size_t *bytes) {
    ApiGuard g;
    if (!f || !bytes || cloud < 0 || cloud >= (int32_t)f->clouds.size()) {
        set_error("bad forest, cloud index or bytes pointer");
        return CAPT_EINVAL;
    }
    const CloudHost &c = f->clouds[cloud];
    const uint32_t version = c.dev.cyclic ? 1u : 2u;
    const BlobLayout L(c.n, c.N, c.set_total, version);
    if (!host_blob) {
        *bytes = L.total;
        return CAPT_OK;
    }
    if (*bytes < L.total) {
        set_error("blob buffer of %zu bytes is smaller than %zu", *bytes, L.total);
        return CAPT_EINVAL;
    }
    char *B = static_cast<char *>(host_blob);
    memset(B, 0, L.total);
    BlobHeader h{BLOB_MAGIC, version, c.n, c.N, c.D, c.dev.flags, f->r_min, f->r_max, c.set_total};
    memcpy(B, &h, sizeof h);
    if (version >= 2) memcpy(B + sizeof h, &c.dev.axes, sizeof(uint64_t));
    std::vector<Leaf> leaves((size_t)c.N);
    std::vector<float> px((size_t)std::max<int64_t>(c.set_padded, 1)), py(px.size()), pz(px.size());
    std::vector<int32_t> pidx(px.size());
    if (c.n > 0) CAPT_HIP(hipMemcpy(B + L.pts, c.dev.pts, sizeof(float) * 3 * (size_t)c.n, hipMemcpyDeviceToHost));
    if (c.N > 1) CAPT_HIP(hipMemcpy(B + L.T, c.dev.T, sizeof(float) * (size_t)(c.N - 1), hipMemcpyDeviceToHost));
    CAPT_HIP(hipMemcpy(B + L.rep, c.rep, sizeof(int32_t) * (size_t)c.N, hipMemcpyDeviceToHost));
    CAPT_HIP(hipMemcpy(B + L.pruned, c.pruned_flag, (size_t)c.N, hipMemcpyDeviceToHost));
    CAPT_HIP(hipMemcpy(leaves.data(), c.dev.leaf, sizeof(Leaf) * (size_t)c.N, hipMemcpyDeviceToHost));
    if (c.set_padded > 0)
        CAPT_HIP(hipMemcpy(pidx.data(), c.dev.pidx, sizeof(int32_t) * (size_t)c.set_padded, hipMemcpyDeviceToHost));
    float *aabb = reinterpret_cast<float *>(B + L.aabb);
    int64_t *off = reinterpret_cast<int64_t *>(B + L.off);
    int32_t *idx = reinterpret_cast<int32_t *>(B + L.idx);
    int64_t o = 0;
    for (int64_t l = 0; l < c.N; ++l) {
        const Leaf &lf = leaves[(size_t)l];
        for (int a = 0; a < 3; ++a) {
            aabb[6 * l + a] = lf.lo[a];
            aabb[6 * l + 3 + a] = lf.hi[a];
        }
        off[l] = o;
        for (uint32_t k = 0; k < lf.count; ++k) idx[o++] = pidx[lf.start + k];
    }
    off[c.N] = o;
    return CAPT_OK;
}

capt_status capt_import(const void *host_blob, size_t bytes, void *stream, capt_forest *out) {
    ApiGuard g;
    if (!host_blob || !out || bytes < sizeof(BlobHeader)) {
        set_error("bad blob arguments");
        return CAPT_EINVAL;
    }
    *out = nullptr;
    const char *B = static_cast<const char *>(host_blob);
    BlobHeader h;
    memcpy(&h, B, sizeof h);
    // every size is bounded here, before the layout is computed from them, so
    // the section offsets below cannot wrap
    if (h.magic != BLOB_MAGIC || h.version < 1 || h.version > BLOB_VERSION || h.n < 0 || h.D < 0 || h.D > 30 ||
        h.N != ((int64_t)1 << h.D) || h.n > h.N || (h.n > 0 && h.N >= 2 * h.n) || h.set_total < 0 ||
        h.set_total >= (int64_t)MAX_SET_ENTRIES || !(h.r_max > 0.0f) || !(h.r_min >= 0.0f) || h.r_min > h.r_max ||
        !std::isfinite(h.r_max) || (h.flags & ~(CAPT_NO_PRUNE | CAPT_INDEXED_SETS))) {
        set_error("blob header is invalid");
        return CAPT_EINVAL;
    }
    uint64_t axes = axes_code(nullptr, h.D);
    if (h.version >= 2) {
        if (bytes < sizeof h + sizeof axes) {
            set_error("blob too short");
            return CAPT_EINVAL;
        }
        memcpy(&axes, B + sizeof h, sizeof axes);
        for (int d = 0; d < 32; ++d)
            if (d < h.D ? axis_at(axes, d) > 2 : axis_at(axes, d) != 0) {
                set_error("blob axis code is invalid");
                return CAPT_EINVAL;
            }
    }
    const BlobLayout L(h.n, h.N, h.set_total, h.version);
    if (bytes < L.total) {
        set_error("blob holds %zu bytes, layout needs %zu", bytes, L.total);
        return CAPT_EINVAL;
    }
    const float *pts = reinterpret_cast<const float *>(B + L.pts);
    const float *aabb = reinterpret_cast<const float *>(B + L.aabb);
    const int64_t *off = reinterpret_cast<const int64_t *>(B + L.off);
    const int32_t *idx = reinterpret_cast<const int32_t *>(B + L.idx);
    const uint8_t *pr = reinterpret_cast<const uint8_t *>(B + L.pruned);
    // all N + 1 offsets before any set is read: start at 0, never decrease,
    // end at S (so every set lies inside the idx section)
    if (off[0] != 0 || off[h.N] != h.set_total) {
        set_error("blob set offsets are invalid");
        return CAPT_EINVAL;
    }
    for (int64_t l = 0; l < h.N; ++l)
        if (off[l + 1] < off[l] || off[l + 1] > h.set_total) {
            set_error("blob set offsets of leaf %lld are invalid", (long long)l);
            return CAPT_EINVAL;
        }
    for (int64_t j = 0; j < 3 * h.n; ++j)
        if (!std::isfinite(pts[j])) {
            set_error("blob point %lld is not finite", (long long)(j / 3));
            return CAPT_EINVAL;
        }
    // place the sets (aligned as the builder does) and check every AABB
    const int32_t *rep = reinterpret_cast<const int32_t *>(B + L.rep);
    std::vector<Leaf> leaves((size_t)h.N);
    int64_t padded = 0, pruned = 0;
    for (int64_t l = 0; l < h.N; ++l) {
        if (off[l + 1] < off[l] || rep[l] < 0 || rep[l] >= h.N) {
            set_error("blob leaf %lld is invalid", (long long)l);
            return CAPT_EINVAL;
        }
        const int64_t cnt = off[l + 1] - off[l];
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t k = off[l]; k < off[l + 1]; ++k) {
            if (idx[k] < 0 || idx[k] >= h.n) {
                set_error("blob set entry %lld is out of range", (long long)k);
                return CAPT_EINVAL;
            }
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], pts[3 * (int64_t)idx[k] + a]);
                hi[a] = std::max(hi[a], pts[3 * (int64_t)idx[k] + a]);
            }
        }
        for (int a = 0; a < 3; ++a)
            if (!(lo[a] == aabb[6 * l + a]) || !(hi[a] == aabb[6 * l + 3 + a])) {
                set_error("blob AABB of leaf %lld is not the bounding box of its set", (long long)l);
                return CAPT_EINVAL;
            }
        Leaf &lf = leaves[(size_t)l];
        for (int a = 0; a < 3; ++a) {
            lf.lo[a] = lo[a];
            lf.hi[a] = hi[a];
        }
        lf.start = (uint32_t)padded;
        lf.count = (uint32_t)cnt;
        padded += cnt ? ((cnt + SET_ALIGN - 1) / SET_ALIGN) * SET_ALIGN : 0;
        pruned += pr[l] ? 1 : 0;
        if (padded >= (int64_t)MAX_SET_ENTRIES) {
            set_error("blob sets too large");
            return CAPT_EUNSUPPORTED;
        }
    }
    const size_t E = (size_t)std::max<int64_t>(padded, (int64_t)CHUNK);
    std::vector<float> pe(3 * E, INFINITY);   // per chunk: 16 x, 16 y, 16 z (set_off)
    std::vector<int32_t> pidx(E, -1);
    for (int64_t l = 0; l < h.N; ++l)
        for (int64_t k = off[l]; k < off[l + 1]; ++k) {
            const size_t e = leaves[(size_t)l].start + (size_t)(k - off[l]);
            const int64_t id = idx[k];
            const int64_t o = set_off((int64_t)e);
            pe[o] = pts[3 * id];
            pe[o + CHUNK] = pts[3 * id + 1];
            pe[o + 2 * CHUNK] = pts[3 * id + 2];
            pidx[e] = (int32_t)id;
        }
    // the box of every 16-entry chunk, relative to its set's box (hbox_encode)
    std::vector<uint4> cbox(E / CHUNK, make_uint4(0u, 0u, 0u, 0u));
    for (int64_t l = 0; l < h.N; ++l) {
        const Leaf &lf = leaves[(size_t)l];
        for (uint32_t c0 = 0; c0 < lf.count; c0 += CHUNK) {
            float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (uint32_t k = c0; k < std::min(lf.count, c0 + CHUNK); ++k) {
                const int64_t id = idx[off[l] + k];
                for (int a = 0; a < 3; ++a) {
                    lo[a] = std::min(lo[a], pts[3 * id + a]);
                    hi[a] = std::max(hi[a], pts[3 * id + a]);
                }
            }
            cbox[(lf.start + c0) / CHUNK] = hbox_encode(lf.lo, lo, hi);
        }
    }

    capt_forest_s *f = new (std::nothrow) capt_forest_s();
    if (!f) {
        set_error("host allocation failed");
        return CAPT_ENOMEM;
    }
    f->clouds.resize(1);
    f->r_min = h.r_min;
    f->r_max = h.r_max;
    f->flags = h.flags;
    f->pruned_total = pruned;
    CloudHost &c = f->clouds[0];
    c.n = h.n;
    c.N = h.N;
    c.D = h.D;
    c.set_total = h.set_total;
    c.set_padded = padded;
    c.pruned = pruned;
    hipStream_t s = (hipStream_t)stream;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t oT = 0;
    const size_t oLeaf = al(sizeof(float) * (size_t)std::max<int64_t>(h.N - 1, 1));
    const size_t oPts = al(oLeaf + sizeof(Leaf) * (size_t)h.N);
    const size_t oRep = al(oPts + sizeof(float) * 3 * (size_t)std::max<int64_t>(h.n, 1));
    const size_t oPr = al(oRep + sizeof(int32_t) * (size_t)h.N);
    const size_t oTb = al(oPr + (size_t)h.N);
    c.fixed_bytes = al(oTb + sizeof(float4) * 4 * (size_t)tree_blocks_count(h.D));
    c.fixed = dev_alloc(c.fixed_bytes, s);
    const bool indexed = (h.flags & CAPT_INDEXED_SETS) != 0;
    c.sets_bytes = sets_bytes(E, indexed);
    c.sets = dev_alloc(c.sets_bytes, s);
    if (!c.fixed || !c.sets) {
        destroy_forest(f);
        set_error("device allocation failed");
        return CAPT_ENOMEM;
    }
    char *F = static_cast<char *>(c.fixed);
    c.dev.T = reinterpret_cast<float *>(F + oT);
    c.dev.leaf = reinterpret_cast<Leaf *>(F + oLeaf);
    c.dev.pts = reinterpret_cast<float *>(F + oPts);
    c.rep = reinterpret_cast<int32_t *>(F + oRep);
    c.pruned_flag = reinterpret_cast<uint8_t *>(F + oPr);
    c.dev.tb = tree_blocks_count(h.D) > 0 ? reinterpret_cast<float4 *>(F + oTb) : nullptr;
    {
        float *qx, *qy, *qz;
        int32_t *qi;
        uint4 *qb;
        sets_layout(c.sets, E, indexed, &qx, &qy, &qz, &qi, &qb);
        c.dev.px = qx;
        c.dev.py = qy;
        c.dev.pz = qz;
        c.dev.pidx = qi;
        c.dev.cbox = qb;
    }
    c.dev.n = h.n;
    c.dev.D = h.D;
    c.dev.flags = h.flags;
    c.dev.axes = axes;
    c.dev.cyclic = axes == axes_code(nullptr, h.D) ? 1 : 0;
    auto cp = [&](void *dst, const void *src, size_t nb) -> capt_status {
        if (nb) CAPT_HIP(hipMemcpy(dst, src, nb, hipMemcpyHostToDevice));
        return CAPT_OK;
    };
    capt_status st = CAPT_OK;
    if (!st) st = cp(const_cast<float *>(c.dev.T), B + L.T, sizeof(float) * (size_t)(h.N - 1));
    if (!st) st = cp(const_cast<Leaf *>(c.dev.leaf), leaves.data(), sizeof(Leaf) * (size_t)h.N);
    if (!st) st = cp(const_cast<float *>(c.dev.pts), pts, sizeof(float) * 3 * (size_t)h.n);
    if (!st) st = cp(c.rep, rep, sizeof(int32_t) * (size_t)h.N);
    if (!st) st = cp(c.pruned_flag, pr, (size_t)h.N);
    if (!st) st = tree_blocks(c.dev.T, (int)h.D, const_cast<float4 *>(c.dev.tb), s);
    if (!indexed && !st) st = cp(const_cast<float *>(c.dev.px), pe.data(), sizeof(float) * 3 * E);
    if (!st) st = cp(const_cast<int32_t *>(c.dev.pidx), pidx.data(), sizeof(int32_t) * E);
    if (!st) st = cp(const_cast<uint4 *>(c.dev.cbox), cbox.data(), sizeof(uint4) * cbox.size());
    if (!st) st = upload_views(f, s);
    if (st) {
        destroy_forest(f);
        return st;
    }
    *out = f;
    return CAPT_OK;
}

capt_status capt_bruteforce_collides(const float *xyz, const int64_t *cloud_off, int32_t ncloud,
                                     const float *spheres, const int64_t *query_off, int32_t group, uint8_t *out,
                                     void *stream) {
    ApiGuard g;
    if (ncloud < 1) {
        set_error("ncloud = %d must be >= 1", ncloud);
        return CAPT_EINVAL;
    }
    capt_status st = check_offsets(cloud_off, ncloud, "cloud_off");
    if (!st) st = check_offsets(query_off, ncloud, "query_off");
    if (st) return st;
    if (group < 1 || group > MAX_GROUP) {
        set_error("group = %d outside 1 .. 2^20", group);
        return CAPT_EINVAL;
    }
    for (int32_t c = 0; c < ncloud; ++c)
        if ((query_off[c + 1] - query_off[c]) % group) {
            set_error("query range of cloud %d is not a multiple of group", c);
            return CAPT_EINVAL;
        }
    if ((cloud_off[ncloud] > 0 && !xyz) || (query_off[ncloud] > 0 && (!spheres || !out))) {
        set_error("NULL buffer");
        return CAPT_EINVAL;
    }
    return bruteforce(xyz, cloud_off, ncloud, spheres, query_off, group, out, (hipStream_t)stream);
}

capt_status capt_query_stats(capt_forest f, const float *spheres, const int64_t *query_off, int32_t *leaf,
                             uint8_t *rejected, int32_t *scanned, uint8_t *hit, void *stream) {
    ApiGuard g;
    capt_status st = check_queries(f, spheres, query_off, 1);
    if (st) return st;
    return query_stats(f, spheres, query_off, leaf, rejected, scanned, hit, (hipStream_t)stream);
}

capt_status capt_query_chunk_stats(capt_forest f, const float *spheres, const int64_t *query_off, int32_t *boxes,
                                   int32_t *chunks, void *stream) {
    ApiGuard g;
    capt_status st = check_queries(f, spheres, query_off, 1);
    if (st) return st;
    return chunk_stats(f, spheres, query_off, boxes, chunks, (hipStream_t)stream);
}


capt_status capt_probe_read(const void *buf, size_t bytes, int32_t passes, int32_t blocks_per_cu, float *sink,
                            void *stream) {
    ApiGuard g;
    if (blocks_per_cu < 1 || blocks_per_cu > 32) {
        set_error("blocks_per_cu = %d outside 1 .. 32", blocks_per_cu);
        return CAPT_EINVAL;
    }
    if (bytes >= 16 && (!buf || !sink)) {
        set_error("buf and sink must be set");
        return CAPT_EINVAL;
    }
    if (passes < 0) {
        set_error("passes = %d is negative", passes);
        return CAPT_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(buf) % 16) {
        set_error("buf is not 16-byte aligned");
        return CAPT_EINVAL;
    }
    return probe_read(buf, bytes, passes, blocks_per_cu, sink, (hipStream_t)stream);
}

capt_status capt_probe_gather(const int32_t *items, int64_t m, const void *leaves, int64_t nleaf, const float *x,
                              const float *y, const float *z, int64_t entries, int32_t lanes_per_item, uint8_t *out,
                              void *stream) {
    ApiGuard g;
    if (m < 0 || nleaf < 0 || entries < 0) {
        set_error("negative size");
        return CAPT_EINVAL;
    }
    if (lanes_per_item != 16 && lanes_per_item != 64) {
        set_error("lanes_per_item = %d, expected 16 or 64", lanes_per_item);
        return CAPT_EINVAL;
    }
    if (m > 0 && (!items || !out || (nleaf > 0 && !leaves) || (entries > 0 && (!x || !y || !z)))) {
        set_error("a buffer is NULL");
        return CAPT_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(items) % 16 || reinterpret_cast<uintptr_t>(leaves) % 16) {
        set_error("items and leaves must be 16-byte aligned");
        return CAPT_EINVAL;
    }
    if (m == 0) return CAPT_OK;
    return probe_gather(items, m, leaves, nleaf, x, y, z, entries, lanes_per_item, out, (hipStream_t)stream);
}

}  // extern "C"
