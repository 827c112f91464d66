/*
 * capt.h - C ABI of the MI355X collision-affording point tree (CAPT) library.
 *
 * A CAPT (Ramsey, Kingston, Thomason, Kavraki, "Collision-Affording Point
 * Trees", arXiv 2406.02807) answers "does a sphere of radius r in
 * [r_min, r_max] touch any point of a 3-D point cloud?" exactly, by descending
 * an implicit k-d tree to one leaf cell and scanning that leaf's affordance
 * set: every cloud point that a sphere of radius <= r_max centred anywhere in
 * the cell could touch (Sec. IV-A, Lemma 1).
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers (HIP global memory of the current device)
 *    unless the comment says "host".
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is ordered on it; entry points return without waiting for it
 *    unless the comment says "synchronises".
 *  - Points are float32 [n][3] (x, y, z) row-major.  Spheres are float32
 *    [m][4] (x, y, z, r) row-major.
 *  - The caller owns every input and output buffer.  A forest owns its own
 *    device memory until capt_destroy.
 *  - Nothing throws across the ABI.  On failure an entry point returns a
 *    non-zero capt_status, writes no output, and capt_last_error() describes
 *    the failure (thread-local).  Host-side argument checks run before any
 *    device work is queued.
 *  - The collision predicate is float32 and fixed: a sphere (x, r) touches p
 *    iff ((dx*dx + dy*dy) + dz*dz) <= r*r with dx = x_x - p_x etc., each
 *    operation rounded to nearest-even, no fused multiply-add.  Answers equal
 *    a brute-force evaluation of that predicate over the whole cloud bit for
 *    bit, for every radius in [r_min, r_max] (Lemma 1).
 */
#ifndef CAPT_H
#define CAPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct capt_forest_s *capt_forest;   /* immutable after build or import */
typedef int32_t capt_status;

#define CAPT_OK           0
#define CAPT_EINVAL       1   /* bad argument, non-finite cloud point, bad blob */
#define CAPT_ENOMEM       2   /* device or host allocation failed */
#define CAPT_EHIP         3   /* a HIP runtime call or kernel failed */
#define CAPT_ERADIUS      4   /* a query radius lies outside [r_min, r_max] (checked mode) */
#define CAPT_EPRUNED      5   /* clearance on a forest with r_min-pruned leaves */
#define CAPT_EUNSUPPORTED 6   /* size beyond the library's limits */

/* Build flags */
#define CAPT_NO_PRUNE     0x1u  /* never apply r_min pruning (Sec. IV-B) */
#define CAPT_INDEXED_SETS 0x10u /* sets hold point indices only; queries gather the
                                   coordinates from the forest's point table */
/* Query flags */
#define CAPT_CHECK_RADII  0x2u  /* validate radii first (one device-to-host sync) */
#define CAPT_PER_CLOUD    0x4u  /* forests: one launch per cloud, not one batched launch */
#define CAPT_NO_GRAPH     0x8u  /* forests: launch the batched kernel directly, no hipGraph */

/* Limits */
#define CAPT_MAX_SHARD_BITS 20  /* capt_build_shard: at most 2^20 shards */

/*
 * Filter (Alg. 2, Sec. IV-C).  For each of the six axis permutations, in the
 * order xyz, xzy, yxz, yzx, zxy, zyx: stable-sort the current points along the
 * Z-order (Morton) curve of that permutation, then keep a point iff its
 * float32 squared distance to the last kept point exceeds r_filter^2.  The
 * Morton grid is 2^21 cells per axis over the cubic bounding box of the input
 * (lower corner = float32 minimum, cell = largest extent / 2^21).  Key bit
 * 3b + (2 - j) holds bit b of the cell coordinate on the permutation's j-th
 * axis.
 *   xyz        [n][3] input points (finite)
 *   r_filter   >= 0, finite
 *   out_xyz    [n][3] capacity; receives the kept points, in final curve
 *              order, bitwise equal to the input coordinates
 *   out_index  [n] capacity or NULL; original index of each kept point
 *   n_out      host; number of kept points
 * n must be below 2^30 (CAPT_EUNSUPPORTED otherwise).  Synchronises on
 * `stream` once at the end to read n_out.  Scratch memory is taken from the
 * allocator (capt_set_allocator) and released before return.  A pass costs
 * time linear in n whatever runs of coincident points the cloud holds.
 */
capt_status capt_filter(const float *xyz, int64_t n, float r_filter,
                        float *out_xyz, int32_t *out_index, int64_t *n_out,
                        void *stream);

/*
 * Filter with a reach crop for a fixed-base arm (Sec. IV-C): a point can only
 * touch the robot if it lies within the arm's reach of its base, so points
 * farther away are removed first and capt_filter runs on the rest, in input
 * order (the Morton grid is over the cropped points).  A point stays iff it
 * is finite and ((dx*dx + dy*dy) + dz*dz) <= fl(reach * reach) in float32,
 * every operation rounded on its own, d = point - base.  The caller folds any
 * margin (link and sphere radii) into reach.
 *   crop       host [4]: base x, y, z (finite), reach (>= 0, may be +inf)
 *   others     as capt_filter; out_index holds input indices
 * n must be below 2^30.  Synchronises on `stream` twice.
 */
capt_status capt_filter_crop(const float *xyz, int64_t n, float r_filter,
                             const float *crop, float *out_xyz,
                             int32_t *out_index, int64_t *n_out, void *stream);

/*
 * Construct (Alg. 1, Sec. IV-A/B) for `ncloud` independent clouds.
 *   xyz        [sum n_c][3] points of all clouds back to back (finite)
 *   cloud_off  host [ncloud + 1]; cloud c is xyz[cloud_off[c] .. cloud_off[c+1])
 *              (non-decreasing, cloud_off[0] = 0; empty clouds allowed)
 *   r_min      0 <= r_min <= r_max, finite; r_min = 0 disables pruning
 *   r_max      > 0, finite
 *   flags      0, CAPT_NO_PRUNE, CAPT_INDEXED_SETS or both.  With
 *              CAPT_INDEXED_SETS the affordance sets store only the index of
 *              each member (4 bytes instead of 16 per entry; the memory of
 *              Sec. IV-B grows with the total set size) and every query reads a
 *              member's coordinates from the forest's copy of the cloud: the
 *              same answers, one more dependent load per scanned chunk.
 *   out        host; receives the forest
 * Each cloud of n points is padded with points at +inf to N = 2^D >= n
 * (Sec. IV-A).  Node i at depth d splits on axis d mod 3 at the coordinate of
 * the lower median under the order (coordinate, original index); points at or
 * below the value go left, children are 2i+1 and 2i+2 (Eytzinger order).  A
 * leaf's affordance set holds every real point whose float64 distance to the
 * leaf's closed cell is <= r_max (1 + 2^-20); when r_min > 0, the cell is
 * bounded and the float64 squared distance from the leaf's representative to
 * the cell's farthest corner is <= r_min^2 (1 - 2^-18), the set is just the
 * representative (Sec. IV-B).  Each leaf also stores the float32 bounding box of its set.
 * Synchronises on `stream` once (to size the affordance sets).  Non-finite
 * points give CAPT_EINVAL and no forest; a cloud of 2^30 points or more, or
 * whose sets (each padded to a multiple of 16 entries) reach 2^30 entries,
 * gives CAPT_EUNSUPPORTED.
 */
capt_status capt_build(const float *xyz, const int64_t *cloud_off, int32_t ncloud,
                       float r_min, float r_max, uint32_t flags, void *stream,
                       capt_forest *out);

/*
 * capt_build with the split axis of every depth given (Sec. IV-A names a
 * random choice of axis as an alternative to the cyclic rule): depth d
 * splits on axis axes[d] instead of d mod 3, the same axis across a depth,
 * so the tree stays implicit; the caller draws the axes (for example at
 * random).  Queries, clearance, counters and export follow the stored axes.
 *   axes       host [30]; values 0 (x), 1 (y), 2 (z); entries past the
 *              depth are ignored
 * A forest of several clouds with non-cyclic axes answers capt_collides with
 * one launch per cloud (the batched kernel takes cyclic forests only).
 */
capt_status capt_build_axes(const float *xyz, const int64_t *cloud_off, int32_t ncloud,
                            float r_min, float r_max, uint32_t flags, const uint8_t *axes,
                            void *stream, capt_forest *out);

/*
 * One shard of a forest too large to hold at once (Sec. VII: a set of CAPTs,
 * each responsible for one neighbourhood of a large cloud).  Shard s of
 * 2^shard_bits is capt_build's forest of the same cloud in which only the
 * leaves l with floor(l 2^shard_bits / N) = s keep their affordance sets;
 * for shard_bits <= D these are the leaves under depth-shard_bits node s,
 * the subtree of the cell that shard s answers for.  The splits, cells and
 * representatives are the whole cloud's; every other leaf holds no points,
 * no box and is never pruned, so a sphere that descends into another shard's
 * subtree is rejected on the leaf box.  Set memory is the shard's share.
 * Every query call takes a shard forest, and the answers combine exactly:
 *   capt_collides   the whole forest's answer = OR over the 2^shard_bits shards
 *   capt_clearance  the whole forest's clearance = min over the shards (a
 *                   sphere outside a shard gets r_max - r and witness -1)
 * Each cloud of a batch is sharded with the same (shard_bits, shard).
 *   shard_bits  0 .. CAPT_MAX_SHARD_BITS; 0 gives capt_build's forest
 *   shard       0 .. 2^shard_bits - 1
 * Other arguments, synchronisation and errors as capt_build; a shard_bits or
 * shard out of range gives CAPT_EINVAL.  A shard exports and imports as any
 * forest.
 */
capt_status capt_build_shard(const float *xyz, const int64_t *cloud_off, int32_t ncloud,
                             float r_min, float r_max, uint32_t flags, int32_t shard_bits,
                             int32_t shard, void *stream, capt_forest *out);

/*
 * Per-frame rebuild (Sec. IV-C followed by Sec. IV-A/B): capt_filter (or,
 * with crop, capt_filter_crop) of one cloud, then capt_build of the kept
 * points, in one call with no host work between the two.  The forest equals
 * capt_build's on the filter's output.
 *   xyz, n, r_filter   as capt_filter
 *   crop       host [4] as capt_filter_crop, or NULL for no crop
 *   r_min, r_max, flags as capt_build (one cloud)
 *   kept_index [n] capacity or NULL; original index of each kept point, in the
 *              order the forest was built from
 *   n_kept     host or NULL; number of kept points
 *   out        host; receives the forest
 * Synchronises on `stream` twice (the kept count, then the set sizes), or
 * three times with a crop.
 */
capt_status capt_build_filtered(const float *xyz, int64_t n, float r_filter,
                                const float *crop, float r_min, float r_max, uint32_t flags,
                                int32_t *kept_index, int64_t *n_kept,
                                void *stream, capt_forest *out);

/*
 * CollisionCheck (Alg. 3, Sec. IV-D) with configuration-level early exit.
 *   f          forest from capt_build / capt_import
 *   spheres    [M][4]; the spheres of cloud c are
 *              spheres[query_off[c] .. query_off[c+1])
 *   query_off  host [ncloud + 1], non-decreasing, each range a multiple of
 *              `group`
 *   group      1 .. 2^20 spheres per configuration
 *   out        [M / group] bytes; out[k] = 1 iff some sphere of configuration
 *              k touches its cloud, else 0
 *   flags      CAPT_CHECK_RADII, CAPT_PER_CLOUD, CAPT_NO_GRAPH
 * Radii must lie in [r_min, r_max] of the forest (Lemma 1); outside it the
 * answer is unspecified, or CAPT_ERADIUS with CAPT_CHECK_RADII.  Non-finite
 * centres give 0.  A forest with more than one cloud is queried with one
 * persistent launch over a cost-sorted tile queue, replayed from a cached
 * hipGraph when `spheres`, `out`, `query_off` and `group` repeat.
 */
capt_status capt_collides(capt_forest f, const float *spheres, const int64_t *query_off,
                          int32_t group, uint8_t *out, uint32_t flags, void *stream);

/*
 * capt_collides that allocates nothing, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments and answers as capt_collides, always
 * one launch per cloud (the kernels of capt_collides with CAPT_PER_CLOUD).  The
 * work-queue counters of the launches live in a library-owned device array of
 * CAPT_NOALLOC_MAX_CLOUDS x 8 counters (128 KiB per GPU, held until the
 * process ends), found once per device; every launch clears its cloud's
 * counters with a fill kernel first.
 *   flags      0 (CAPT_CHECK_RADII needs a host read-back and is refused)
 * A forest of more than CAPT_NOALLOC_MAX_CLOUDS clouds gives
 * CAPT_EUNSUPPORTED.  Every call on one GPU shares that array: calls on one
 * stream are ordered and safe, calls that overlap on one GPU (different
 * streams, different threads) race on the counters and give wrong answers.
 */
#define CAPT_NOALLOC_MAX_CLOUDS 256
capt_status capt_collides_noalloc(capt_forest f, const float *spheres, const int64_t *query_off,
                                  int32_t group, uint8_t *out, uint32_t flags, void *stream);

/*
 * Diagnostic form of capt_collides that checks the batched kernel's work
 * queue: the same answers, always from one launch of the batched kernel over
 * all clouds (tiles of configurations popped from one queue; no graph, no
 * cached plan), which also adds 1 to visits[k] each time it decides
 * configuration k.  With visits zeroed beforehand every entry reads 1 after
 * the call: each configuration lies in exactly one tile and each tile is
 * taken exactly once.
 *   visits  [M / group] int32 (device), added to with atomics
 * Other arguments as capt_collides (flags are implied 0).  Synchronises the
 * stream before it returns.  Forests built with per-depth split axes
 * (capt_build_axes) give CAPT_EUNSUPPORTED.
 */
capt_status capt_collides_visits(capt_forest f, const float *spheres, const int64_t *query_off,
                                 int32_t group, uint8_t *out, int32_t *visits, void *stream);

/*
 * capt_collides with query padding (Sec. V-B, after the filter lemma): every
 * radius r becomes fl(r + pad) before the test, so that a forest built from a
 * filtered cloud answers conservatively (pad = r_filter per filter pass that
 * removed points: a dropped point lies within r_filter of a point its pass
 * kept).  Every padded radius must lie in [r_min, r_max] of the forest
 * (CAPT_CHECK_RADII validates that).  Same arguments as capt_collides; pad is
 * finite and >= 0; flags: 0 or CAPT_CHECK_RADII.  Forests of several clouds
 * take one launch per cloud.
 */
capt_status capt_collides_padded(capt_forest f, const float *spheres,
                                 const int64_t *query_off, int32_t group, float pad,
                                 uint8_t *out, uint32_t flags, void *stream);

/*
 * CollisionCheck (Alg. 3) on robot configurations given as rigid poses of one
 * sphere template, grouped into edges (runs of consecutive configurations, as
 * a planner validates a motion) with early exit at the first colliding sphere
 * of an edge in order (configurations in order, spheres in template order).
 * Reading the template and a 48-byte pose per configuration replaces reading
 * g materialised spheres.
 *   tmpl      [g][4] template spheres (x, y, z, r) in the robot frame;
 *             1 <= g <= 1024
 *   poses     [P][12] per configuration: rotation R row-major (9 floats), then
 *             translation t (3 floats); sphere k of configuration c is centred
 *             at ((R0 x + R1 y) + R2 z) + t0, ((R3 x + R4 y) + R5 z) + t1,
 *             ((R6 x + R7 y) + R8 z) + t2, every product and sum rounded to
 *             float32 on its own, radius r
 *   pose_off  host [ncloud + 1]: the poses of cloud c are
 *             poses[pose_off[c] .. pose_off[c+1]), each range a multiple of edge
 *   edge      configurations per edge (edge * g <= 2^20)
 *   out       [P / edge] bytes; out[k] = 1 iff some sphere of some configuration
 *             of edge k touches its cloud (the float32 predicate of
 *             capt_collides), else 0
 *   flags     CAPT_CHECK_RADII (template radii against [r_min, r_max]) or 0
 * Asynchronous on `stream`; CAPT_EINVAL on bad arguments.  The answers equal
 * capt_collides on the materialised spheres with group = edge * g.
 */
capt_status capt_collides_posed(capt_forest f, const float *tmpl, int32_t g, const float *poses,
                                const int64_t *pose_off, int32_t edge, uint8_t *out, uint32_t flags,
                                void *stream);

/*
 * Clearance of each sphere: c = min(d, r_max) - r, with d the float32
 * distance from the centre to the nearest point of the sphere's leaf
 * affordance set (equal to the nearest point of the whole cloud whenever
 * d < r_max, by Lemma 1 case 1).  witness = original index of that point
 * (smallest index on ties), or -1 when d >= r_max.  The forest must have no
 * pruned leaf (build it with CAPT_NO_PRUNE or r_min = 0), else CAPT_EPRUNED.
 *   spheres    [M][4];  query_off  host [ncloud + 1]
 *   clearance  [M] float32;  witness  [M] int32
 */
capt_status capt_clearance(capt_forest f, const float *spheres, const int64_t *query_off,
                           float *clearance, int32_t *witness, void *stream);

/*
 * Backward of capt_clearance (the clearance is c = min(d, r_max) - r): for
 * each sphere, with g = grad_clearance[s] and p* the witness point of its
 * cloud,
 *   grad_center[s] = g * (x - p*) / |x - p*|   if witness >= 0 and x != p*
 *                    (0, 0, 0)                  otherwise (clamped, or x = p*)
 *   grad_radius[s] = -g
 * The direction is computed in float32: d = x - p* per axis, |d| as the
 * correctly rounded square root of ((dx*dx + dy*dy) + dz*dz).
 *   spheres        [M][4];  query_off  host [ncloud + 1]
 *   witness        [M] int32 from capt_clearance on the same spheres and forest
 *                  (-1 or an index into that cloud's capt_build input)
 *   grad_clearance [M] float32
 *   grad_center    [M][3] float32 (d/dx, d/dy, d/dz)
 *   grad_radius    [M] float32, or NULL to skip it
 * Asynchronous on `stream`.  CAPT_EPRUNED on a forest with pruned leaves;
 * CAPT_EINVAL for NULL buffers with M > 0.  A witness outside the cloud's
 * index range is not detected (it comes from capt_clearance).
 */
capt_status capt_clearance_backward(capt_forest f, const float *spheres,
                                    const int64_t *query_off, const int32_t *witness,
                                    const float *grad_clearance, float *grad_center,
                                    float *grad_radius, void *stream);

/* Release a forest's device memory (waits for the device first).  NULL is a no-op. */
void capt_destroy(capt_forest f);

/* Release a forest's device memory in stream order on `stream`, without
 * waiting: the caller has ordered every use of the forest (its build, every
 * query, clearance and stats call) on `stream` before this call, or made
 * `stream` wait for them.  The handle is invalid on return.  A forest that
 * holds a captured batched launch (a capt_collides call over several clouds)
 * waits for the device first, as capt_destroy does.  NULL is a no-op. */
void capt_destroy_async(capt_forest f, void *stream);

/* Thread-local description of the last failure on this thread ("" if none). */
const char *capt_last_error(void);

/*
 * Per-cloud sizes of a forest (host outputs, any may be NULL).
 *   n: real points; D: depth (N = 2^D leaves); set_total: stored set entries
 *   (without alignment padding); pruned: pruned leaves; bytes: device bytes
 */
capt_status capt_forest_info(capt_forest f, int32_t cloud, int64_t *n, int32_t *D,
                             int64_t *set_total, int64_t *pruned, int64_t *bytes);

/*
 * Export cloud `cloud` of a forest to a host blob, or import a one-cloud
 * forest from one.  With host_blob == NULL, capt_export only writes the
 * required size to *bytes.  Export synchronises.  Blob layout (little endian,
 * every section starts at a multiple of 8 bytes):
 *   header   uint32 magic 0x54504143 ("CAPT"), uint32 version (1 or 2),
 *            int64 n, int64 N, int32 D, uint32 flags, float r_min, float r_max,
 *            int64 set_total (S)                                  (48 bytes)
 *   uint64   axes                version 2 only: bits 2d, 2d+1 hold the split
 *                                axis (0 x, 1 y, 2 z) of depth d < D, all
 *                                higher bits 0.  Export writes version 2 for a
 *                                forest from capt_build_axes whose axes are
 *                                not the cyclic d mod 3, version 1 otherwise
 *                                (version 1 means d mod 3)
 *   float    points [n][3]       the cloud as given to capt_build
 *   float    T [N-1]             test sequence (Eytzinger order)
 *   int32    rep [N]             representative index per leaf (>= n: padding)
 *   float    aabb [N][6]         lo xyz, hi xyz of each stored set
 *   uint8    pruned [N]
 *   int64    set_off [N+1]       set of leaf l is entries set_off[l] .. set_off[l+1]
 *   int32    set_idx [S]         original point indices in stored (scan) order
 * capt_import checks the header (D <= 30, N = 2^D, n <= N < 2n, S < 2^30),
 * the blob size, that the N + 1 set offsets start at 0, never decrease and
 * end at S before any set is read, that every set entry and representative is
 * in range, every point is finite and every AABB is the bounding box of its
 * set (CAPT_EINVAL otherwise); it does not re-derive the sets.  Import
 * synchronises.
 */
capt_status capt_export(capt_forest f, int32_t cloud, void *host_blob, size_t *bytes);
capt_status capt_import(const void *host_blob, size_t bytes, void *stream, capt_forest *out);

/*
 * Device memory hooks for forests and scratch.  alloc returns NULL on failure.
 * Passing NULL for both restores the default, the device's stream-ordered pool
 * (hipMallocAsync / hipFreeAsync).  The stream handed to the hooks is the one
 * the memory is used on in order: the caller's stream, or a side stream the
 * library forks from it (a build's grid binning runs on one) and joins back
 * into it before the entry point's work ends on the caller's stream.  Not thread-safe with respect to concurrent entry points.
 */
capt_status capt_set_allocator(void *(*alloc)(size_t bytes, void *stream, void *ctx),
                               void (*release)(void *ptr, void *stream, void *ctx),
                               void *ctx);

/*
 * GPU brute force (the baseline of the benchmark): every sphere against every
 * point of its cloud with the same predicate, one launch per cloud, one
 * wavefront per configuration, exiting at the first hit.
 *   xyz, cloud_off, ncloud as in capt_build; spheres, query_off, group, out
 *   as in capt_collides.
 */
capt_status capt_bruteforce_collides(const float *xyz, const int64_t *cloud_off,
                                     int32_t ncloud, const float *spheres,
                                     const int64_t *query_off, int32_t group,
                                     uint8_t *out, void *stream);

/*
 * Work accounting for one collision query (not on the hot path): per sphere,
 * the leaf reached, whether the leaf AABB rejected it, how many set entries a
 * scan in stored order tests up to and including its first hit (the whole set
 * if none), and whether it hit.  Any output may be NULL.
 *   leaf [M] int32, rejected [M] uint8, scanned [M] int32, hit [M] uint8
 */
capt_status capt_query_stats(capt_forest f, const float *spheres, const int64_t *query_off,
                             int32_t *leaf, uint8_t *rejected, int32_t *scanned, uint8_t *hit,
                             void *stream);

/*
 * Work of the collision kernel's two-level set scan (not on the hot path).
 * capt_collides stores every set as chunks of 16 entries, each with a
 * bounding box, tests the boxes and scans only the entries of chunks whose
 * box lies within the sphere's radius; a box is never farther than any of its
 * points, so the answers are those of the full scan of Alg. 3.  A chunk's box
 * is kept as half-precision offsets from the lower corner b of its set's box
 * (the leaf AABB): per axis, the lower bound's offset is the nearest half to
 * lo - b (float32), then moved down one half at a time while b + offset > lo
 * in float32, the upper bound's likewise moved up while b + offset < hi; the
 * test uses the box b + offset.  Per sphere
 * whose leaf AABB does not reject it, for a scan in stored order up to and
 * including the chunk that holds its first hit (all chunks if none):
 *   boxes  [M] int32  chunk boxes tested
 *   chunks [M] int32  chunks whose 16 entries were tested
 * Both are 0 for a rejected sphere.  Either output may be NULL.
 */
capt_status capt_query_chunk_stats(capt_forest f, const float *spheres, const int64_t *query_off,
                                   int32_t *boxes, int32_t *chunks, void *stream);

/*
 * Launch shape of the collision kernels (chosen by the autotuner).
 *   waves_per_group  wavefronts per workgroup (1 .. 16)
 *   groups_per_cu    persistent workgroups per compute unit (1 .. 16)
 *   tile_cfgs        configurations a wavefront takes per queue pop in the
 *                    batched kernel (1 .. 4096)
 *   lds_levels       tree levels kept in LDS (1 .. 15; fewer if they do not fit)
 *   scan_unroll      64-lane steps of the entry scan kept in flight, 4 chunks
 *                    per step (1, 2 or 4)
 * Zero fields keep their current value.  Applies to later calls.
 */
typedef struct {
    int32_t waves_per_group;
    int32_t groups_per_cu;
    int32_t tile_cfgs;
    int32_t lds_levels;
    int32_t scan_unroll;
} capt_tuning;

capt_status capt_set_tuning(const capt_tuning *t);
capt_status capt_get_tuning(capt_tuning *t);

/*
 * Achievable-bandwidth yardsticks (measurement only, not the hot path).  The
 * benchmark divides a query's algorithmic bytes by what these reach, to state
 * how close the query runs to the memory roofline it can actually attain.
 *
 * capt_probe_read: reads the buffer's float4s `passes` times over (bytes / 16
 * float4s; a tail below 16 bytes is not read), each of the 8 XCDs one eighth
 * of the buffer with blocks_per_cu x (compute units) blocks of 256 threads
 * in all.  A buffer far larger than the caches measures HBM; one whose eighth
 * fits an XCD's L2 (4 MB) or whose whole fits the MALL measures that level.
 *   buf            device, 16-byte aligned
 *   blocks_per_cu  1 .. 32
 *   sink           device [1] float; written only if the loads sum to -1
 *
 * capt_probe_gather: the collision query's memory pattern without its
 * arithmetic.  Item k (16 bytes, int32 leaf, len, unused, unused) reads
 * leaves[leaf] (32 bytes: float lo[3], hi[3], uint32 start, uint32 count),
 * then entries start .. start + min(len, count) - 1 of x, y and z, and writes
 * out[k] (1 iff the sum of the loads is -1).  Items whose leaf is outside
 * [0, nleaf) read nothing past their descriptor; runs are cut at `entries`.
 *   items          device [m][4] int32
 *   leaves         device [nleaf] records as above
 *   x, y, z        device [entries] float32
 *   lanes_per_item 16 or 64: the lanes that share one item's run
 *   out            device [m] bytes
 * Both are asynchronous on `stream`; CAPT_EINVAL on bad arguments.
 */
capt_status capt_probe_read(const void *buf, size_t bytes, int32_t passes, int32_t blocks_per_cu, float *sink,
                            void *stream);
capt_status capt_probe_gather(const int32_t *items, int64_t m, const void *leaves, int64_t nleaf,
                              const float *x, const float *y, const float *z, int64_t entries,
                              int32_t lanes_per_item, uint8_t *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CAPT_H */
