/*
 * CPU oracle for collision-affording point trees (CAPTs).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no code,
 * header, table or helper with the GPU library; it is written directly from the
 * paper (Ramsey, Kingston, Thomason, Kavraki, "Collision-Affording Point Trees",
 * arXiv 2406.02807) and is deliberately plain and slow.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared
 * (contraction off so every float/double product and sum rounds on its own;
 * x86-64 SSE arithmetic has FLT_EVAL_METHOD == 0).
 *
 * Readings the paper leaves open:
 *  - distance test (Alg. 3 and Sec. IV-D): a sphere (x, r) touches p iff
 *    fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)) <= fl(r*r) in float32, with
 *    dx = fl(x_x - p_x) etc.: closed ball, no square root, no fused multiply-add.
 *  - traversal tie (Alg. 3 vs. the prose of Sec. IV-D): x_d <= T_i goes left.
 *  - median (Sec. III, Alg. 1): rank split of the node's points under the
 *    strict order (coordinate, original index); the left half is the first
 *    |PC|/2 points and T_i is the coordinate of the last of them.
 *  - "c affords p at r_max" (Sec. IV-A): float64 distance from p to the closed
 *    cell (bounds may be infinite) compared with R = r_max (1 + 2^-20).
 *  - r_min pruning (Alg. 1, Sec. IV-B): prune iff r_min > 0, the cell is
 *    bounded, and the float64 squared distance from the representative to the
 *    farthest cell corner is <= r_min^2 (1 - 2^-18).
 *  - padding (Sec. IV-A): points at (+inf, +inf, +inf) with index >= n take part
 *    in the splits but are never stored in an affordance set.
 *  - Morton key (Sec. II-B, Alg. 2): 21-bit grid on the input cloud's cubic
 *    bounding box; key bit 3b + (2 - j) is bit b of the cell coordinate on
 *    axis X[j]; permutations in lexicographic order; stable sort; a point is
 *    kept iff its float32 squared distance to the last kept point exceeds
 *    fl(r_f * r_f).
 *  - clearance (not in the paper): min(min_p ||x - p||, r_max) - r in float64
 *    over all points, witness = smallest index attaining the minimum, -1 when
 *    the clamp is active.
 */
#define _GNU_SOURCE
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

/* Thread count of the OpenMP loops (the benchmark times the query on one
 * thread and on all host cores). */
ORC_API void orc_set_threads(int32_t k) { omp_set_num_threads(k > 0 ? k : 1); }
ORC_API int32_t orc_max_threads(void) { return (int32_t)omp_get_max_threads(); }

/* ------------------------------------------------------------------------- */
/* The float32 sphere-point predicate (Alg. 3, "||x - p|| <= r").            */
/* ------------------------------------------------------------------------- */
static float sqdist_f32(const float *a, const float *b)
{
    float dx = a[0] - b[0];
    float dy = a[1] - b[1];
    float dz = a[2] - b[2];
    float sx = dx * dx;
    float sy = dy * dy;
    float sz = dz * dz;
    float s = sx + sy;
    s = s + sz;
    return s;
}

static int touches_f32(const float *sphere, const float *p)
{
    float r2 = sphere[3] * sphere[3];
    return sqdist_f32(sphere, p) <= r2;
}

ORC_API float orc_sqdist_f32(const float *a, const float *b) { return sqdist_f32(a, b); }

/* O1: brute force, float32 predicate.  out[c] = 1 iff some sphere of group c
 * (spheres c*g .. c*g+g-1) touches some point.  m must be a multiple of g. */
/* Spheres of a template under rigid poses (the posed query's definition):
 * sphere k of configuration c is template sphere k with centre
 * ((R0 x + R1 y) + R2 z) + t0, ((R3 x + R4 y) + R5 z) + t1,
 * ((R6 x + R7 y) + R8 z) + t2, every product and sum in float32, radius kept;
 * pose c = R row-major (9 floats), then t (3 floats).  out [P * g][4],
 * configuration-major. */
ORC_API void orc_pose_spheres(const float *tmpl, int32_t g, const float *poses, int64_t P, float *out)
{
    for (int64_t c = 0; c < P; ++c) {
        const float *R = poses + 12 * c;
        for (int32_t k = 0; k < g; ++k) {
            const float x = tmpl[4 * k], y = tmpl[4 * k + 1], z = tmpl[4 * k + 2];
            float *o = out + 4 * (c * g + k);
            for (int i = 0; i < 3; ++i) {
                float a = R[3 * i] * x;
                float b = R[3 * i + 1] * y;
                float s = a + b;
                float d = R[3 * i + 2] * z;
                s = s + d;
                o[i] = s + R[9 + i];
            }
            o[3] = tmpl[4 * k + 3];
        }
    }
}

ORC_API void orc_brute_f32(const float *pts, int64_t n, const float *sph, int64_t m,
                           int32_t g, uint8_t *out)
{
    int64_t ncfg = m / g;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < ncfg; ++c) {
        int hit = 0;
        for (int64_t s = c * g; s < (c + 1) * g && !hit; ++s)
            for (int64_t j = 0; j < n && !hit; ++j)
                hit = touches_f32(sph + 4 * s, pts + 3 * j);
        out[c] = (uint8_t)hit;
    }
}

/* O2: the same test in float64 on the float32 inputs, per sphere, plus the
 * smallest relative margin |d^2 - r^2| / r^2 over all points. */
ORC_API void orc_brute_f64(const float *pts, int64_t n, const float *sph, int64_t m,
                           uint8_t *out, double *margin)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < m; ++s) {
        const float *q = sph + 4 * s;
        double r2 = (double)q[3] * (double)q[3];
        int hit = 0;
        double best = INFINITY;
        for (int64_t j = 0; j < n; ++j) {
            const float *p = pts + 3 * j;
            double dx = (double)q[0] - (double)p[0];
            double dy = (double)q[1] - (double)p[1];
            double dz = (double)q[2] - (double)p[2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 <= r2) hit = 1;
            double mg = fabs(d2 - r2) / r2;
            if (mg < best) best = mg;
        }
        out[s] = (uint8_t)hit;
        if (margin) margin[s] = best;
    }
}

/* O3: clearance in float64 over all points.  clr = min(d_min, r_max) - r,
 * witness = smallest index with the minimal squared distance, or -1 when
 * d_min >= r_max.  grad = d clr / d x = (x - p*) / ||x - p*|| when the witness
 * exists and d_min > 0, else 0 (d clr / d r = -1 always). */
ORC_API void orc_clearance_f64(const float *pts, int64_t n, const float *sph, int64_t m,
                               float r_max, double *clr, int32_t *witness, double *grad)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t s = 0; s < m; ++s) {
        const float *q = sph + 4 * s;
        double best = INFINITY;
        int64_t arg = -1;
        for (int64_t j = 0; j < n; ++j) {
            const float *p = pts + 3 * j;
            double dx = (double)q[0] - (double)p[0];
            double dy = (double)q[1] - (double)p[1];
            double dz = (double)q[2] - (double)p[2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < best) { best = d2; arg = j; }
        }
        double d = sqrt(best);
        double g[3] = {0.0, 0.0, 0.0};
        if (arg >= 0 && d < (double)r_max) {
            clr[s] = d - (double)q[3];
            witness[s] = (int32_t)arg;
            if (d > 0.0)
                for (int a = 0; a < 3; ++a)
                    g[a] = ((double)q[a] - (double)pts[3 * arg + a]) / d;
        } else {
            clr[s] = (double)r_max - (double)q[3];
            witness[s] = -1;
        }
        if (grad)
            for (int a = 0; a < 3; ++a) grad[3 * s + a] = g[a];
    }
}

/* ------------------------------------------------------------------------- */
/* O4: Construct (Alg. 1), sequential and recursive, carrying the cell c and */
/* the afforded set z exactly as Sec. IV-B describes.                        */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t n, N;          /* real points, padded size 2^D */
    int32_t D;
    float r_min, r_max;
    int prune;
    uint8_t axes[64];      /* split axis of every depth (d mod 3 unless given) */
    const float *pts;      /* [n][3] input */
    float *T;              /* [N-1] test sequence, Eytzinger order */
    int32_t *rep;          /* [N] representative index per leaf (>= n: padding) */
    float *cell;           /* [N][6] lo xyz, hi xyz */
    float *aabb;           /* [N][6] lo xyz, hi xyz of the stored set */
    uint8_t *pruned;       /* [N] */
    int64_t *cnt;          /* [N] set sizes */
    int32_t **sets;        /* [N] sorted original indices */
    int64_t *off;          /* [N+1] after finalisation */
    int32_t *idx;          /* flattened sets */
    int no_sets;           /* splits only: no affordance sets, AABBs or pruning */
} orc_tree;

ORC_API void orc_tree_free(orc_tree *t);

static double R_afford2(float r_max)
{
    double R = (double)r_max * (1.0 + 0x1p-20);
    return R * R;
}

/* c affords p at r_max: float64 distance from p to the closed cell c. */
static int affords(const float *c, const float *p, double R2)
{
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double below = (double)c[a] - (double)p[a];      /* lo - p */
        double above = (double)p[a] - (double)c[3 + a];  /* p - hi */
        double g = below > above ? below : above;
        if (g < 0.0) g = 0.0;
        d2 = d2 + g * g;
    }
    return d2 <= R2;
}

/* Every q in the cell is within r_min of the representative t (float64
 * farthest-corner test with a relative margin of 2^-18). */
static int prunable(const float *c, const float *t, float r_min)
{
    if (!(r_min > 0.0f)) return 0;
    for (int a = 0; a < 6; ++a)
        if (!isfinite(c[a])) return 0;
    double far2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double lo = (double)t[a] - (double)c[a];
        double hi = (double)c[3 + a] - (double)t[a];
        double l2 = lo * lo, h2 = hi * hi;
        far2 = far2 + (l2 > h2 ? l2 : h2);
    }
    double thr = ((double)r_min * (double)r_min) * (1.0 - 0x1p-18);
    return far2 <= thr;
}

ORC_API int orc_prunable(const float *cell, const float *t, float r_min)
{
    return prunable(cell, t, r_min);
}

typedef struct {
    const float *pts;
    int64_t n;
    int axis;
} sort_ctx;

static float coord(const sort_ctx *s, int32_t i)
{
    return i < s->n ? s->pts[3 * (int64_t)i + s->axis] : INFINITY;
}

static int cmp_coord_index(const void *a, const void *b, void *ctx)
{
    const sort_ctx *s = (const sort_ctx *)ctx;
    int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
    float u = coord(s, i), v = coord(s, j);
    if (u < v) return -1;
    if (u > v) return 1;
    return (i > j) - (i < j);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
    return (i > j) - (i < j);
}

static const float INF3[3] = {INFINITY, INFINITY, INFINITY};

static const float *point(const orc_tree *t, int32_t i)
{
    return i < t->n ? t->pts + 3 * (int64_t)i : INF3;
}

static void construct(orc_tree *t, int32_t *pc, int64_t m, float c[6],
                      int32_t *z, int64_t nz, int64_t i, int depth)
{
    double R2 = R_afford2(t->r_max);
    if (m == 1) {
        int64_t leaf = i - (t->N - 1);
        int32_t x = pc[0];
        memcpy(t->cell + 6 * leaf, c, 6 * sizeof(float));
        t->rep[leaf] = x;
        if (t->no_sets) {
            t->sets[leaf] = (int32_t *)malloc(sizeof(int32_t));
            return;
        }
        int real = x < t->n;
        int pr = real && t->prune && prunable(c, point(t, x), t->r_min);
        int64_t k = 0;
        int32_t *set = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nz + 1));
        if (real) set[k++] = x;
        if (!pr)
            for (int64_t j = 0; j < nz; ++j) set[k++] = z[j];
        qsort(set, (size_t)k, sizeof(int32_t), cmp_i32);
        float *bb = t->aabb + 6 * leaf;
        for (int a = 0; a < 3; ++a) { bb[a] = INFINITY; bb[3 + a] = -INFINITY; }
        for (int64_t j = 0; j < k; ++j) {
            const float *p = point(t, set[j]);
            for (int a = 0; a < 3; ++a) {
                if (p[a] < bb[a]) bb[a] = p[a];
                if (p[a] > bb[3 + a]) bb[3 + a] = p[a];
            }
        }
        t->pruned[leaf] = (uint8_t)pr;
        t->cnt[leaf] = k;
        t->sets[leaf] = set;
        return;
    }
    /* median split along the axis of this depth under (coordinate, index) */
    const int d = t->axes[depth];
    sort_ctx sc = {t->pts, t->n, d};
    qsort_r(pc, (size_t)m, sizeof(int32_t), cmp_coord_index, &sc);
    int64_t h = m / 2;
    float Ti = coord(&sc, pc[h - 1]);
    t->T[i] = Ti;
    int32_t *B1 = pc, *B2 = pc + h;
    float c1[6], c2[6];
    memcpy(c1, c, sizeof c1);
    memcpy(c2, c, sizeof c2);
    c1[3 + d] = Ti;   /* shrink the upper bound of c1 */
    c2[d] = Ti;       /* raise the lower bound of c2 */
    /* z1 = {p in z u B2 : c1 affords p}, z2 = {p in z u B1 : c2 affords p};
     * padding points are never afforded. */
    int32_t *z1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(t->no_sets ? 1 : nz + h + 1));
    int32_t *z2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(t->no_sets ? 1 : nz + h + 1));
    int64_t n1 = 0, n2 = 0;
    for (int64_t j = 0; j < nz; ++j) {
        const float *p = point(t, z[j]);
        if (affords(c1, p, R2)) z1[n1++] = z[j];
        if (affords(c2, p, R2)) z2[n2++] = z[j];
    }
    for (int64_t j = 0; j < h && !t->no_sets; ++j) {
        if (B2[j] < t->n && affords(c1, point(t, B2[j]), R2)) z1[n1++] = B2[j];
        if (B1[j] < t->n && affords(c2, point(t, B1[j]), R2)) z2[n2++] = B1[j];
    }
    /* each child re-sorts only its own half of pc */
    construct(t, B1, h, c1, z1, n1, 2 * i + 1, depth + 1);
    free(z1);
    construct(t, B2, h, c2, z2, n2, 2 * i + 2, depth + 1);
    free(z2);
}

/* axes: the split axis (0, 1, 2) of each depth 0 .. D-1, or NULL for the
 * cyclic rule d mod 3 of Sec. IV-A (the paper names a random choice of axis
 * as an alternative; here a sequence of axes per depth keeps the tree
 * implicit). */
static orc_tree *build(const float *pts, int64_t n, float r_min, float r_max, int prune,
                       const uint8_t *axes, int no_sets)
{
    orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
    t->no_sets = no_sets;
    int64_t N = 1;
    int D = 0;
    while (N < n) { N <<= 1; ++D; }
    for (int d = 0; d < 64; ++d) t->axes[d] = (uint8_t)(axes && d < D ? axes[d] : d % 3);
    t->n = n; t->N = N; t->D = D;
    t->r_min = r_min; t->r_max = r_max; t->prune = prune;
    t->pts = pts;
    t->T = (float *)calloc((size_t)(N > 1 ? N - 1 : 1), sizeof(float));
    t->rep = (int32_t *)calloc((size_t)N, sizeof(int32_t));
    t->cell = (float *)calloc((size_t)N * 6, sizeof(float));
    t->aabb = (float *)calloc((size_t)N * 6, sizeof(float));
    t->pruned = (uint8_t *)calloc((size_t)N, 1);
    t->cnt = (int64_t *)calloc((size_t)N, sizeof(int64_t));
    t->sets = (int32_t **)calloc((size_t)N, sizeof(int32_t *));
    t->off = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    int32_t *pc = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    for (int64_t j = 0; j < N; ++j) pc[j] = (int32_t)j;
    float c[6] = {-INFINITY, -INFINITY, -INFINITY, INFINITY, INFINITY, INFINITY};
    if (n == 0) {
        /* empty cloud: one leaf holding nothing */
        t->rep[0] = 0;
        memcpy(t->cell, c, sizeof c);
        for (int a = 0; a < 3; ++a) { t->aabb[a] = INFINITY; t->aabb[3 + a] = -INFINITY; }
        t->sets[0] = (int32_t *)malloc(sizeof(int32_t));
    } else {
        construct(t, pc, N, c, NULL, 0, 0, 0);
    }
    free(pc);
    for (int64_t l = 0; l < N; ++l) t->off[l + 1] = t->off[l] + t->cnt[l];
    t->idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(t->off[N] > 0 ? t->off[N] : 1));
    for (int64_t l = 0; l < N; ++l) {
        memcpy(t->idx + t->off[l], t->sets[l], sizeof(int32_t) * (size_t)t->cnt[l]);
        free(t->sets[l]);
    }
    free(t->sets);
    t->sets = NULL;
    return t;
}

ORC_API orc_tree *orc_build(const float *pts, int64_t n, float r_min, float r_max, int prune,
                            const uint8_t *axes)
{
    return build(pts, n, r_min, r_max, prune, axes, 0);
}

/* Construct's splits alone (Sec. IV-A): T and the representative of every
 * leaf, without affordance sets; the same recursion as orc_build. */
ORC_API void orc_build_splits(const float *pts, int64_t n, const uint8_t *axes, float *T, int32_t *rep)
{
    orc_tree *t = build(pts, n, 0.0f, 1.0f, 0, axes, 1);
    if (T && t->N > 1) memcpy(T, t->T, sizeof(float) * (size_t)(t->N - 1));
    if (rep) memcpy(rep, t->rep, sizeof(int32_t) * (size_t)t->N);
    orc_tree_free(t);
}

/* The closed cell of every leaf from the test sequence alone (Alg. 1: a
 * left descent at node i caps the cell at T_i on the node's axis, a right
 * descent raises its lower bound to T_i; bounds never met stay infinite).
 * Leaf l is reached by the bits of l, most significant first, 1 = right. */
ORC_API void orc_leaf_cells(int64_t N, int32_t D, const float *T, const uint8_t *axes, float *cells)
{
    for (int64_t l = 0; l < N; ++l) {
        float c[6] = {-INFINITY, -INFINITY, -INFINITY, INFINITY, INFINITY, INFINITY};
        int64_t i = 0;
        for (int d = 0; d < D; ++d) {
            const int a = axes ? axes[d] : d % 3;
            if ((l >> (D - 1 - d)) & 1) {
                c[a] = T[i];
                i = 2 * i + 2;
            } else {
                c[3 + a] = T[i];
                i = 2 * i + 1;
            }
        }
        memcpy(cells + 6 * l, c, sizeof c);
    }
}

/* Lemma 1, case 1, written out: the affordance set of a closed cell is every
 * real point it affords at r_max, the set Construct's incremental z reaches.
 * orc_afford_count gives the size for each of k cells, orc_afford_fill the
 * members in increasing index order at the caller's offsets. */
ORC_API void orc_afford_count(const float *pts, int64_t n, const float *cells, int64_t k, float r_max,
                              int64_t *cnt)
{
    const double R2 = R_afford2(r_max);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t l = 0; l < k; ++l) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) c += affords(cells + 6 * l, pts + 3 * j, R2);
        cnt[l] = c;
    }
}

ORC_API void orc_afford_fill(const float *pts, int64_t n, const float *cells, int64_t k, float r_max,
                             const int64_t *off, int32_t *idx)
{
    const double R2 = R_afford2(r_max);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t l = 0; l < k; ++l) {
        int64_t c = off[l];
        for (int64_t j = 0; j < n; ++j)
            if (affords(cells + 6 * l, pts + 3 * j, R2)) idx[c++] = (int32_t)j;
    }
}

ORC_API void orc_tree_dims(const orc_tree *t, int64_t *n, int64_t *N, int32_t *D, int64_t *total)
{
    *n = t->n; *N = t->N; *D = t->D; *total = t->off[t->N];
}

ORC_API void orc_tree_copy(const orc_tree *t, float *T, int32_t *rep, float *cell, float *aabb,
                           uint8_t *pruned, int64_t *off, int32_t *idx)
{
    int64_t N = t->N;
    if (T && N > 1) memcpy(T, t->T, sizeof(float) * (size_t)(N - 1));
    if (rep) memcpy(rep, t->rep, sizeof(int32_t) * (size_t)N);
    if (cell) memcpy(cell, t->cell, sizeof(float) * 6 * (size_t)N);
    if (aabb) memcpy(aabb, t->aabb, sizeof(float) * 6 * (size_t)N);
    if (pruned) memcpy(pruned, t->pruned, (size_t)N);
    if (off) memcpy(off, t->off, sizeof(int64_t) * (size_t)(N + 1));
    if (idx) memcpy(idx, t->idx, sizeof(int32_t) * (size_t)t->off[N]);
}

ORC_API void orc_tree_free(orc_tree *t)
{
    if (!t) return;
    free(t->T); free(t->rep); free(t->cell); free(t->aabb); free(t->pruned);
    free(t->cnt); free(t->off); free(t->idx);
    free(t);
}

/* ------------------------------------------------------------------------- */
/* O5: CollisionCheck (Alg. 3) on a tree given as plain arrays: T [N-1],      */
/* AABBs [N][6], set offsets [N+1] and the set points in stored order         */
/* (xyz [total][3]).  Per sphere: the boolean, the leaf, whether the AABB    */
/* rejected, and m_s = points tested until the first hit (all if none).       */
/* ------------------------------------------------------------------------- */
static int aabb_rejects(const float *bb, const float *s)
{
    float dd[3];
    for (int a = 0; a < 3; ++a) {
        float below = bb[a] - s[a];
        float above = s[a] - bb[3 + a];
        float g = fmaxf(below, above);
        dd[a] = fmaxf(g, 0.0f);
    }
    float sx = dd[0] * dd[0];
    float sy = dd[1] * dd[1];
    float sz = dd[2] * dd[2];
    float b2 = sx + sy;
    b2 = b2 + sz;
    float r2 = s[3] * s[3];
    return b2 > r2;
}

ORC_API void orc_query(int64_t N, int32_t D, const float *T, const float *aabb,
                       const int64_t *off, const float *setxyz,
                       const float *sph, int64_t m,
                       uint8_t *hit, int32_t *leaf, uint8_t *rejected, int32_t *scanned,
                       const uint8_t *axes)
{
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < m; ++s) {
        const float *q = sph + 4 * s;
        int64_t i = 0;
        for (int lv = 0; lv < D; ++lv) {
            const int d = axes ? axes[lv] : lv % 3;
            if (q[d] <= T[i]) i = 2 * i + 1;
            else i = 2 * i + 2;
        }
        int64_t l = i - (N - 1);
        int h = 0, rej = 0;
        int32_t ms = 0;
        if (aabb_rejects(aabb + 6 * l, q)) {
            rej = 1;
        } else {
            for (int64_t j = off[l]; j < off[l + 1]; ++j) {
                ++ms;
                if (touches_f32(q, setxyz + 3 * j)) { h = 1; break; }
            }
        }
        hit[s] = (uint8_t)h;
        if (leaf) leaf[s] = (int32_t)l;
        if (rejected) rejected[s] = (uint8_t)rej;
        if (scanned) scanned[s] = ms;
    }
}

/* Single-threaded variant of O5 for timing against the paper's one-thread
 * figure; same arithmetic, no OpenMP. */
ORC_API void orc_query_serial(int64_t N, int32_t D, const float *T, const float *aabb,
                              const int64_t *off, const float *setxyz,
                              const float *sph, int64_t m, int32_t g, uint8_t *out,
                              const uint8_t *axes)
{
    for (int64_t c = 0; c < m / g; ++c) {
        int any = 0;
        for (int64_t s = c * g; s < (c + 1) * g && !any; ++s) {
            const float *q = sph + 4 * s;
            int64_t i = 0;
            for (int lv = 0; lv < D; ++lv) {
                const int d = axes ? axes[lv] : lv % 3;
                if (q[d] <= T[i]) i = 2 * i + 1;
                else i = 2 * i + 2;
            }
            int64_t l = i - (N - 1);
            if (aabb_rejects(aabb + 6 * l, q)) continue;
            for (int64_t j = off[l]; j < off[l + 1]; ++j)
                if (touches_f32(q, setxyz + 3 * j)) { any = 1; break; }
        }
        out[c] = (uint8_t)any;
    }
}

/* ------------------------------------------------------------------------- */
/* O6: Morton keys and Filter (Alg. 2).                                      */
/* ------------------------------------------------------------------------- */
static const int PERMS[6][3] = {
    {0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

/* Interleave three 21-bit cell coordinates: bit 3b + (2 - j) of the key is
 * bit b of q[X[j]], so the first axis of the permutation is the most
 * significant within every triple. */
ORC_API uint64_t orc_morton_key(const uint32_t q[3], int perm)
{
    uint64_t key = 0;
    for (int b = 0; b < 21; ++b)
        for (int j = 0; j < 3; ++j) {
            uint64_t bit = (q[PERMS[perm][j]] >> b) & 1u;
            key |= bit << (3 * b + (2 - j));
        }
    return key;
}

/* Grid of the Morton curve: float32 lower corner of the input cloud's bounding
 * box and 2^21 / E in float64, E the largest extent (0 when E == 0). */
ORC_API void orc_morton_grid(const float *pts, int64_t n, float lo[3], double *scale)
{
    float hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int64_t j = 0; j < n; ++j)
        for (int a = 0; a < 3; ++a) {
            float v = pts[3 * j + a];
            if (v < lo[a]) lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    double E = 0.0;
    for (int a = 0; a < 3 && n > 0; ++a) {
        double e = (double)hi[a] - (double)lo[a];
        if (e > E) E = e;
    }
    *scale = E > 0.0 ? 2097152.0 / E : 0.0;
}

ORC_API void orc_morton_cell(const float *p, const float lo[3], double scale, uint32_t q[3])
{
    for (int a = 0; a < 3; ++a) {
        double v = floor(((double)p[a] - (double)lo[a]) * scale);
        if (v < 0.0) v = 0.0;
        if (v > 2097151.0) v = 2097151.0;
        q[a] = (uint32_t)v;
    }
}

typedef struct {
    uint64_t key;
    int64_t pos;
} keyed;

static int cmp_keyed(const void *a, const void *b)
{
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->pos > y->pos) - (x->pos < y->pos);
}

/* Filter (Alg. 2) with the first `npass` permutations (6 for the full
 * filter).  out_idx receives the original indices of the kept points in their
 * final order; counts[p] the size after pass p.  Returns the kept count. */
ORC_API int64_t orc_filter(const float *pts, int64_t n, float r_filter, int npass,
                           int32_t *out_idx, int64_t *counts)
{
    if (n <= 0) {
        for (int p = 0; p < npass; ++p) if (counts) counts[p] = 0;
        return 0;
    }
    float lo[3];
    double scale;
    orc_morton_grid(pts, n, lo, &scale);
    float rf2 = r_filter * r_filter;
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    keyed *kv = (keyed *)malloc(sizeof(keyed) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) cur[j] = (int32_t)j;
    int64_t m = n;
    for (int p = 0; p < npass; ++p) {
        /* sort PC' along the Z-order curve of permutation p (stable) */
        for (int64_t j = 0; j < m; ++j) {
            uint32_t q[3];
            orc_morton_cell(pts + 3 * (int64_t)cur[j], lo, scale, q);
            kv[j].key = orc_morton_key(q, p);
            kv[j].pos = j;
        }
        qsort(kv, (size_t)m, sizeof(keyed), cmp_keyed);
        for (int64_t j = 0; j < m; ++j) tmp[j] = cur[kv[j].pos];
        /* greedy scan: keep j iff it is farther than r_filter from the last
         * kept point */
        int64_t i = 0;
        cur[0] = tmp[0];
        for (int64_t j = 1; j < m; ++j) {
            if (sqdist_f32(pts + 3 * (int64_t)cur[i], pts + 3 * (int64_t)tmp[j]) > rf2) {
                ++i;
                cur[i] = tmp[j];
            }
        }
        m = i + 1;
        if (counts) counts[p] = m;
    }
    memcpy(out_idx, cur, sizeof(int32_t) * (size_t)m);
    free(cur); free(tmp); free(kv);
    return m;
}
