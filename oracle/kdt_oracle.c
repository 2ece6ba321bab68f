/*
 * kdt_oracle.c -- plain, slow, single-threaded CPU oracle for the k-d tree
 * hot path (test infrastructure only).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the HIP path and must never
 * be called by it.
 *
 * What it computes, and where each piece comes from:
 *   - squared Euclidean distance (Eq. 1 with p = 2) in IEEE float32, summed
 *     left to right over the axes, every operation rounded on its own
 *     (build with -ffp-contract=off so that no multiply-add is fused);
 *   - the same distance on the D-torus of periods L_a (the periodic boundary
 *     conditions of Sec. 2.1 and Sec. 2.4): per axis the shorter way round,
 *     min(|x - q|, L - |x - q|), for coordinates in [0, L);
 *   - brute-force kNN, ball counts/lists and friends-of-friends groups: the
 *     plain definitions, O(N^2) (also on the torus);
 *   - the sliding-midpoint k-d tree of Sec. 2.1 (Algorithm 1, serial);
 *   - best-first kNN over that tree with a node min-heap and a candidate
 *     max-heap (Algorithm 2), results sorted at the end (Sec. 2.3);
 *   - recursive ball query with whole-node acceptance (Algorithm 3);
 *   - friends-of-friends grouping by union-find over ball queries (Sec. 4.1);
 *   - adaptive SPH particle-to-mesh deposit with the M4 cubic spline and
 *     per-particle normalisation (Sec. 4.2), and its adjoint, in float64;
 *   - brute-force kNN and ball counts/lists on float64 coordinates (the
 *     double-precision real kind of Sec. 2.4): the same definitions with the
 *     squared distance in IEEE float64, summed left to right over the axes.
 *
 * Readings of the paper taken here (it is silent or self-contradictory):
 *   - ties in squared distance are broken by the lower point index, so a kNN
 *     result is the k smallest (d2, index) keys in ascending order; rows are
 *     padded with (index -1, d2 +inf) when k exceeds n; a query that is itself
 *     a data point finds itself at distance 0;
 *   - the ball is closed: a point at squared distance exactly fl(r*r) is in;
 *     Algorithm 3 takes all points of a node whose farthest corner is inside
 *     and then stops descending that node (the listing omits the return);
 *   - Algorithm 2 reads the worst candidate before k candidates exist: the
 *     candidate heap starts filled with (+inf, INT32_MAX) sentinels;
 *   - a node is a leaf when it holds at most N_leaf points (Algorithm 1 uses
 *     "<=");  the split axis is the longest side of the node's tight point
 *     bounding box (ties: lowest axis); a node whose points all coincide is a
 *     leaf whatever its size;  when the midpoint leaves one side empty, the
 *     single extreme point nearest the plane (ties: lowest original index) is
 *     moved to the empty side;
 *   - friends-of-friends links i != j when d2(i, j) <= fl(l*l); the group
 *     label is the smallest point index of the connected component;
 *   - deposit: q = 2 r / H_i with H_i = max(h_i, cell), M4 profile
 *     w(q) = 1 - 1.5 q^2 + 0.75 q^3 (q < 1), 0.25 (2 - q)^3 (1 <= q < 2),
 *     0 beyond; cells outside the grid are dropped and the weights of each
 *     particle are normalised over the in-grid cells, so mass is conserved;
 *     cell (i, j, k) is centred at lo + (i + 1/2, j + 1/2, k + 1/2) * cell and
 *     the grid is stored x slowest, z fastest;
 *   - periodic deposit (the periodic boundaries of Sec. 2.4 applied to the
 *     mesh of Sec. 4.2): the mesh box is a 3-torus of periods n_a * cell; the
 *     distance from a particle to a cell centre takes per axis the shorter way
 *     round (as the torus metric of the queries); every H_i must be below half
 *     of every period, so no cell is reached twice, and no cell is dropped;
 *   - fixed-cloud deposits (the NGP, CIC and TSC schemes Sec. 4.2 compares
 *     against, after Hockney and Eastwood): per axis, with s the position in
 *     units of cells from the first cell centre, NGP puts weight 1 on the
 *     nearest centre, CIC weights 1 - f and f on the two centres around s,
 *     TSC 0.5 (0.5 - u)^2, 0.75 - u^2, 0.5 (0.5 + u)^2 on the nearest centre
 *     and its neighbours (u = s - nearest); the weight of a cell is the
 *     product over the axes.  On an open mesh the weights of cells outside are
 *     dropped and the rest renormalised (the paper calls the schemes
 *     conservative); on a periodic mesh indices wrap (n_a >= 3 cells).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

/* ------------------------------------------------------------------------ */
/* Distances (Eq. 1, p = 2), float32, fixed order, no contraction.          */
/* ------------------------------------------------------------------------ */

static float sq_dist(const float *p, const float *q, int d)
{
    float s = 0.0f;
    for (int a = 0; a < d; ++a) {
        float t = p[a] - q[a];
        float t2 = t * t;
        s = s + t2;
    }
    return s;
}

/* Squared distance on the D-torus with periods L[a] (Sec. 2.1: the metric of
 * a D-toroid; Sec. 2.4: periodic boundary conditions), for coordinates in
 * [0, L[a]): along each axis the gap |p - q| or the way round, L - |p - q|,
 * whichever is shorter; then squares summed as in sq_dist. */
static float torus_sq_dist(const float *p, const float *q, int d, const float *L)
{
    float s = 0.0f;
    for (int a = 0; a < d; ++a) {
        float g = fabsf(p[a] - q[a]);
        float w = L[a] - g;
        float t = w < g ? w : g;
        float t2 = t * t;
        s = s + t2;
    }
    return s;
}

/* Open boundaries (L == NULL) or the torus. */
static float metric_sq_dist(const float *p, const float *q, int d, const float *L)
{
    return L ? torus_sq_dist(p, q, d, L) : sq_dist(p, q, d);
}

/* Every coordinate of the n x d array inside [0, L[a]). */
static int inside_period(const float *x, int64_t n, int d, const float *L)
{
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < d; ++a)
            if (!(x[i * d + a] >= 0.0f && x[i * d + a] < L[a])) return 0;
    return 1;
}

/* Smallest squared distance from q to any point of the box [lo, hi]. */
static float box_min_dist(const float *q, const float *lo, const float *hi, int d)
{
    float s = 0.0f;
    for (int a = 0; a < d; ++a) {
        float t = 0.0f;
        if (q[a] < lo[a]) t = lo[a] - q[a];
        else if (q[a] > hi[a]) t = q[a] - hi[a];
        float t2 = t * t;
        s = s + t2;
    }
    return s;
}

/* Largest squared distance from q to any point of the box [lo, hi]. */
static float box_max_dist(const float *q, const float *lo, const float *hi, int d)
{
    float s = 0.0f;
    for (int a = 0; a < d; ++a) {
        float t1 = fabsf(q[a] - lo[a]);
        float t2 = fabsf(q[a] - hi[a]);
        float t = t1 > t2 ? t1 : t2;
        float tt = t * t;
        s = s + tt;
    }
    return s;
}

/* (d2, index) keys, compared lexicographically. */
typedef struct {
    float d2;
    int32_t idx;
} key_t;

static int key_less(key_t a, key_t b)
{
    return a.d2 < b.d2 || (a.d2 == b.d2 && a.idx < b.idx);
}

static int key_cmp(const void *pa, const void *pb)
{
    key_t a = *(const key_t *)pa, b = *(const key_t *)pb;
    if (key_less(a, b)) return -1;
    if (key_less(b, a)) return 1;
    return 0;
}

static int idx_cmp(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    return (a > b) - (a < b);
}

static void write_knn_row(const key_t *sorted, int k, int32_t *oi, float *od)
{
    for (int j = 0; j < k; ++j) {
        if (sorted[j].idx == INT32_MAX) {
            oi[j] = -1;
            od[j] = INFINITY;
        } else {
            oi[j] = sorted[j].idx;
            od[j] = sorted[j].d2;
        }
    }
}

float orc_sq_dist(const float *p, const float *q, int d) { return sq_dist(p, q, d); }

/* ------------------------------------------------------------------------ */
/* Brute force: the plain definitions.                                      */
/* ------------------------------------------------------------------------ */

/* k smallest (d2, idx) keys over all n points, ascending; on the torus of
 * periods L when L is not NULL. */
static int knn_brute(const float *pts, int64_t n, int d, const float *q, int64_t nq,
                     int k, const float *L, int32_t *out_idx, float *out_d2)
{
    if (!pts || !q || !out_idx || !out_d2 || n < 0 || nq < 0 || k < 1 || d < 1)
        return ORC_EINVAL;
    if (L && (!inside_period(pts, n, d, L) || !inside_period(q, nq, d, L)))
        return ORC_EINVAL;
    key_t *best = (key_t *)malloc(sizeof(key_t) * (size_t)k);
    if (!best) return ORC_ENOMEM;
    for (int64_t t = 0; t < nq; ++t) {
        const float *qt = q + t * d;
        for (int j = 0; j < k; ++j) {
            best[j].d2 = INFINITY;
            best[j].idx = INT32_MAX;
        }
        for (int64_t i = 0; i < n; ++i) {
            key_t c = {metric_sq_dist(pts + i * d, qt, d, L), (int32_t)i};
            if (!key_less(c, best[k - 1])) continue;
            int j = k - 1;
            while (j > 0 && key_less(c, best[j - 1])) {
                best[j] = best[j - 1];
                --j;
            }
            best[j] = c;
        }
        write_knn_row(best, k, out_idx + t * k, out_d2 + t * k);
    }
    free(best);
    return ORC_OK;
}

int orc_knn_brute(const float *pts, int64_t n, int d, const float *q, int64_t nq,
                  int k, int32_t *out_idx, float *out_d2)
{
    return knn_brute(pts, n, d, q, nq, k, NULL, out_idx, out_d2);
}

int orc_knn_brute_torus(const float *pts, int64_t n, int d, const float *q, int64_t nq,
                        int k, const float *L, int32_t *out_idx, float *out_d2)
{
    if (!L) return ORC_EINVAL;
    return knn_brute(pts, n, d, q, nq, k, L, out_idx, out_d2);
}

/* Number of points with d2 <= fl(r*r), and optionally their indices
 * (ascending); on the torus of periods L when L is not NULL. */
static int range_brute(const float *pts, int64_t n, int d, const float *q, int64_t nq,
                       float r, const float *L, int64_t *out_count, int64_t *offsets,
                       int32_t *out_idx)
{
    if (!pts || !q || !out_count || n < 0 || nq < 0 || d < 1 || !(r >= 0.0f))
        return ORC_EINVAL;
    if (L && (!inside_period(pts, n, d, L) || !inside_period(q, nq, d, L)))
        return ORC_EINVAL;
    float r2 = r * r;
    int64_t pos = 0;
    for (int64_t t = 0; t < nq; ++t) {
        const float *qt = q + t * d;
        int64_t c = 0;
        if (offsets) offsets[t] = pos;
        for (int64_t i = 0; i < n; ++i) {
            if (metric_sq_dist(pts + i * d, qt, d, L) <= r2) {
                if (out_idx) out_idx[pos] = (int32_t)i;
                ++pos;
                ++c;
            }
        }
        out_count[t] = c;
    }
    if (offsets) offsets[nq] = pos;
    return ORC_OK;
}

int orc_range_brute(const float *pts, int64_t n, int d, const float *q, int64_t nq,
                    float r, int64_t *out_count, int64_t *offsets, int32_t *out_idx)
{
    return range_brute(pts, n, d, q, nq, r, NULL, out_count, offsets, out_idx);
}

int orc_range_brute_torus(const float *pts, int64_t n, int d, const float *q, int64_t nq,
                          float r, const float *L, int64_t *out_count, int64_t *offsets,
                          int32_t *out_idx)
{
    if (!L) return ORC_EINVAL;
    return range_brute(pts, n, d, q, nq, r, L, out_count, offsets, out_idx);
}

/* ------------------------------------------------------------------------ */
/* Float64 coordinates (Sec. 2.4, double-precision real kind): brute force.  */
/* ------------------------------------------------------------------------ */

static double sq_dist64(const double *p, const double *q, int d)
{
    double s = 0.0;
    for (int a = 0; a < d; ++a) {
        double t = p[a] - q[a];
        s += t * t;
    }
    return s;
}

typedef struct {
    double d2;
    int32_t idx;
} key64_t;

static int key64_less(key64_t a, key64_t b)
{
    return a.d2 < b.d2 || (a.d2 == b.d2 && a.idx < b.idx);
}

/* The k smallest (d2, idx) keys over all n points, ascending; rows padded
 * with (-1, +inf) when k > n. */
int orc_knn_brute_f64(const double *pts, int64_t n, int d, const double *q, int64_t nq, int k,
                      int32_t *out_idx, double *out_d2)
{
    if (!pts || !q || !out_idx || !out_d2 || n < 0 || nq < 0 || k < 1 || d < 1)
        return ORC_EINVAL;
    key64_t *best = (key64_t *)malloc(sizeof(key64_t) * (size_t)k);
    if (!best) return ORC_ENOMEM;
    for (int64_t t = 0; t < nq; ++t) {
        const double *qt = q + t * d;
        for (int j = 0; j < k; ++j) {
            best[j].d2 = INFINITY;
            best[j].idx = INT32_MAX;
        }
        for (int64_t i = 0; i < n; ++i) {
            key64_t c = {sq_dist64(pts + i * d, qt, d), (int32_t)i};
            if (!key64_less(c, best[k - 1])) continue;
            int j = k - 1;
            while (j > 0 && key64_less(c, best[j - 1])) {
                best[j] = best[j - 1];
                --j;
            }
            best[j] = c;
        }
        for (int j = 0; j < k; ++j) {
            const int pad = best[j].idx == INT32_MAX;
            out_idx[t * k + j] = pad ? -1 : best[j].idx;
            out_d2[t * k + j] = pad ? INFINITY : best[j].d2;
        }
    }
    free(best);
    return ORC_OK;
}

/* Number of points with d2 <= fl64(r*r), and optionally their indices
 * (ascending). */
int orc_range_brute_f64(const double *pts, int64_t n, int d, const double *q, int64_t nq,
                        double r, int64_t *out_count, int64_t *offsets, int32_t *out_idx)
{
    if (!pts || !q || !out_count || n < 0 || nq < 0 || d < 1 || !(r >= 0.0)) return ORC_EINVAL;
    const double r2 = r * r;
    int64_t pos = 0;
    for (int64_t t = 0; t < nq; ++t) {
        const double *qt = q + t * d;
        int64_t c = 0;
        if (offsets) offsets[t] = pos;
        for (int64_t i = 0; i < n; ++i) {
            if (sq_dist64(pts + i * d, qt, d) <= r2) {
                if (out_idx) out_idx[pos] = (int32_t)i;
                ++pos;
                ++c;
            }
        }
        out_count[t] = c;
    }
    if (offsets) offsets[nq] = pos;
    return ORC_OK;
}

/* Friends-of-friends by breadth-first search over all pairs; on the torus of
 * periods L when L is not NULL. */
static int fof_brute(const float *pts, int64_t n, int d, float l, const float *L,
                     int32_t *labels)
{
    if (!pts || !labels || n < 0 || d < 1 || !(l >= 0.0f)) return ORC_EINVAL;
    if (L && !inside_period(pts, n, d, L)) return ORC_EINVAL;
    float l2 = l * l;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!queue) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; ++i) labels[i] = -1;
    for (int64_t s = 0; s < n; ++s) {
        if (labels[s] >= 0) continue;
        /* every smaller index is already labelled, so s is the component minimum */
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        labels[s] = (int32_t)s;
        while (head < tail) {
            int64_t u = queue[head++];
            for (int64_t v = 0; v < n; ++v) {
                if (labels[v] >= 0 || v == u) continue;
                if (metric_sq_dist(pts + u * d, pts + v * d, d, L) <= l2) {
                    labels[v] = (int32_t)s;
                    queue[tail++] = v;
                }
            }
        }
    }
    free(queue);
    return ORC_OK;
}

int orc_fof_brute(const float *pts, int64_t n, int d, float l, int32_t *labels)
{
    return fof_brute(pts, n, d, l, NULL, labels);
}

int orc_fof_brute_torus(const float *pts, int64_t n, int d, float l, const float *L,
                        int32_t *labels)
{
    if (!L) return ORC_EINVAL;
    return fof_brute(pts, n, d, l, L, labels);
}

/* ------------------------------------------------------------------------ */
/* Sliding-midpoint k-d tree (Sec. 2.1, Algorithm 1).                        */
/* ------------------------------------------------------------------------ */

typedef struct orc_tree {
    int d;
    int leaf_size;
    int64_t n;
    float *pts;      /* tree-ordered copy of the points, [n][d] */
    int32_t *idx;    /* original index of each copied point */
    int64_t n_nodes, cap;
    int64_t *begin, *end;   /* point range [begin, end) of each node */
    int64_t *left, *right;  /* children, -1 for a leaf */
    int32_t *axis;          /* split axis, -1 for a leaf */
    float *split;           /* split value (the plane after any slide) */
    float *lo, *hi;         /* tight bounding box, [n_nodes][d] each */
    int32_t depth;          /* number of edges on the longest root-leaf path */
} orc_tree;

static int tree_grow(orc_tree *t)
{
    int64_t c = t->cap ? 2 * t->cap : 64;
    int d = t->d;
#define GROW(ptr, type, per)                                                    \
    do {                                                                        \
        type *p_ = (type *)realloc(t->ptr, sizeof(type) * (size_t)(c * (per))); \
        if (!p_) return ORC_ENOMEM;                                             \
        t->ptr = p_;                                                            \
    } while (0)
    GROW(begin, int64_t, 1);
    GROW(end, int64_t, 1);
    GROW(left, int64_t, 1);
    GROW(right, int64_t, 1);
    GROW(axis, int32_t, 1);
    GROW(split, float, 1);
    GROW(lo, float, d);
    GROW(hi, float, d);
#undef GROW
    t->cap = c;
    return ORC_OK;
}

static int64_t tree_new_node(orc_tree *t, int64_t b, int64_t e)
{
    if (t->n_nodes == t->cap && tree_grow(t) != ORC_OK) return -1;
    int64_t id = t->n_nodes++;
    int d = t->d;
    t->begin[id] = b;
    t->end[id] = e;
    t->left[id] = t->right[id] = -1;
    t->axis[id] = -1;
    t->split[id] = 0.0f;
    float *lo = t->lo + id * d, *hi = t->hi + id * d;
    for (int a = 0; a < d; ++a) {
        lo[a] = INFINITY;
        hi[a] = -INFINITY;
    }
    for (int64_t i = b; i < e; ++i) {
        const float *p = t->pts + i * d;
        for (int a = 0; a < d; ++a) {
            if (p[a] < lo[a]) lo[a] = p[a];
            if (p[a] > hi[a]) hi[a] = p[a];
        }
    }
    return id;
}

void orc_tree_free(orc_tree *t)
{
    if (!t) return;
    free(t->pts);
    free(t->idx);
    free(t->begin);
    free(t->end);
    free(t->left);
    free(t->right);
    free(t->axis);
    free(t->split);
    free(t->lo);
    free(t->hi);
    free(t);
}

/* Moves the points of [b, e) whose flag is set to the front, keeping order. */
static int stable_split(orc_tree *t, int64_t b, int64_t e, const unsigned char *go_left,
                        float *tmp_p, int32_t *tmp_i)
{
    int d = t->d;
    int64_t w = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int64_t i = b; i < e; ++i)
            if ((go_left[i - b] != 0) == (pass == 0)) {
                memcpy(tmp_p + w * d, t->pts + i * d, sizeof(float) * (size_t)d);
                tmp_i[w] = t->idx[i];
                ++w;
            }
    memcpy(t->pts + b * d, tmp_p, sizeof(float) * (size_t)((e - b) * d));
    memcpy(t->idx + b, tmp_i, sizeof(int32_t) * (size_t)(e - b));
    return ORC_OK;
}

int orc_tree_build(const float *pts, int64_t n, int d, int leaf_size, orc_tree **out)
{
    if (!pts || !out || n < 0 || d < 1 || leaf_size < 1) return ORC_EINVAL;
    for (int64_t i = 0; i < n * d; ++i)
        if (!isfinite(pts[i])) return ORC_EINVAL;
    orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
    if (!t) return ORC_ENOMEM;
    t->d = d;
    t->leaf_size = leaf_size;
    t->n = n;
    size_t nn = (size_t)(n > 0 ? n : 1);
    t->pts = (float *)malloc(sizeof(float) * nn * (size_t)d);
    t->idx = (int32_t *)malloc(sizeof(int32_t) * nn);
    float *tmp_p = (float *)malloc(sizeof(float) * nn * (size_t)d);
    int32_t *tmp_i = (int32_t *)malloc(sizeof(int32_t) * nn);
    unsigned char *flag = (unsigned char *)malloc(nn);
    int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * 2 * nn + 16);
    int32_t *level = (int32_t *)malloc(sizeof(int32_t) * 2 * nn + 16);
    if (!t->pts || !t->idx || !tmp_p || !tmp_i || !flag || !stack || !level) goto nomem;
    memcpy(t->pts, pts, sizeof(float) * (size_t)(n * d));
    for (int64_t i = 0; i < n; ++i) t->idx[i] = (int32_t)i;

    if (tree_new_node(t, 0, n) < 0) goto nomem;
    int64_t sp = 0;
    stack[sp] = 0;
    level[sp] = 0;
    ++sp;
    while (sp > 0) {
        --sp;
        int64_t id = stack[sp];
        int32_t lev = level[sp];
        if (lev > t->depth) t->depth = lev;
        int64_t b = t->begin[id], e = t->end[id], m = e - b;
        if (m <= leaf_size) continue;                      /* leaf (Alg. 1) */
        const float *lo = t->lo + id * d, *hi = t->hi + id * d;
        int ax = 0;
        float ext = hi[0] - lo[0];
        for (int a = 1; a < d; ++a)
            if (hi[a] - lo[a] > ext) {
                ext = hi[a] - lo[a];
                ax = a;
            }
        if (!(ext > 0.0f)) continue;                       /* all points coincide */
        float split = lo[ax] + (hi[ax] - lo[ax]) * 0.5f;   /* box midpoint */
        int64_t n_left = 0;
        for (int64_t i = b; i < e; ++i) {
            flag[i - b] = t->pts[i * d + ax] < split;
            n_left += flag[i - b];
        }
        if (n_left == 0 || n_left == m) {
            /* slide: the extreme point nearest the plane moves to the empty side */
            int want_min = (n_left == 0);
            int64_t pick = -1;
            for (int64_t i = b; i < e; ++i) {
                float v = t->pts[i * d + ax];
                if (pick < 0) { pick = i; continue; }
                float pv = t->pts[pick * d + ax];
                int better = want_min ? (v < pv) : (v > pv);
                if (better || (v == pv && t->idx[i] < t->idx[pick])) pick = i;
            }
            split = t->pts[pick * d + ax];
            for (int64_t i = b; i < e; ++i) flag[i - b] = want_min ? (i == pick) : (i != pick);
            n_left = want_min ? 1 : m - 1;
        }
        stable_split(t, b, e, flag, tmp_p, tmp_i);
        int64_t l = tree_new_node(t, b, b + n_left);
        if (l < 0) goto nomem;
        int64_t r = tree_new_node(t, b + n_left, e);
        if (r < 0) goto nomem;
        t->left[id] = l;
        t->right[id] = r;
        t->axis[id] = ax;
        t->split[id] = split;
        stack[sp] = r;
        level[sp] = lev + 1;
        ++sp;
        stack[sp] = l;
        level[sp] = lev + 1;
        ++sp;
    }
    free(tmp_p);
    free(tmp_i);
    free(flag);
    free(stack);
    free(level);
    *out = t;
    return ORC_OK;
nomem:
    free(tmp_p);
    free(tmp_i);
    free(flag);
    free(stack);
    free(level);
    orc_tree_free(t);
    return ORC_ENOMEM;
}

/* Read-only views used by the invariant tests. */
int64_t orc_tree_n_nodes(const orc_tree *t) { return t->n_nodes; }
int32_t orc_tree_depth(const orc_tree *t) { return t->depth; }

int orc_tree_export(const orc_tree *t, float *pts, int32_t *idx, int64_t *begin, int64_t *end,
                    int64_t *left, int64_t *right, int32_t *axis, float *split, float *lo,
                    float *hi)
{
    int64_t m = t->n_nodes;
    int d = t->d;
    if (pts) memcpy(pts, t->pts, sizeof(float) * (size_t)(t->n * d));
    if (idx) memcpy(idx, t->idx, sizeof(int32_t) * (size_t)t->n);
    if (begin) memcpy(begin, t->begin, sizeof(int64_t) * (size_t)m);
    if (end) memcpy(end, t->end, sizeof(int64_t) * (size_t)m);
    if (left) memcpy(left, t->left, sizeof(int64_t) * (size_t)m);
    if (right) memcpy(right, t->right, sizeof(int64_t) * (size_t)m);
    if (axis) memcpy(axis, t->axis, sizeof(int32_t) * (size_t)m);
    if (split) memcpy(split, t->split, sizeof(float) * (size_t)m);
    if (lo) memcpy(lo, t->lo, sizeof(float) * (size_t)(m * d));
    if (hi) memcpy(hi, t->hi, sizeof(float) * (size_t)(m * d));
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* kNN query (Algorithm 2): best-first over a node min-heap, candidates in a */
/* max-heap, results sorted at the end.                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    float dist;
    int64_t node;
} qitem_t;

static void qheap_push(qitem_t *h, int64_t *nh, qitem_t it)
{
    int64_t i = (*nh)++;
    h[i] = it;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].dist <= h[i].dist) break;
        qitem_t s = h[p];
        h[p] = h[i];
        h[i] = s;
        i = p;
    }
}

static qitem_t qheap_pop(qitem_t *h, int64_t *nh)
{
    qitem_t top = h[0];
    h[0] = h[--(*nh)];
    int64_t i = 0, m = *nh;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < m && h[l].dist < h[s].dist) s = l;
        if (r < m && h[r].dist < h[s].dist) s = r;
        if (s == i) break;
        qitem_t x = h[s];
        h[s] = h[i];
        h[i] = x;
        i = s;
    }
    return top;
}

/* replace the largest key of a max-heap and restore the heap property */
static void kheap_replace_top(key_t *h, int k, key_t c)
{
    h[0] = c;
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, s = i;
        if (l < k && key_less(h[s], h[l])) s = l;
        if (r < k && key_less(h[s], h[r])) s = r;
        if (s == i) break;
        key_t x = h[s];
        h[s] = h[i];
        h[i] = x;
        i = s;
    }
}

int orc_knn_tree(const orc_tree *t, const float *q, int64_t nq, int k, int32_t *out_idx,
                 float *out_d2)
{
    if (!t || !q || !out_idx || !out_d2 || nq < 0 || k < 1) return ORC_EINVAL;
    int d = t->d;
    key_t *K = (key_t *)malloc(sizeof(key_t) * (size_t)k);
    qitem_t *Q = (qitem_t *)malloc(sizeof(qitem_t) * (size_t)(t->n_nodes + 1));
    if (!K || !Q) {
        free(K);
        free(Q);
        return ORC_ENOMEM;
    }
    for (int64_t s = 0; s < nq; ++s) {
        const float *p = q + s * d;
        for (int j = 0; j < k; ++j) {
            K[j].d2 = INFINITY;
            K[j].idx = INT32_MAX;
        }
        int64_t nh = 0;
        qitem_t root = {box_min_dist(p, t->lo, t->hi, d), 0};
        qheap_push(Q, &nh, root);
        while (nh > 0) {
            qitem_t it = qheap_pop(Q, &nh);
            if (it.dist > K[0].d2) continue;
            int64_t id = it.node;
            if (t->left[id] < 0) {
                for (int64_t i = t->begin[id]; i < t->end[id]; ++i) {
                    key_t c = {sq_dist(t->pts + i * d, p, d), t->idx[i]};
                    if (key_less(c, K[0])) kheap_replace_top(K, k, c);
                }
            } else {
                int64_t ch[2] = {t->left[id], t->right[id]};
                for (int c = 0; c < 2; ++c) {
                    float md = box_min_dist(p, t->lo + ch[c] * d, t->hi + ch[c] * d, d);
                    if (md <= K[0].d2) {
                        qitem_t ci = {md, ch[c]};
                        qheap_push(Q, &nh, ci);
                    }
                }
            }
        }
        qsort(K, (size_t)k, sizeof(key_t), key_cmp);
        write_knn_row(K, k, out_idx + s * k, out_d2 + s * k);
    }
    free(K);
    free(Q);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Ball query (Algorithm 3).                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t *buf;
    int64_t n, cap;
} ivec_t;

static int ivec_push(ivec_t *v, int32_t x)
{
    if (v->n == v->cap) {
        int64_t c = v->cap ? 2 * v->cap : 256;
        int32_t *b = (int32_t *)realloc(v->buf, sizeof(int32_t) * (size_t)c);
        if (!b) return ORC_ENOMEM;
        v->buf = b;
        v->cap = c;
    }
    v->buf[v->n++] = x;
    return ORC_OK;
}

/* Collects the original indices of all points with d2 <= r2 (unsorted). */
static int ball_collect(const orc_tree *t, int64_t id, const float *p, float r2, ivec_t *out)
{
    int d = t->d;
    const float *lo = t->lo + id * d, *hi = t->hi + id * d;
    if (box_min_dist(p, lo, hi, d) > r2) return ORC_OK;
    if (box_max_dist(p, lo, hi, d) <= r2) {
        for (int64_t i = t->begin[id]; i < t->end[id]; ++i)
            if (ivec_push(out, t->idx[i]) != ORC_OK) return ORC_ENOMEM;
        return ORC_OK;
    }
    if (t->left[id] < 0) {
        for (int64_t i = t->begin[id]; i < t->end[id]; ++i)
            if (sq_dist(t->pts + i * d, p, d) <= r2)
                if (ivec_push(out, t->idx[i]) != ORC_OK) return ORC_ENOMEM;
        return ORC_OK;
    }
    if (ball_collect(t, t->left[id], p, r2, out) != ORC_OK) return ORC_ENOMEM;
    return ball_collect(t, t->right[id], p, r2, out);
}

/*
 * Ball query for nq points.  out_count[s] is the number of points within r.
 * When out_idx is given, offsets[nq+1] must be given too and the lists are
 * written in ascending index order; capacity bounds out_idx.
 */
int orc_range_tree(const orc_tree *t, const float *q, int64_t nq, float r, int64_t *out_count,
                   int64_t *offsets, int32_t *out_idx, int64_t capacity)
{
    if (!t || !q || !out_count || nq < 0 || !(r >= 0.0f)) return ORC_EINVAL;
    float r2 = r * r;
    ivec_t v = {0, 0, 0};
    int64_t pos = 0;
    for (int64_t s = 0; s < nq; ++s) {
        v.n = 0;
        if (t->n > 0 && ball_collect(t, 0, q + s * t->d, r2, &v) != ORC_OK) {
            free(v.buf);
            return ORC_ENOMEM;
        }
        out_count[s] = v.n;
        if (offsets) offsets[s] = pos;
        if (out_idx) {
            if (pos + v.n > capacity) {
                free(v.buf);
                return ORC_EINVAL;
            }
            if (v.n > 0) { /* an empty ball may have no buffer yet */
                qsort(v.buf, (size_t)v.n, sizeof(int32_t), idx_cmp);
                memcpy(out_idx + pos, v.buf, sizeof(int32_t) * (size_t)v.n);
            }
        }
        pos += v.n;
    }
    if (offsets) offsets[nq] = pos;
    free(v.buf);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Friends-of-friends (Sec. 4.1): union-find over ball queries.             */
/* ------------------------------------------------------------------------ */

static int32_t uf_find(int32_t *parent, int32_t x)
{
    while (parent[x] != x) x = parent[x];
    return x;
}

int orc_fof_tree(const orc_tree *t, const float *pts, float l, int32_t *labels)
{
    if (!t || !pts || !labels || !(l >= 0.0f)) return ORC_EINVAL;
    int64_t n = t->n;
    int d = t->d;
    float l2 = l * l;
    for (int64_t i = 0; i < n; ++i) labels[i] = (int32_t)i;
    ivec_t v = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        v.n = 0;
        if (ball_collect(t, 0, pts + i * d, l2, &v) != ORC_OK) {
            free(v.buf);
            return ORC_ENOMEM;
        }
        for (int64_t j = 0; j < v.n; ++j) {
            /* union: the larger root is hung under the smaller one, so every
               root is the smallest index of its set */
            int32_t a = uf_find(labels, (int32_t)i), b = uf_find(labels, v.buf[j]);
            if (a < b) labels[b] = a;
            else if (b < a) labels[a] = b;
        }
    }
    for (int64_t i = 0; i < n; ++i) labels[i] = uf_find(labels, (int32_t)i);
    free(v.buf);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Adaptive SPH particle-to-mesh deposit (Sec. 4.2), float64.               */
/* ------------------------------------------------------------------------ */

/* M4 cubic spline profile on q in [0, 2] and its derivative. */
double orc_m4_w(double q)
{
    if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    if (q < 2.0) {
        double u = 2.0 - q;
        return 0.25 * u * u * u;
    }
    return 0.0;
}

double orc_m4_dw(double q)
{
    if (q < 1.0) return -3.0 * q + 2.25 * q * q;
    if (q < 2.0) {
        double u = 2.0 - q;
        return -0.75 * u * u;
    }
    return 0.0;
}

typedef struct {
    double lo[3];
    double cell;
    int32_t n[3];
    int32_t periodic; /* 1: the mesh box is a 3-torus of periods n[a] * cell */
} orc_grid;

static int grid_ok(const orc_grid *g)
{
    return g && g->cell > 0.0 && g->n[0] > 0 && g->n[1] > 0 && g->n[2] > 0;
}

static int inside_grid(const orc_grid *g, const double *x)
{
    for (int a = 0; a < 3; ++a) {
        double top = g->lo[a] + g->cell * g->n[a];
        if (!(x[a] >= g->lo[a] && x[a] < top)) return 0;
    }
    return 1;
}

/* Cell index range [c0, c1] per axis that can hold centres within H of x.
   brute != 0 returns the whole grid instead.  On a periodic mesh the range
   is not clipped: indices below 0 or above n - 1 stand for the cells one
   period away (an unwrapped index; see wrap_cell). */
static void cell_box(const orc_grid *g, const double *x, double H, int brute, int32_t *c0,
                     int32_t *c1)
{
    for (int a = 0; a < 3; ++a) {
        if (brute) {
            c0[a] = 0;
            c1[a] = g->n[a] - 1;
            continue;
        }
        double f0 = (x[a] - H - g->lo[a]) / g->cell - 0.5;
        double f1 = (x[a] + H - g->lo[a]) / g->cell - 0.5;
        int64_t i0 = (int64_t)floor(f0) - 1, i1 = (int64_t)ceil(f1) + 1;
        if (!g->periodic) {
            if (i0 < 0) i0 = 0;
            if (i1 > g->n[a] - 1) i1 = g->n[a] - 1;
        } else {
            /* H < period / 2: keep at most one copy of each cell, the n
               cells whose centres lie within half a period of x (every
               centre within H is among them, at its nearest copy) */
            if (i1 - i0 + 1 > g->n[a]) {
                i0 = (int64_t)ceil((x[a] - g->lo[a]) / g->cell - 0.5 - 0.5 * g->n[a]);
                i1 = i0 + g->n[a] - 1;
            }
        }
        c0[a] = (int32_t)i0;
        c1[a] = (int32_t)i1;
    }
}

/* Centre of (unwrapped) cell c along axis a. */
static double cell_centre(const orc_grid *g, int a, int32_t c)
{
    return g->lo[a] + ((double)c + 0.5) * g->cell;
}

/* Storage index along axis a of unwrapped cell c (c itself on an open mesh). */
static int32_t wrap_cell(const orc_grid *g, int a, int32_t c)
{
    if (!g->periodic) return c;
    int32_t w = c % g->n[a];
    return w < 0 ? w + g->n[a] : w;
}

/* Per-axis offset from the centre of storage cell c to x on the mesh: on a
   periodic mesh the shorter way round (used by the whole-mesh form only). */
static double axis_offset(const orc_grid *g, int a, const double *x, int32_t c)
{
    double v = x[a] - cell_centre(g, a, c);
    if (g->periodic) {
        double L = g->cell * g->n[a];
        double u = fabs(v);
        if (L - u < u) v = v > 0.0 ? v - L : v + L;
    }
    return v;
}

/* The smoothing length must stay below half of every period on a periodic
   mesh: beyond, a particle's support would reach a cell from both sides. */
static int support_ok(const orc_grid *g, double H)
{
    if (!g->periodic) return 1;
    for (int a = 0; a < 3; ++a)
        if (!(2.0 * H < g->cell * g->n[a])) return 0;
    return 1;
}

/*
 * rho[c] = sum_i m_i w(2 |x_i - x_c| / H_i) / S_i,  S_i = sum over in-grid c.
 * x is [n][3], rho has n[0]*n[1]*n[2] entries and is overwritten.
 */
static int p2m_forward(const double *x, const double *m, const double *h, int64_t n,
                       const orc_grid *g, double *rho, int brute)
{
    if (!x || !m || !h || !rho || n < 0 || !grid_ok(g)) return ORC_EINVAL;
    int64_t ncell = (int64_t)g->n[0] * g->n[1] * g->n[2];
    for (int64_t c = 0; c < ncell; ++c) rho[c] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *xi = x + 3 * i;
        if (!inside_grid(g, xi) || !(h[i] >= 0.0)) return ORC_EINVAL;
        double H = h[i] > g->cell ? h[i] : g->cell;
        if (!support_ok(g, H)) return ORC_EINVAL;
        int32_t c0[3], c1[3];
        cell_box(g, xi, H, brute, c0, c1);
        /* Two passes over the same cells: the normalisation S, then the
           deposit.  The support-box form measures from the unwrapped cell
           centre (the nearest copy of the cell, as H < period / 2); the
           whole-mesh form (brute) takes the shorter way round per axis. */
        double S = 0.0;
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1 && !(S > 0.0)) return ORC_EINVAL;
            for (int32_t a = c0[0]; a <= c1[0]; ++a)
                for (int32_t b = c0[1]; b <= c1[1]; ++b)
                    for (int32_t c = c0[2]; c <= c1[2]; ++c) {
                        double dx, dy, dz;
                        if (brute) {
                            dx = axis_offset(g, 0, xi, a);
                            dy = axis_offset(g, 1, xi, b);
                            dz = axis_offset(g, 2, xi, c);
                        } else {
                            dx = xi[0] - cell_centre(g, 0, a);
                            dy = xi[1] - cell_centre(g, 1, b);
                            dz = xi[2] - cell_centre(g, 2, c);
                        }
                        double r = sqrt(dx * dx + dy * dy + dz * dz);
                        double w = orc_m4_w(2.0 * r / H);
                        if (pass == 0) {
                            S += w;
                        } else if (w != 0.0) {
                            int64_t at = ((int64_t)wrap_cell(g, 0, a) * g->n[1] +
                                          wrap_cell(g, 1, b)) * g->n[2] + wrap_cell(g, 2, c);
                            rho[at] += m[i] * w / S;
                        }
                    }
        }
    }
    return ORC_OK;
}

int orc_p2m(const double *x, const double *m, const double *h, int64_t n, const orc_grid *g,
            double *rho)
{
    return p2m_forward(x, m, h, n, g, rho, 0);
}

int orc_p2m_brute(const double *x, const double *m, const double *h, int64_t n,
                  const orc_grid *g, double *rho)
{
    return p2m_forward(x, m, h, n, g, rho, 1);
}

/* Per-axis weights of the fixed-cloud schemes (1 NGP, 2 CIC, 3 TSC) for a
   particle at s (cells, from the first centre): w[0 .. order-1] on cells
   base, base + 1, ...  Returns the number of cells. */
static int cloud_axis(int scheme, double s, int64_t *base, double *w)
{
    if (scheme == 1) {
        /* the cell holding the particle, floor((x - lo) / cell); the caller
           passes that index, decided in float32 (see cloud_forward) */
        *base = (int64_t)floor(s + 0.5);
        w[0] = 1.0;
        return 1;
    }
    if (scheme == 2) {
        double i0 = floor(s), f = s - i0;
        *base = (int64_t)i0;
        w[0] = 1.0 - f;
        w[1] = f;
        return 2;
    }
    double c = floor(s + 0.5), u = s - c;
    *base = (int64_t)c - 1;
    w[0] = 0.5 * (0.5 - u) * (0.5 - u);
    w[1] = 0.75 - u * u;
    w[2] = 0.5 * (0.5 + u) * (0.5 + u);
    return 3;
}

/* The same weights from the shape function of the scheme, W(v) for a cell
   whose centre is v cells from the particle (v = i - s):
   NGP 1 for -1/2 < v <= 1/2 (a particle on a cell face belongs to the cell
   above it); CIC max(0, 1 - |v|); TSC 3/4 - v^2 for |v| <= 1/2,
   (3/2 - |v|)^2 / 2 for 1/2 < |v| < 3/2, else 0. */
double orc_cloud_shape(int scheme, double v)
{
    double a = fabs(v);
    if (scheme == 1) return (v > -0.5 && v <= 0.5) ? 1.0 : 0.0;
    if (scheme == 2) return a < 1.0 ? 1.0 - a : 0.0;
    if (a <= 0.5) return 0.75 - v * v;
    if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
    return 0.0;
}

/*
 * Fixed-cloud deposit rho[c] = sum_i m_i W_ic / S_i (S_i = the particle's
 * in-mesh weight; 1 unless cells fall outside an open mesh).  brute != 0
 * visits every cell of the mesh with the shape function (offsets the
 * shorter way round on a periodic mesh) instead of the per-axis stencil.
 */
static int cloud_forward(const double *x, const double *m, int64_t n, const orc_grid *g,
                         int scheme, double *rho, int brute)
{
    if (!x || !m || !rho || n < 0 || !grid_ok(g) || scheme < 1 || scheme > 3) return ORC_EINVAL;
    if (g->periodic)
        for (int a = 0; a < 3; ++a)
            if (g->n[a] < scheme) return ORC_EINVAL;
    int64_t ncell = (int64_t)g->n[0] * g->n[1] * g->n[2];
    for (int64_t c = 0; c < ncell; ++c) rho[c] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *xi = x + 3 * i;
        if (!inside_grid(g, xi)) return ORC_EINVAL;
        int64_t base[3];
        double w[3][3];
        int cnt[3];
        for (int a = 0; a < 3; ++a) {
            if (brute) {
                base[a] = 0;
                cnt[a] = g->n[a];
            } else if (scheme == 1) {
                /* NGP decides an integer from the position: the cell index
                   floor((x - lo) / cell) is taken in float32, as the GPU
                   takes it (the other schemes' weights are continuous) */
                float t = ((float)xi[a] - (float)g->lo[a]) / (float)g->cell;
                cnt[a] = cloud_axis(scheme, (double)floorf(t), &base[a], w[a]);
            } else {
                cnt[a] = cloud_axis(scheme, (xi[a] - g->lo[a]) / g->cell - 0.5, &base[a], w[a]);
            }
        }
        double S = 0.0;
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1 && !(S > 0.0)) return ORC_EINVAL;
            for (int p = 0; p < cnt[0]; ++p)
                for (int q = 0; q < cnt[1]; ++q)
                    for (int r = 0; r < cnt[2]; ++r) {
                        int64_t idx[3] = {base[0] + p, base[1] + q, base[2] + r};
                        double wt = 1.0;
                        int in = 1;
                        for (int a = 0; a < 3; ++a) {
                            int k = a == 0 ? p : a == 1 ? q : r;
                            if (brute) {
                                double v = (double)idx[a] - ((xi[a] - g->lo[a]) / g->cell - 0.5);
                                if (g->periodic) {
                                    double L = g->n[a];
                                    double u = fabs(v);
                                    if (L - u < u) v = v > 0.0 ? v - L : v + L;
                                }
                                wt *= orc_cloud_shape(scheme, v);
                            } else {
                                wt *= w[a][k];
                                if (g->periodic) {
                                    idx[a] %= g->n[a];
                                    if (idx[a] < 0) idx[a] += g->n[a];
                                } else if (idx[a] < 0 || idx[a] >= g->n[a]) {
                                    in = 0;
                                }
                            }
                        }
                        if (!in || wt == 0.0) continue;
                        if (pass == 0) {
                            S += wt;
                        } else {
                            int64_t at = (idx[0] * g->n[1] + idx[1]) * g->n[2] + idx[2];
                            rho[at] += m[i] * wt / S;
                        }
                    }
        }
    }
    return ORC_OK;
}

int orc_p2m_cloud(const double *x, const double *m, int64_t n, const orc_grid *g, int scheme,
                  double *rho, int brute)
{
    return cloud_forward(x, m, n, g, scheme, rho, brute);
}

/*
 * Adjoint of orc_p2m for L = sum_c g_c rho_c with h held fixed:
 *   dL/dm_i = A_i / S_i,
 *   dL/dx_i = (m_i / S_i) (C_i - (A_i / S_i) B_i),
 * with S = sum w, A = sum g w, B = sum grad w, C = sum g grad w over the
 * particle's in-grid cells and grad w = w'(q) (2 / H) (x_i - x_c) / r.
 */
int orc_p2m_backward(const double *x, const double *m, const double *h, int64_t n,
                     const orc_grid *g, const double *gg, double *dm, double *dx)
{
    if (!x || !m || !h || !gg || n < 0 || !grid_ok(g)) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        const double *xi = x + 3 * i;
        if (!inside_grid(g, xi) || !(h[i] >= 0.0)) return ORC_EINVAL;
        double H = h[i] > g->cell ? h[i] : g->cell;
        if (!support_ok(g, H)) return ORC_EINVAL;
        int32_t c0[3], c1[3];
        cell_box(g, xi, H, 0, c0, c1);
        double S = 0.0, A = 0.0, B[3] = {0, 0, 0}, C[3] = {0, 0, 0};
        for (int32_t a = c0[0]; a <= c1[0]; ++a)
            for (int32_t b = c0[1]; b <= c1[1]; ++b)
                for (int32_t c = c0[2]; c <= c1[2]; ++c) {
                    double v[3] = {xi[0] - cell_centre(g, 0, a), xi[1] - cell_centre(g, 1, b),
                                   xi[2] - cell_centre(g, 2, c)};
                    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                    double q = 2.0 * r / H;
                    double w = orc_m4_w(q);
                    double gc = gg[((int64_t)wrap_cell(g, 0, a) * g->n[1] + wrap_cell(g, 1, b)) *
                                       g->n[2] + wrap_cell(g, 2, c)];
                    S += w;
                    A += gc * w;
                    if (r > 0.0) {
                        double f = orc_m4_dw(q) * (2.0 / H) / r;
                        for (int e = 0; e < 3; ++e) {
                            B[e] += f * v[e];
                            C[e] += gc * f * v[e];
                        }
                    }
                }
        if (!(S > 0.0)) return ORC_EINVAL;
        double G = A / S;
        if (dm) dm[i] = G;
        if (dx)
            for (int e = 0; e < 3; ++e) dx[3 * i + e] = (m[i] / S) * (C[e] - G * B[e]);
    }
    return ORC_OK;
}
