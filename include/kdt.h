/*
 * kdt.h -- C ABI of the MI355X (gfx950) k-d tree library.
 *
 * The library builds k-d trees on the GPU and answers batched k-nearest-
 * neighbour (any k up to KDT_MAX_K_SORTED), fixed-radius (ball) and
 * axis-aligned box queries over them, in open space or on the D-torus of
 * periodic boundaries, then uses those queries for friends-of-friends
 * grouping and for an adaptive SPH particle-to-mesh deposit with its adjoint.  The method is the one of "cosmokdtree: a flexible
 * OpenMP-parallelized k-d tree for computational astrophysics applications"
 * (tree construction Sec. 2.1 and Algorithm 1, queries Sec. 2.3 and
 * Algorithms 2-3, applications Sec. 4.1-4.2); the GPU design differs from the
 * paper's CPU one (balanced median splits, level-synchronous build).
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers on the current HIP device; the
 *     caller owns them.  Pointers named h_* or documented as "host" are host
 *     memory.  Points are float32 rows, row-major [n][d].
 *   - Every call is asynchronous on `stream` unless it documents a wait.
 *     A call never frees or reallocates caller memory.
 *   - Nothing throws.  Each call returns a kdt_status; on anything but KDT_OK
 *     the calling thread's kdt_last_error() describes the failure and no
 *     output may be relied on.
 *   - Indices in results are int32 and refer to the caller's input order.
 *   - Distances are squared Euclidean distances (Eq. 1 with p = 2) in float32,
 *     summed over axes 0..d-1 left to right with every operation rounded on
 *     its own (no fused multiply-add); on the torus each axis takes the
 *     shorter way round first (kdt_query_opts.period).  Equal distances are ordered by the
 *     lower index.  These rules make kNN, ball and grouping results exact and
 *     reproducible, independent of the tree's shape.
 */
#ifndef KDT_H
#define KDT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KDT_OK = 0,
    KDT_EINVAL = 1,       /* bad argument, or non-finite input coordinates */
    KDT_EUNSUPPORTED = 2, /* dimension or k outside what the kernels are built for */
    KDT_ENOMEM = 3,       /* a device or host allocation failed */
    KDT_ECAPACITY = 4,    /* an output buffer is too small; see `required` */
    KDT_EDEVICE = 5       /* a HIP runtime call failed */
} kdt_status;

/* The largest k that kdt_knn keeps in registers (the batched forest's limit
   too), and the largest k it accepts: above KDT_MAX_K it switches to a
   per-query ball and sort (Sec. 3.3 measures k up to 10^4). */
#define KDT_MAX_K 64
#define KDT_MAX_K_SORTED (1 << 20)
/* d must be one of 2, 3, 4, 8, 16. */

typedef struct kdt_tree kdt_tree;             /* device-resident tree, library-owned */
typedef struct kdt_batch_plan kdt_batch_plan; /* many trees, fixed shapes, library-owned */

typedef struct {
    int32_t leaf_size;    /* N_leaf: a node with <= leaf_size points is a leaf
                             (Sec. 2.1 step 4), 2..256.  0: the autotuned
                             choice for (d, n, tune_k) from the library's
                             tuning table (kdt_tuning_get). */
    int32_t check_finite; /* 1 (default when opts is NULL): kdt_build waits for its
                             first pass and rejects NaN/Inf coordinates with
                             KDT_EINVAL.  2: deferred -- no wait; the check's
                             result stays with the tree and kdt_tree_check
                             reports it (a tree of non-finite points is
                             built but its query results are meaningless).
                             Sliding-midpoint builds wait in any case and
                             treat 2 as 1.  0: no check.  With 0 or 2 a
                             non-finite coordinate is built as 0. */
    int32_t split_rule;   /* 0 (default): balanced median splits (see kdt_build).
                             1: the paper's sliding-midpoint rule (Sec. 2.1,
                             Algorithm 1): split the longest side of the
                             node's tight box at its midpoint, sliding to the
                             nearest point when a side would be empty.  The
                             depth then depends on the data (at most 96
                             levels, KDT_EUNSUPPORTED beyond) and the build
                             waits on its stream once per level.  Such a tree
                             answers kdt_knn (k <= KDT_MAX_K, open
                             boundaries; one traversal per lane),
                             kdt_knn_noalloc, kdt_range (open boundaries;
                             one traversal per lane), kdt_fof and
                             kdt_query_order; kdt_box, kdt_fof_torus, larger
                             k and periods return KDT_EUNSUPPORTED.  Results
                             are the same as on a median tree. */
    int32_t tune_k;       /* With leaf_size 0: the k of the kNN queries the tree
                             is built for, to pick its N_leaf (0: 32). */
} kdt_build_opts;

typedef struct {
    int32_t sort_queries; /* 1: reorder external queries along the tree before the
                             traversal (more coherent waves); 0: input order.
                             Results are identical either way. */
    int32_t traversal;    /* kNN and ball counts.  0: default.  1: one
                             independent traversal per lane.  2: one traversal
                             shared by the 64 queries of a wave, leaves staged
                             in LDS (trees with leaf_size <= 64; larger leaves
                             use 1).  0 picks, for kNN, the queries per
                             traversal the tuning table gives for (d, the
                             tree's n, k) (kdt_tuning_get: 1 -> 1, 64 -> 2;
                             as measured, 1 up to d = 8 and 2 for d = 16),
                             and 2 for ball counts.  Results are identical
                             either way. */
    const int32_t *order; /* NULL, or a device permutation [nq] from
                             kdt_query_order to use instead of sorting again. */
    int32_t split_budget; /* Ball counts with traversal 2.  0: default (a wave
                             still running in the launch's tail hands the big
                             subtrees of its stack on to later launches after
                             512 node visits, then every 32).  > 0: every wave
                             hands subtrees on after this many visits, in
                             every launch.  Results are identical either way;
                             it exists for tuning and for testing the
                             hand-off.  Negative: KDT_EINVAL. */
    const float *period;  /* NULL: open boundaries.  Else a host array of d
                             periods L_a (finite, > 0): kdt_knn and kdt_range
                             measure distances on the D-torus
                             (the periodic boundary conditions of Sec. 2.1 and
                             Sec. 2.4): per axis the shorter way round,
                             min(|x - q|, L - |x - q|), squared and summed in
                             float32 like the open distance.  Every tree point
                             and query must lie in [0, L_a) (KDT_EINVAL
                             otherwise; the call waits on its stream to check).
                             kNN and lists take one traversal per lane,
                             ball counts the wave-shared one (leaf_size <=
                             64), k > KDT_MAX_K the ball-and-sort path
                             with the torus distance; traversal and
                             split_budget are ignored.  kdt_box returns
                             KDT_EUNSUPPORTED. */
    int32_t tree_rows;    /* Self queries (d_q NULL) of kdt_knn, kdt_range and
                             their _f64 and _noalloc forms.  0: row i of every
                             output belongs to input point i.  1: row t
                             belongs to the tree's t-th point in tree order
                             (input point kdt_tree_perm[t]), so the rows are
                             written in the order the traversal visits them,
                             as contiguous runs, and they line up with the
                             tree-ordered deposit (kdt_p2m_tree).  Results
                             are otherwise identical.  1 with external
                             queries, or another value: KDT_EINVAL. */
    int32_t counts_given; /* kdt_range lists (d_idx and d_offsets set), open or
                             periodic: 1 = d_count and d_offsets already hold
                             what the sizing call (d_idx NULL) of the same
                             tree, queries, radius and options wrote, so the
                             call skips the counting pass and the offset scan
                             and only fills and sorts the lists (it still
                             reads the total back).  Other values of d_count
                             and d_offsets give undefined lists.  0: count
                             again.  1 without lists, or another value:
                             KDT_EINVAL.  Ignored by the other calls. */
} kdt_query_opts;

/* Uniform mesh for the particle-to-mesh deposit: n[0]*n[1]*n[2] cells of side
   `cell`, cell (i,j,k) centred at lo + (i+1/2, j+1/2, k+1/2)*cell, stored with
   x slowest and z fastest.  periodic = 1 makes the mesh box a 3-torus of
   periods n[a]*cell (the periodic boundaries of Sec. 2.4 applied to the mesh
   of Sec. 4.2): distances to cell centres take per axis the shorter way
   round and no support is cut at a face; 0: an open mesh. */
typedef struct {
    float lo[3];
    float cell;
    int32_t n[3];
    int32_t periodic;
} kdt_grid;

/* Shape of a built tree, for diagnostics and the structural tests. */
typedef struct {
    int64_t n;          /* points */
    int32_t d;          /* dimension */
    int32_t leaf_size;  /* N_leaf used */
    int32_t levels;     /* median tree: L, splits on every root-to-leaf path
                           (2^L leaves); sliding-midpoint tree: the depth of
                           the deepest leaf */
    int32_t stride;     /* floats per point record in tree order */
    int64_t n_nodes;    /* median tree: 2^(L+1) - 1; sliding-midpoint tree: the
                           nodes it has (2 x leaves - 1) */
} kdt_tree_info;

/*
 * kdt_build -- build a k-d tree over n points (Sec. 2.1, Algorithm 1).
 *
 * d_pts  [n][d] float32, device.  Only read; it may be freed or overwritten once
 *        the work queued on `stream` by this call has run: the tree keeps its own
 *        copy of positions and indices (the tree is self-contained, Sec. 3.4).
 * n      1 <= n <= 2^31 - 1.     d in {2, 3, 4, 8, 16}.
 * opts   may be NULL (every field 0 except check_finite = 1: autotuned leaf
 *        size, finiteness check on, median splits).
 * out    receives the tree handle; release it with kdt_free.
 *
 * With split_rule 0 (the default) splits are balanced: node (l, j) owns
 * points [floor(j n / 2^l), floor((j+1) n / 2^l)) of the tree order and is
 * split along the longest side of its tight bounding box (lowest axis on
 * ties) at the median, so that the depth is L = ceil(log2(ceil(n /
 * leaf_size))) for every leaf; the depth is known from n alone, which fixes
 * the launch schedule and lets the build run without host waits (other than
 * the finiteness check).  With split_rule 1 the paper's sliding-midpoint rule
 * (Sec. 2.1 steps 1-4) is used: the depth depends on the data, so the build
 * waits on `stream` once per level to size the next one.  Query results do
 * not depend on the split rule.
 *
 * Errors: KDT_EINVAL (NULL pointer, n out of range, non-finite coordinate when
 * checked), KDT_EUNSUPPORTED (d), KDT_ENOMEM, KDT_EDEVICE.
 */
kdt_status kdt_build(const float *d_pts, int64_t n, int32_t d, const kdt_build_opts *opts,
                     hipStream_t stream, kdt_tree **out);

/* Releases a tree.  Waits for the tree's build stream; the caller must have
   finished (or ordered before this call) every query that uses the tree. */
kdt_status kdt_free(kdt_tree *tree);

/*
 * Releases the device scratch the library keeps for `stream` between calls
 * (the particle-to-mesh deposits keep theirs, sized by the largest call so
 * far, so that repeated calls allocate nothing).  The memory is returned in
 * stream order (work already queued on `stream` finishes first).  Call it
 * before destroying a stream that ran deposits, or to give the memory back;
 * the next deposit on the stream allocates again.  Errors: KDT_EDEVICE.
 */
kdt_status kdt_stream_release(hipStream_t stream);

/* Fills *info (host). */
kdt_status kdt_tree_get_info(const kdt_tree *tree, kdt_tree_info *info);

/* The deferred finiteness check of a tree built with check_finite = 2: waits
   on `stream` and returns KDT_EINVAL if a coordinate was NaN or infinite,
   KDT_OK otherwise (also for trees built with check_finite 0 or 1). */
kdt_status kdt_tree_check(const kdt_tree *tree, hipStream_t stream);

/*
 * kdt_tree_gather, kdt_tree_scatter -- per-point arrays between input order
 * and the tree's order: rows of `width` 4-byte elements (float32 or int32;
 * 1 <= width <= 4096), d_in and d_out [n][width] device, not the same
 * array.  Gather: d_out[t] = d_in[kdt_tree_perm[t]] (input -> tree order);
 * scatter: d_out[kdt_tree_perm[t]] = d_in[t] (tree -> input order).
 * Asynchronous on `stream`; n = 0 does nothing.
 * Errors: KDT_EINVAL (NULL tree or arrays, width, d_in == d_out),
 * KDT_EDEVICE.
 */
kdt_status kdt_tree_gather(const kdt_tree *tree, const void *d_in, int32_t width, void *d_out,
                           hipStream_t stream);
kdt_status kdt_tree_scatter(const kdt_tree *tree, const void *d_in, int32_t width, void *d_out,
                            hipStream_t stream);

/*
 * Copies the tree to host memory for inspection (waits on `stream`).
 * h_pts [n][d] tree-ordered positions, h_perm [n] original index of each,
 * h_lo / h_hi [n_nodes][d] tight bounding box of each node in the numbering
 * of kdt_tree_nodes (heap order, node (l, j) at 2^l - 1 + j, for a median
 * tree), h_axis [n_nodes] split axis (-1 for leaves), h_split [n_nodes] split
 * coordinate (after any slide).  Any pointer may be NULL.
 */
kdt_status kdt_tree_export(const kdt_tree *tree, float *h_pts, int32_t *h_perm, float *h_lo,
                           float *h_hi, int32_t *h_axis, float *h_split, hipStream_t stream);

/*
 * Copies the node records to host memory (waits on `stream`): for each of
 * the n_nodes nodes, h_left the left child (-1 for a leaf; the right child is
 * h_left + 1), [h_begin, h_end) its points in tree order, h_level its depth.
 * Median trees report their implicit layout (node (l, j) at 2^l - 1 + j);
 * sliding-midpoint trees number their nodes level by level.  Any pointer may
 * be NULL.
 */
kdt_status kdt_tree_nodes(const kdt_tree *tree, int32_t *h_left, int32_t *h_begin,
                          int32_t *h_end, int32_t *h_level, hipStream_t stream);

/*
 * kdt_knn -- k nearest neighbours of nq query points (Sec. 2.3, Algorithm 2).
 *
 * d_q    [nq][d] float32 queries, or NULL to query every point of the tree
 *        itself (then nq must equal n and row i belongs to input point i).
 *        A query that is a data point finds itself at distance 0.
 * k      1 <= k <= KDT_MAX_K_SORTED.  Up to KDT_MAX_K the neighbour lists live
 *        in registers.  Above it each query first takes its 64th neighbour,
 *        scales that squared distance by 1.1 (k/64)^(2/d), grows it (from
 *        the density its count shows) until its closed ball holds at least
 *        k points, writes the
 *        (d2, index) keys of that ball and sorts them per query; results are
 *        the same as the register path's.  This mode waits on `stream` a few
 *        times, takes scratch of 16 bytes per candidate (queries are taken in
 *        chunks of at most 2^27 candidates, 2 GiB) from the stream-ordered
 *        pool, and fails with KDT_EUNSUPPORTED above 2^31-1 queries.
 * kth_only 0: write k results per row, ascending by (d2, index):
 *             d_idx [nq][k] int32 (may be NULL), d_d2 [nq][k] float32.
 *          1: write only the k-th squared distance, d_d2 [nq].
 *          2: write only the k-th distance sqrt(d2_k), d_d2 [nq] (an SPH
 *             smoothing length, Sec. 4.2).
 * Rows of a tree with fewer than k points are padded with (-1, +inf).
 * nq = 0 is an empty query set: nothing is read or written and every
 * pointer may be NULL (k and kth_only are still checked).
 * opts   may be NULL (sort_queries = 1).
 *
 * Errors: KDT_EINVAL, KDT_EUNSUPPORTED (k), KDT_ENOMEM, KDT_EDEVICE.
 */
kdt_status kdt_knn(const kdt_tree *tree, const float *d_q, int64_t nq, int32_t k,
                   int32_t *d_idx, float *d_d2, int32_t kth_only, const kdt_query_opts *opts,
                   hipStream_t stream);

/*
 * kdt_range -- ball query: the points within distance r of each query
 * (Sec. 2.3, Algorithm 3).  The ball is closed: a point is in when
 * d2 <= fl32(r * r).
 *
 * d_q       [nq][d] float32, or NULL for the tree's own points (nq == n).
 * r         finite, >= 0.
 * d_count   [nq] int32: number of points in each ball (required).
 * d_offsets [nq + 1] int64, or NULL.  When given together with d_idx the call
 *           also returns the lists in CSR form: row i is
 *           d_idx[d_offsets[i] .. d_offsets[i+1]) in ascending index order.
 *           This mode waits on `stream` once to learn the total size.
 * capacity  number of int32 slots in d_idx.
 * required  host, may be NULL: receives the total list length (list mode).
 * nq = 0 is an empty query set: d_q and d_count may be NULL; d_offsets, if
 * given, receives its single 0 and *required 0.
 * Scratch (the query order, and about 120 MB of task lists through which
 * heavy traversals are split over several launches) comes from the
 * stream-ordered pool and is released in stream order.  Counts are exact
 * integers however the work was split.
 *
 * Errors: KDT_EINVAL, KDT_ECAPACITY (total > capacity; *required is set and
 * d_count / d_offsets are valid), KDT_ENOMEM, KDT_EDEVICE.
 */
kdt_status kdt_range(const kdt_tree *tree, const float *d_q, int64_t nq, float r,
                     int32_t *d_count, int64_t *d_offsets, int32_t *d_idx, int64_t capacity,
                     int64_t *required, const kdt_query_opts *opts, hipStream_t stream);

/*
 * kdt_box -- axis-aligned box query: the rectangular ranges that Sec. 2.3
 * names beside the ball query.  Point x is inside box i when
 * d_lo[i][a] <= x[a] <= d_hi[i][a] on every axis a (closed on every side);
 * a box with lo > hi on some axis, or with a NaN bound, holds no point.
 *
 * d_lo, d_hi [nq][d] float32 (device): the boxes' corners; infinite bounds
 *           are allowed.
 * d_count   [nq] int32: number of points in each box (required).
 * d_offsets [nq + 1] int64, or NULL; with d_idx the call also returns the
 *           input indices in CSR form, ascending within each row.  This mode
 *           waits on `stream` once to learn the total size.
 * capacity, required: as for kdt_range.
 * opts      may be NULL; sort_queries orders the boxes by their centres along
 *           the tree; traversal 1 counts with one traversal per lane, 0 or 2
 *           with the wave-shared traversal of the ball counts (trees with
 *           leaf_size <= 64); split_budget as for kdt_range.  Results are
 *           identical either way.
 * nq = 0 is an empty query set: d_lo, d_hi and d_count may be NULL.
 * Scratch (the order, list staging) comes from the stream-ordered pool.
 *
 * Errors: KDT_EINVAL (also a traversal outside 0..2 or a negative
 * split_budget), KDT_ECAPACITY (total > capacity; *required is set and
 * d_count / d_offsets are valid), KDT_EUNSUPPORTED, KDT_ENOMEM, KDT_EDEVICE.
 */
kdt_status kdt_box(const kdt_tree *tree, const float *d_lo, const float *d_hi, int64_t nq,
                   int32_t *d_count, int64_t *d_offsets, int32_t *d_idx, int64_t capacity,
                   int64_t *required, const kdt_query_opts *opts, hipStream_t stream);

/*
 * kdt_fof -- friends-of-friends groups of the tree's points (Sec. 4.1).
 *
 * Points i != j are friends when d2(i, j) <= fl32(l * l); groups are the
 * connected components of that relation.  d_labels [n] int32 receives, for
 * every input point, the smallest input index of its group, so labels are
 * canonical and independent of scheduling.  n_groups (host, may be NULL)
 * receives the number of groups; asking for it waits on `stream`.
 *
 * Errors: KDT_EINVAL (l negative or non-finite), KDT_ENOMEM, KDT_EDEVICE.
 */
kdt_status kdt_fof(const kdt_tree *tree, float l, int32_t *d_labels, int64_t *n_groups,
                   hipStream_t stream);

/*
 * kdt_fof_torus -- friends-of-friends groups on the D-torus (Sec. 4.1 with the
 * periodic boundary conditions of Sec. 2.1 and Sec. 2.4): as kdt_fof, with
 * the distance of kdt_query_opts.period.  period: host array of d periods
 * L_a (finite, > 0); every tree point must lie in [0, L_a) (KDT_EINVAL
 * otherwise).  The call waits on `stream` once to check the periods against
 * the tree's bounding box.  One search per point and lane.
 *
 * Errors: KDT_EINVAL (l, period, points outside), KDT_ENOMEM, KDT_EDEVICE.
 */
kdt_status kdt_fof_torus(const kdt_tree *tree, float l, const float *period, int32_t *d_labels,
                         int64_t *n_groups, hipStream_t stream);

/*
 * kdt_p2m -- adaptive SPH particle-to-mesh deposit (Sec. 4.2).
 *
 * d_x [n][3], d_m [n], d_h [n] float32 device: positions, masses and
 * smoothing lengths (h_i = distance to the k-th neighbour, e.g. from
 * kdt_knn with kth_only = 2).  Every position must lie in the grid box.
 * Each particle spreads m_i over the cells whose centres lie within
 * H_i = max(h_i, cell) with the M4 cubic spline w(q), q = 2 r / H_i,
 * normalised over its in-grid cells, so the deposit conserves mass:
 *   rho_c = sum_i m_i w(q_ic) / S_i,   S_i = sum_c w(q_ic).
 * d_order [n] int32 or NULL: visiting order of the particles (for example the
 * tree order from kdt_tree_perm); it only changes speed and rounding order.
 * d_grid [n0*n1*n2] float32: overwritten with the mass per cell.  The sums are
 * accumulated in float64 and rounded once (the float64 summation order
 * follows the scheduling, a difference far below the float32 rounding).
 * On a periodic mesh (grid->periodic = 1) cells are reached the shorter way
 * round and nothing is cut at the faces; every H_i must then stay below half
 * of every period n[a]*cell (KDT_EINVAL otherwise) and n below 2^28.
 * n = 0 writes an all-zero mesh (the particle pointers may then be NULL).
 * The call waits on `stream` once, after the first pass, to read the
 * per-tile particle counts that size its lists (and the validity flag), and
 * again at the end; its buffers come from the stream-ordered pool.
 *
 * Errors: KDT_EINVAL (NULL pointer, bad grid, particle outside the box or an
 * invalid h -- detected on the device), KDT_EUNSUPPORTED (n >= 2^31, or
 * 2^28 on a periodic mesh, or a mesh of more than 2^30 tiles of 16^3 cells),
 * KDT_ENOMEM, KDT_EDEVICE.
 */
kdt_status kdt_p2m(const float *d_x, const float *d_m, const float *d_h, int64_t n,
                   const kdt_grid *grid, const int32_t *d_order, float *d_grid,
                   hipStream_t stream);

/*
 * kdt_p2m_cloud -- fixed-cloud particle-to-mesh deposit, the comparison the
 * paper draws against the adaptive kernel (Sec. 4.2, Table 3): scheme 1 NGP
 * (the cell holding the particle, floor((x - lo) / cell) in float32), 2 CIC
 * (weights 1 - f and f on the two cell centres around the particle per axis),
 * 3 TSC (0.5 (0.5 - u)^2, 0.75 - u^2, 0.5 (0.5 + u)^2 on the nearest centre
 * and its two neighbours, u the offset from the nearest centre in cells); a
 * cell's weight is the product over the axes.  On an open mesh cells outside
 * are dropped and the particle's weights renormalised, so mass is conserved;
 * a periodic mesh wraps (at least `scheme` cells per axis).  Arguments,
 * waits, accumulation and errors as kdt_p2m, without smoothing lengths.
 * Errors also: KDT_EINVAL for another scheme.
 */
kdt_status kdt_p2m_cloud(const float *d_x, const float *d_m, int64_t n, const kdt_grid *grid,
                         int32_t scheme, const int32_t *d_order, float *d_grid,
                         hipStream_t stream);

/*
 * kdt_p2m_backward -- adjoint of kdt_p2m for a loss L = sum_c g_c rho_c with
 * the smoothing lengths held fixed:
 *   dL/dm_i = A_i / S_i,   dL/dx_i = (m_i / S_i) (C_i - (A_i / S_i) B_i),
 * S = sum w, A = sum g w, B = sum grad w, C = sum g grad w over the particle's
 * in-grid cells, grad w = w'(q) (2 / H_i) (x_i - x_c) / r.  The weights are
 * recomputed, nothing per (particle, cell) is stored.
 * d_ggrid [cells] float32 upstream gradient.  d_gm [n], d_gx [n][3] float32
 * outputs, either may be NULL.  One lane per particle gathers in a fixed
 * order, so the result is reproducible.  Other arguments as kdt_p2m (n = 0:
 * nothing to do, pointers may be NULL); waits on `stream` at the end for the
 * validity flag.
 */
kdt_status kdt_p2m_backward(const float *d_x, const float *d_m, const float *d_h, int64_t n,
                            const kdt_grid *grid, const int32_t *d_order,
                            const float *d_ggrid, float *d_gm, float *d_gx,
                            hipStream_t stream);

/*
 * kdt_p2m_tree, kdt_p2m_tree_backward -- the deposit and its adjoint over
 * the points of a tree (Sec. 4.2 with the particles held in the tree's
 * order, the order every pass of the deposit visits them in): positions
 * come from the tree's own records, and d_m [n], d_h [n] and the outputs
 * d_gm [n], d_gx [n][3] are in tree order (row t belongs to input point
 * kdt_tree_perm[t]; kdt_tree_gather and kdt_tree_scatter convert, and
 * kdt_knn with tree_rows = 1 writes smoothing lengths in this order).  Every
 * pass then streams contiguous arrays instead of gathering through an
 * order.  scheme 0: the adaptive SPH kernel (d_h required); 1, 2, 3: the
 * fixed clouds NGP, CIC, TSC of kdt_p2m_cloud (d_h ignored).  The backward
 * is the adjoint of scheme 0.  Results are those of kdt_p2m /
 * kdt_p2m_cloud / kdt_p2m_backward with the tree order as d_order and the
 * per-particle arrays permuted accordingly.  A tree built with the deferred
 * finiteness check that found a NaN or infinite coordinate gives
 * KDT_EINVAL (read on the device with the validity flag); a tree built
 * without any check must not hold one (such a coordinate enters the tree as
 * 0).  Waits, accumulation, grid and other errors as kdt_p2m.
 * Errors also: KDT_EINVAL (NULL tree, scheme outside 0..3),
 * KDT_EUNSUPPORTED (d != 3, or a tree of float64 coordinates).
 */
kdt_status kdt_p2m_tree(const kdt_tree *tree, const float *d_m, const float *d_h,
                        const kdt_grid *grid, int32_t scheme, float *d_grid, hipStream_t stream);
kdt_status kdt_p2m_tree_backward(const kdt_tree *tree, const float *d_m, const float *d_h,
                                 const kdt_grid *grid, const float *d_ggrid, float *d_gm,
                                 float *d_gx, hipStream_t stream);

/*
 * kdt_query_order -- writes into d_order [nq] (int32, device) a deterministic
 * permutation of the queries that follows the tree's space, for reuse
 * through kdt_query_opts.order (the queries calls then skip their own sort).
 * kind 0: for d <= 4 the order of a Hilbert curve over the root bounding box
 *   (30 / d bits per axis), computed without touching the tree -- the order
 *   kdt_knn uses with one traversal per lane, and kdt_range; above d = 4 as
 *   kind 1.
 * kind 1: queries sorted by the leaf reached when descending towards the
 *   nearer child at every level -- the order the wave-packet kNN uses.
 * Results of the queries never depend on the order, only their speed.
 * nq = 0 does nothing (pointers may be NULL).
 * Errors: KDT_EINVAL (NULL pointer, nq outside [0, 2^31-1], other kind),
 * KDT_ENOMEM, KDT_EDEVICE.
 */
kdt_status kdt_query_order(const kdt_tree *tree, const float *d_q, int64_t nq, int32_t kind,
                           int32_t *d_order, hipStream_t stream);

/*
 * Float64 coordinates (the double-precision real kind of Sec. 2.4).
 *
 * kdt_build_f64 builds a tree over d_pts [n][d] float64 (device; n, d, opts
 * as for kdt_build, split_rule 0 or 1).  The tree's shape comes from the
 * float32 build over the coordinates rounded to float32 (clamped to the
 * float32 range, so coordinates beyond it are fine); the tree then stores
 * the float64 coordinates in tree order and the tight float64 box of every
 * node, and its queries compute in float64 only.  With check_finite (the
 * default) NaN/Inf coordinates give KDT_EINVAL (the call waits on `stream`).
 * Such a tree answers kdt_knn_f64, kdt_range_f64, kdt_query_order (from
 * float32 queries: the order only steers the work), kdt_tree_get_info,
 * kdt_tree_perm and kdt_tree_export (which exports the float32 rounding of
 * the coordinates); the float32 query calls return KDT_EUNSUPPORTED.
 * Release it with kdt_free.
 *
 * kdt_knn_f64: the k (1..KDT_MAX_K) smallest (d2, index) keys of each query
 * d_q [nq][d] float64 (NULL: every tree point, nq = n, row i = input point i), with
 * d2 the float64 squared distance summed over the axes in order (each
 * operation rounded on its own), ties by lower index, ascending; rows padded
 * with (-1, +inf) when k > n.  d_idx [nq][k] int32 (may be NULL), d_d2
 * [nq][k] float64.  opts: sort_queries and order as for kdt_knn (the order
 * may come from kdt_query_order); traversal and split_budget are ignored
 * (one traversal per lane); a period gives KDT_EUNSUPPORTED.
 *
 * kdt_range_f64: closed-ball counts (d2 <= fl64(r * r)) into d_count [nq]
 * int32, and with d_offsets [nq + 1] int64 the CSR lists as in kdt_range
 * (the call waits on `stream` to read the total; *required gets it;
 * d_idx may be NULL to size first; capacity below the total gives
 * KDT_ECAPACITY; every row ascending by input index).
 *
 * nq = 0 does nothing (pointers may be NULL).
 * Errors: KDT_EINVAL (NULL pointers, a tree not built by kdt_build_f64,
 * sizes out of range, r < 0 or NaN, k < 1), KDT_EUNSUPPORTED (d, k above
 * KDT_MAX_K, a period), KDT_ENOMEM, KDT_ECAPACITY, KDT_EDEVICE.
 */
kdt_status kdt_build_f64(const double *d_pts, int64_t n, int32_t d, const kdt_build_opts *opts,
                         hipStream_t stream, kdt_tree **out);
kdt_status kdt_knn_f64(const kdt_tree *tree, const double *d_q, int64_t nq, int32_t k,
                       int32_t *d_idx, double *d_d2, const kdt_query_opts *opts,
                       hipStream_t stream);
kdt_status kdt_range_f64(const kdt_tree *tree, const double *d_q, int64_t nq, double r,
                         int32_t *d_count, int64_t *d_offsets, int32_t *d_idx, int64_t capacity,
                         int64_t *required, const kdt_query_opts *opts, hipStream_t stream);

/*
 * The tuning table behind leaf_size = 0 and traversal = 0 (the paper tunes
 * N_leaf by hand, Sec. 2.1 and App. A; here it is measured).  An entry gives,
 * for a shape (d, n, k), the leaf size and the queries per traversal (1: one
 * per lane, 64: one shared by a wave) that the autotuner
 * (paper_2609_18316_amd/autotune.py) measured fastest.  The library holds
 * the table that tool last wrote; kdt_tuning_set adds or replaces an entry
 * for the rest of the process (thread-safe; keyed by d, log2 n rounded and
 * k; leaf_size = queries_per_wave = 0 removes the run-time entry of the
 * shape again).  A lookup takes the entry of dimension d nearest in
 * (log2 n, log2 k).
 *
 * kdt_tuning_get writes (host pointers, each may be NULL) the looked-up
 * leaf size and queries per traversal, and the traversal stack depth a
 * median tree of that shape needs: its depth L + 1 with
 * L = ceil(log2(ceil(n / leaf))) -- fixed by n and the leaf size, so it is
 * derived rather than tuned.
 *
 * Errors: KDT_EINVAL (d not in {2,3,4,8,16}, n < 1, k < 1; for _set also
 * leaf_size outside [2, 256] or queries_per_wave not 1 or 64).
 */
kdt_status kdt_tuning_set(int32_t d, int64_t n, int32_t k, int32_t leaf_size,
                          int32_t queries_per_wave);
kdt_status kdt_tuning_get(int32_t d, int64_t n, int32_t k, int32_t *leaf_size,
                          int32_t *queries_per_wave, int32_t *stack_depth);

/* Device pointer to the tree order: perm[t] is the input index of the point at
   tree position t (n int32, owned by the tree).  NULL on error. */
const int32_t *kdt_tree_perm(const kdt_tree *tree);

/*
 * Batched mode: many independent point sets of uneven size, concatenated.
 *
 * kdt_batch_plan_create fixes the shapes on the host: h_offsets [n_sets+1]
 * (host, int64, set s owns rows h_offsets[s] .. h_offsets[s+1], every set at
 * least one point, KDT_EINVAL otherwise), d, k, and the
 * options.  It allocates every buffer the pipeline needs, so a launch
 * allocates nothing.
 *
 * kdt_batch_launch builds one tree per set and runs, per set, kNN of every
 * point of the set (k from the plan) and friends-of-friends with the set's
 * linking length d_l[s] (device, float32 [n_sets]).  Outputs use set-local
 * indices: d_idx / d_d2 [total][k], d_labels [total].  Results are identical
 * to kdt_build + kdt_knn(NULL) + kdt_fof on each set.
 * use_graph = 1: the batched pipeline (forest build whose level kernels cover
 *   every set, persistent work-queue kNN and grouping kernels) is captured into
 *   a hipGraph on the first call and replayed; a call with different pointers
 *   captures again.  Nothing is allocated per call.
 * use_graph = 2: the same batched kernels launched eagerly (no graph).
 * use_graph = 0: the per-set baseline -- kdt_build, kdt_knn and kdt_fof called
 *   once per set, eagerly (waits on `stream` to read d_l).
 * bopts->leaf_size sets N_leaf for every set; 0 (or NULL bopts) gives each
 * set the tuned N_leaf of its own size (kdt_tuning_get(d, n_s, k));
 * qopts->traversal
 * picks the batched kNN kernel (0 and 2: wave packets, the measured default
 * for all-points queries; 1: one query per lane; leaf_size > 64 always uses
 * 1); qopts may be NULL and its other fields are unused.  Results are
 * identical either way.
 *
 * Errors: KDT_EINVAL, KDT_EUNSUPPORTED, KDT_ENOMEM, KDT_EDEVICE.
 */
kdt_status kdt_batch_plan_create(const int64_t *h_offsets, int32_t n_sets, int32_t d,
                                 int32_t k, const kdt_build_opts *bopts,
                                 const kdt_query_opts *qopts, kdt_batch_plan **out);
kdt_status kdt_batch_launch(kdt_batch_plan *plan, const float *d_pts, const float *d_l,
                            int32_t *d_idx, float *d_d2, int32_t *d_labels, int32_t use_graph,
                            hipStream_t stream);
kdt_status kdt_batch_plan_free(kdt_batch_plan *plan);

/*
 * kdt_knn_noalloc -- kdt_knn for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  It allocates nothing (no hipMalloc, no stream-ordered pool,
 * no allocating library routine) and waits on nothing.
 *
 * Arguments, results and errors as kdt_knn, restricted to what needs no
 * allocation: 1 <= k <= KDT_MAX_K and open boundaries (opts->period must be
 * NULL; otherwise KDT_EUNSUPPORTED).  The tree must live on the current
 * device (KDT_EINVAL otherwise).
 *
 * Its only scratch, the query order of sorted external queries, lives in a
 * static device array of KDT_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on every GPU it runs on until the process ends.  Ordering more than
 * KDT_NOALLOC_MAX_SORTED queries does not fit: KDT_ECAPACITY, with the limit
 * in kdt_last_error().  Queries in input order (sort_queries = 0), an order
 * passed in opts->order, and self queries (d_q NULL) use no scratch and have
 * no limit.
 *
 * All calls on one GPU share that GPU's array: calls that overlap in time on
 * one GPU (two streams, two threads) race on it and must be ordered by the
 * caller.  The array keeps the last call's contents; nothing in it has to
 * start at zero.
 */
#define KDT_NOALLOC_MAX_SORTED (1 << 22)
#define KDT_NOALLOC_SCRATCH_BYTES ((size_t)72 << 20)
kdt_status kdt_knn_noalloc(const kdt_tree *tree, const float *d_q, int64_t nq, int32_t k,
                           int32_t *d_idx, float *d_d2, int32_t kth_only,
                           const kdt_query_opts *opts, hipStream_t stream);

/* Message for the calling thread's last non-OK status ("" if none). */
const char *kdt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KDT_H */
