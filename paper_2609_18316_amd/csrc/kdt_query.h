// kdt_query.h -- device-side tree view and traversal helpers shared by the
// query, grouping and batched kernels.
#pragma once

#include "kdt_internal.h"

namespace kdt {

constexpr int kMaxDepth = 32;  // levels <= 30 for n < 2^31 and leaf_size >= 2

struct TreeView {
  const float* rec;  // [n][rec_stride(D)] tree-ordered records
  const float* box;  // [n_nodes][2 * pad4(D)]
  int64_t n;
  int32_t levels;    // depth of the deepest leaf
  const int4* nodes = nullptr;  // stored node records (sliding-midpoint trees), else NULL
  unsigned long long* visits = nullptr;  // work counters of the instrumented build, else NULL
};

// The wave-shared counts (and their list fill) over a median tree treat the
// nodes of one level as their leaves: the coarsest level whose nodes hold at
// most kCountLeaf points, never below the tree's own leaves.  Node ranges
// and tight boxes exist at every level, so the counts are the same; only
// the cost differs -- ball counts at r = 0.01 on 2^24 clustered points took
// 3.6 ms with 32-point leaves and 4.8 ms with 16-point ones.  Returns that
// view and, in *cap, its largest node (the LDS slices' leaf capacity).
constexpr int kCountLeaf = 32;
// The view at the coarsest level whose nodes hold at most `most` points.
inline TreeView coarse_view(TreeView v, int leaf, int most, int* cap) {
  int l = v.levels;
  while (l > 0 && ((v.n + (int64_t(1) << (l - 1)) - 1) >> (l - 1)) <= most) --l;
  const int64_t big = (v.n + (int64_t(1) << l) - 1) >> l;
  *cap = big > leaf ? (int)big : leaf;
  v.levels = l;
  return v;
}
inline TreeView count_view(TreeView v, int leaf, int* cap) {
  return coarse_view(v, leaf, kCountLeaf, cap);
}

// Where the wave-shared counts write CSR lists in fill mode: the indices of
// row r go to out[off[r] ..], a slot at a time reserved with an atomic on the
// row's cursor cur[r] (zero before the first pass), so the subtrees a wave
// hands on to later passes append the same way.  The order within a row
// depends on the schedule; callers sort each row afterwards.
struct FillOut {
  int32_t* out;
  const int64_t* off;
  int32_t* cur;
};

// Work counters of the instrumented build (compiled with KDT_COUNT_VISITS):
// how many node boxes and point records the traversals read, for the
// algorithmic bytes of the roofline.  Slots: kVisitNodes / kVisitPoints /
// kVisitInsert for one traversal per lane (nodes visited, i.e. node boxes
// tested -- the root and both children of every expanded node --, leaf
// records scanned, records read again to insert a candidate), kVisitReload
// for a box read again when its node leaves the stack (the stack keeps node
// ids only), kVisitWaveNodes / kVisitWavePoints for the wave-shared
// traversals (one box read and one leaf staged into LDS count once per
// wave).  Each slot has kVisitShards
// counters (workgroup b adds to shard b % kVisitShards).  In the product
// build the macros compile to nothing.
enum : int { kVisitNodes = 0, kVisitPoints = 1, kVisitInsert = 2, kVisitWaveNodes = 3,
             kVisitWavePoints = 4, kVisitReload = 5, kVisitSlots = 8 };
constexpr int kVisitShards = 64;
#ifdef KDT_COUNT_VISITS
__device__ __forceinline__ void count_visit(const TreeView& t, int slot, uint32_t n) {
  if (t.visits)
    atomicAdd(t.visits + slot * kVisitShards + (blockIdx.x % kVisitShards),
              (unsigned long long)n);
}
#define KDT_LANE_VISIT(t, slot, n) count_visit((t), (slot), (uint32_t)(n))
#define KDT_WAVE_VISIT(t, slot, n)                                  \
  do {                                                              \
    if (lane_id() == 0) count_visit((t), (slot), (uint32_t)(n));    \
  } while (0)
#else
#define KDT_LANE_VISIT(t, slot, n) ((void)0)
#define KDT_WAVE_VISIT(t, slot, n) ((void)0)
#endif

// Node layout of a tree, as the traversals see it.  A median tree is
// implicit: node (l, j) sits at 2^l - 1 + j, its children at 2v + 1 and
// 2v + 2, and it owns points [floor(j n / 2^l), floor((j + 1) n / 2^l)), so
// every leaf holds floor(n / 2^L) or one more.  A sliding-midpoint tree
// (Sec. 2.1, data-dependent depth) stores per node (left child or -1 for a
// leaf, first point, end point, level); its right child follows the left.
struct MedianShape {
  static constexpr bool kUniformLeaves = true;
  int64_t n;
  int levels;
  uint32_t first_leaf;
  __device__ __forceinline__ explicit MedianShape(const TreeView& t)
      : n(t.n), levels(t.levels), first_leaf((1u << t.levels) - 1u) {}
  __device__ __forceinline__ bool is_leaf(uint32_t v) const { return v >= first_leaf; }
  __device__ __forceinline__ uint32_t left(uint32_t v) const { return 2 * v + 1; }
  __device__ __forceinline__ void range(uint32_t v, int64_t& b, int64_t& e) const {
    const int lev = 31 - __clz(v + 1);
    const int64_t j = (int64_t)v - ((int64_t(1) << lev) - 1);
    b = (j * n) >> lev;
    e = ((j + 1) * n) >> lev;
  }
};

struct StoredShape {
  static constexpr bool kUniformLeaves = false;
  const int4* node;
  __device__ __forceinline__ explicit StoredShape(const TreeView& t) : node(t.nodes) {}
  __device__ __forceinline__ bool is_leaf(uint32_t v) const { return node[v].x < 0; }
  __device__ __forceinline__ uint32_t left(uint32_t v) const { return (uint32_t)node[v].x; }
  __device__ __forceinline__ void range(uint32_t v, int64_t& b, int64_t& e) const {
    const int4 r = node[v];
    b = r.y;
    e = r.z;
  }
};

template <int D>
struct Pt {
  float v[D];
};

template <int D>
__device__ __forceinline__ void load_box(const float* __restrict__ box, uint32_t node, float lo[D],
                                         float hi[D]) {
  constexpr int P = pad4(D);
  const float4* b = reinterpret_cast<const float4*>(box + (size_t)node * 2 * P);
#pragma unroll
  for (int q = 0; q < P / 4; ++q) {
    float4 l = b[q], h = b[P / 4 + q];
    if (4 * q + 0 < D) lo[4 * q + 0] = l.x, hi[4 * q + 0] = h.x;
    if (4 * q + 1 < D) lo[4 * q + 1] = l.y, hi[4 * q + 1] = h.y;
    if (4 * q + 2 < D) lo[4 * q + 2] = l.z, hi[4 * q + 2] = h.z;
    if (4 * q + 3 < D) lo[4 * q + 3] = l.w, hi[4 * q + 3] = h.w;
  }
}

// Smallest squared distance from p to the box: the same float32 operations,
// in the same axis order, as the point distance, so it never exceeds the
// rounded distance of any point inside the box.
// The axis gap max(lo - p, p - hi, 0) is exactly lo - p below the box, p - hi
// above it and 0 inside (a max does not round), taken without branches.
template <int D>
__device__ __forceinline__ float box_mindist(const float lo[D], const float hi[D], const float p[D]) {
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float t = fmaxf(fmaxf(lo[a] - p[a], p[a] - hi[a]), 0.0f);
    float t2 = t * t;
    s = s + t2;
  }
  return s;
}

// Largest squared distance from p to the box (never below any point's).
template <int D>
__device__ __forceinline__ float box_maxdist(const float lo[D], const float hi[D], const float p[D]) {
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float t1 = fabsf(p[a] - lo[a]);
    float t2 = fabsf(p[a] - hi[a]);
    float t = t1 > t2 ? t1 : t2;
    float tt = t * t;
    s = s + tt;
  }
  return s;
}

// Squared Euclidean distance (Eq. 1, p = 2): float32, axes left to right,
// every operation rounded on its own (the library is built without FMA
// contraction).
template <int D>
__device__ __forceinline__ float sq_dist(const float* __restrict__ x, const float p[D]) {
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float t = x[a] - p[a];
    float t2 = t * t;
    s = s + t2;
  }
  return s;
}

template <int D>
__device__ __forceinline__ void load_rec(const float* __restrict__ rec, int64_t i, float x[D],
                                         int32_t& idx) {
  constexpr int S = rec_stride(D);
  const float4* r = reinterpret_cast<const float4*>(rec + i * S);
#pragma unroll
  for (int q = 0; q < S / 4; ++q) {
    float4 v = r[q];
    float w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int a = 4 * q + c;
      if (a < D) x[a] = w[c];
      if (a == D) idx = __float_as_int(w[c]);
    }
  }
}

// Reads of wave-uniform addresses in data that no kernel writes while it
// runs (node boxes): through the constant address space, so the compiler
// issues scalar loads, one per wave.
typedef const __attribute__((address_space(4))) float cfloat;
__device__ __forceinline__ const cfloat* as_uniform(const float* p) {
  return (const cfloat*)p;
}

// Box of a node whose index is wave-uniform.
template <int D>
__device__ __forceinline__ void load_box_uniform(const float* box, uint32_t node, float lo[D],
                                                 float hi[D]) {
  constexpr int P = pad4(D);
  const cfloat* b = as_uniform(box) + (size_t)node * 2 * P;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lo[a] = b[a];
    hi[a] = b[P + a];
  }
}

// Leaf points a wave-uniform scan keeps in flight (a loop unroll factor).
template <int D>
constexpr int uniform_batch() {
  return D <= 4 ? 8 : (32 / D > 0 ? 32 / D : 1);
}

// Key of an empty candidate slot: squared distance +inf, index 0xFFFFFFFF, so
// it sorts after every real point (indices are below 2^31).
constexpr uint64_t kEmptyKey = 0x7F800000FFFFFFFFull;

// Sorted register list of the KC smallest 64-bit keys (d2 bits << 32 | index).
// Only the last k slots are live: the first KC - k hold 0 and never move.
//
// The keys are stored as float64 bit patterns: for d2 >= 0 (never NaN) the
// key's sign bit is 0 and its exponent field can never be all ones, so the
// float64 order of the patterns is exactly the unsigned order of the keys
// (keys below 2^52 are subnormal doubles, which the float64 min/max keep
// exact because float64 subnormals are not flushed).  That turns each
// compare-and-carry step into one v_min_f64 and one v_max_f64.
template <int KC>
struct TopK {
  double a[KC];
  __device__ __forceinline__ void init(int k) {
#pragma unroll
    for (int i = 0; i < KC; ++i) a[i] = (i < KC - k) ? 0.0 : __longlong_as_double((long long)kEmptyKey);
  }
  __device__ __forceinline__ uint64_t key(int i) const {
    return (uint64_t)__double_as_longlong(a[i]);
  }
  __device__ __forceinline__ uint64_t worst() const { return key(KC - 1); }
  __device__ __forceinline__ float worst_d2() const {
    return __uint_as_float((uint32_t)(worst() >> 32));
  }
  // Inserts x if it is below worst(), otherwise leaves the list unchanged
  // (no branch, so it can run on every lane of a wave).  One bottom-up pass
  // of compare-and-carry: each slot keeps the smaller of itself and the carry
  // and hands the larger upwards; the largest key falls off the top.
  //
  // Every key read as a float64 is finite and non-negative (the high word is
  // a non-negative float32, so the float64 exponent stays below 0x7FF), so
  // the hardware min/max order keys exactly.  They are issued directly: the
  // library fmin/fmax would first canonicalise both operands of every slot
  // (IEEE mode), half as many instructions again.
  __device__ __forceinline__ void insert(uint64_t x) {
    double carry = __longlong_as_double((long long)x);
#pragma unroll
    for (int i = 0; i < KC; ++i) {
      double up;
      asm("v_max_f64 %1, %0, %2\n\tv_min_f64 %0, %0, %2"
          : "+v"(a[i]), "=&v"(up)
          : "v"(carry));
      carry = up;
    }
  }
  __device__ __forceinline__ void offer(float d2, int32_t id);
};

__device__ __forceinline__ uint64_t make_key(float d2, int32_t idx) {
  return ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)idx;
}

template <int KC>
__device__ __forceinline__ void TopK<KC>::offer(float d2, int32_t id) {
  const uint64_t key = make_key(d2, id);
  if (key < worst()) insert(key);
}

// The k smallest squared distances alone, for queries that want only the
// k-th distance: its value does not depend on how equal distances are
// ordered, so no index is kept and the list takes half the registers of
// TopK.  Entries are the bit patterns of non-negative float32 values (or
// +inf), which order like the values, so integer min/max keep the list
// sorted without any float rounding or denormal handling.
template <int KC>
struct TopD {
  uint32_t a[KC];
  __device__ __forceinline__ void init(int k) {
#pragma unroll
    for (int i = 0; i < KC; ++i) a[i] = (i < KC - k) ? 0u : 0x7F800000u;
  }
  __device__ __forceinline__ float worst_d2() const { return __uint_as_float(a[KC - 1]); }
  __device__ __forceinline__ void offer(float d2, int32_t) {
    const uint32_t x = __float_as_uint(d2);
    if (x < a[KC - 1]) {
      uint32_t carry = x;
#pragma unroll
      for (int i = 0; i < KC; ++i) {
        const uint32_t up = max(a[i], carry);
        a[i] = min(a[i], carry);
        carry = up;
      }
    }
  }
};

// Open-space metric of the traversals: the point distance (Eq. 1, p = 2) and
// the lower and upper bounds over a node box.  Other metrics (the D-torus of
// periodic boundaries) supply the same three.
template <int D>
struct OpenMetric {
  __device__ __forceinline__ float dist(const float x[D], const float p[D]) const {
    return sq_dist<D>(x, p);
  }
  __device__ __forceinline__ float mindist(const float lo[D], const float hi[D],
                                           const float p[D]) const {
    return box_mindist<D>(lo, hi, p);
  }
  __device__ __forceinline__ float maxdist(const float lo[D], const float hi[D],
                                           const float p[D]) const {
    return box_maxdist<D>(lo, hi, p);
  }
};

// kNN of one query p over tree t (Algorithm 2 semantics): depth-first, nearer
// child first, a node is skipped when its box is farther than the current
// k-th candidate.  `stk` is this lane's column of an LDS stack with stride
// `ld` entries.
template <int D, class List, class Metric = OpenMetric<D>, class Shape = MedianShape>
__device__ __forceinline__ void knn_one(const TreeView& t, const float p[D], List& best,
                                        uint32_t* stk, int ld, const Metric& metric = Metric()) {
  const Shape sh(t);
  // median trees: every leaf holds floor(n / 2^L) or one more points
  const int lmin = (int)(t.n >> t.levels);
  const int lmax = (int)((t.n + (int64_t(1) << t.levels) - 1) >> t.levels);
  float lo[D], hi[D];
  load_box<D>(t.box, 0, lo, hi);
  KDT_LANE_VISIT(t, kVisitNodes, 1);
  uint32_t node = 0;
  float nd = metric.mindist(lo, hi, p);
  int sp = 0;
  for (;;) {
    if (nd <= best.worst_d2()) {
      if (sh.is_leaf(node)) {
        int64_t b, e;
        sh.range(node, b, e);
        KDT_LANE_VISIT(t, kVisitPoints, e - b);
        // Two passes per block of up to 64 leaf points.  The first computes
        // every distance and marks the points that can enter the list (float
        // test against the current k-th distance, ties kept); the second
        // inserts the marked points, recomputing their distances.  The
        // insertion is the expensive step and runs for the whole wave when
        // any lane inserts, so marking first makes the wave pay for the
        // largest number of insertions of one lane in this leaf, not for
        // every position at which some lane inserts.
        for (int64_t c = b; c < e; c += 64) {
          const float w = best.worst_d2();
          uint64_t mask = 0;
          if (Shape::kUniformLeaves && lmax <= 32) {
            // Every leaf holds lmin or lmin + 1 points: the first lmin are
            // scanned with a wave-uniform trip count, the possible last one
            // on its own (one block: e - b <= 32).
            uint32_t m32 = 0;
#pragma unroll 1  // unrolling costs occupancy (measured slower at k = 32)
            for (int i = 0; i < lmin; ++i) {
              float x[D];
              int32_t id = 0;
              load_rec<D>(t.rec, b + i, x, id);
              m32 |= (uint32_t)(metric.dist(x, p) <= w) << i;
            }
            if (e - b > lmin) {
              float x[D];
              int32_t id = 0;
              load_rec<D>(t.rec, b + lmin, x, id);
              m32 |= (uint32_t)(metric.dist(x, p) <= w) << lmin;
            }
            mask = m32;
          } else {
            const int m = (int)((e - c) < 64 ? (e - c) : 64);
            for (int i = 0; i < m; ++i) {
              float x[D];
              int32_t id = 0;
              load_rec<D>(t.rec, c + i, x, id);
              if (metric.dist(x, p) <= w) mask |= 1ull << i;
            }
          }
          KDT_LANE_VISIT(t, kVisitInsert, __popcll(mask));
          while (mask) {
            const int i = __builtin_ctzll(mask);
            mask &= mask - 1;
            float x[D];
            int32_t id = 0;
            load_rec<D>(t.rec, c + i, x, id);
            best.offer(metric.dist(x, p), id);
          }
        }
      } else {
        const uint32_t c0 = sh.left(node), c1 = c0 + 1;
        KDT_LANE_VISIT(t, kVisitNodes, 2);
        load_box<D>(t.box, c0, lo, hi);
        const float d0 = metric.mindist(lo, hi, p);
        load_box<D>(t.box, c1, lo, hi);
        const float d1 = metric.mindist(lo, hi, p);
        const bool first0 = d0 <= d1;
        const uint32_t nn = first0 ? c0 : c1, ff = first0 ? c1 : c0;
        const float dn = first0 ? d0 : d1, df = first0 ? d1 : d0;
        if (df <= best.worst_d2()) stk[sp++ * ld] = ff;
        node = nn;
        nd = dn;
        continue;
      }
    }
    if (sp == 0) break;
    // only the node id is kept on the stack; its box distance is recomputed
    // (the box is cache-resident), halving the stack's LDS footprint
    node = stk[--sp * ld];
    KDT_LANE_VISIT(t, kVisitReload, 1);
    load_box<D>(t.box, node, lo, hi);
    nd = metric.mindist(lo, hi, p);
  }
}

// Writes one kNN row: mode 0 -> k (index, d2) pairs, 1 -> d2 of the k-th,
// 2 -> distance of the k-th.
template <int KC>
__device__ __forceinline__ void knn_write(const TopK<KC>& best, int k, int mode, int64_t row,
                                          int32_t* __restrict__ oidx, float* __restrict__ od2) {
  if (mode == 0) {
#pragma unroll
    for (int j = 0; j < KC; ++j) {
      if (j < KC - k) continue;
      const uint64_t key = best.key(j);
      const bool empty = key == kEmptyKey;
      const int64_t o = row * k + (j - (KC - k));
      if (oidx) oidx[o] = empty ? -1 : (int32_t)(uint32_t)key;
      od2[o] = empty ? INFINITY : __uint_as_float((uint32_t)(key >> 32));
    }
  } else {
    const uint64_t key = best.key(KC - 1);
    const float d2 = key == kEmptyKey ? INFINITY : __uint_as_float((uint32_t)(key >> 32));
    od2[row] = mode == 2 ? sqrtf(d2) : d2;
  }
}

// The k-th squared distance (mode 1) or distance (mode 2) of a TopD list.
template <int KC>
__device__ __forceinline__ void knn_write_kth(const TopD<KC>& best, int mode, int64_t row,
                                              float* __restrict__ od2) {
  const float d2 = best.worst_d2();
  od2[row] = mode == 2 ? sqrtf(d2) : d2;
}

// Lock-free union-find on int32 parents with parent[y] <= y.
__device__ __forceinline__ int32_t uf_ld(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void uf_st(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x.  Only roots change owner, so shortcutting a non-root to any of
// its ancestors is always valid.
__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t x) {
  int32_t cur = uf_ld(parent + x);
  if (cur == x) return x;
  int32_t prev = x;
  for (;;) {
    const int32_t next = uf_ld(parent + cur);
    if (next >= cur) break;
    uf_st(parent + prev, next);
    prev = cur;
    cur = next;
  }
  return cur;
}

// Joins the set of the element whose known ancestor is `a` (updated to an
// ancestor of the joined set's root) with the set of b: the larger root is
// hooked under the smaller, so every root is the smallest index of its set.
// A root found once stays an ancestor of its elements after it is hooked
// (only roots change parent), so a lane that links one point many times
// keeps its last root in `a` and starts every search there.
//
// Two elements that share any ancestor are in one set, so when b is a or b's
// parent is a (the usual case once paths are compressed) nothing is left to
// do after a single load.
__device__ __forceinline__ void uf_union_from(int32_t* parent, int32_t& a, int32_t b) {
  if (b == a) return;
  const int32_t pb = uf_ld(parent + b);
  if (pb == a) return;
  int32_t ra = uf_find(parent, a), rb = pb == b ? b : uf_find(parent, pb);
  while (ra != rb) {
    if (ra < rb) {
      const int32_t old = atomicCAS(parent + rb, rb, ra);
      if (old == rb) break;
      rb = old;
    } else {
      const int32_t old = atomicCAS(parent + ra, ra, rb);
      if (old == ra) {
        ra = rb;
        break;
      }
      ra = old;
    }
  }
  a = ra;
}

// Joins the sets of a and b.
__device__ __forceinline__ void uf_union(int32_t* parent, int32_t a, int32_t b) {
  uf_union_from(parent, a, b);
}

// Squared diagonal of a box: every pair of points inside is at most this far
// apart (same operation order as the point distance).
template <int D>
__device__ __forceinline__ float box_diag2(const float lo[D], const float hi[D]) {
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float t = hi[a] - lo[a];
    float t2 = t * t;
    s = s + t2;
  }
  return s;
}

__device__ __forceinline__ uint32_t flag_ld(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void flag_st(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Friends-of-friends links of the point p at tree position `pos` (index me)
// of tree t.  Union-find indices are base + index.  conn[v] != 0 records that
// every point of node v is already (or will be, once the running unions land)
// in one component; such a node needs a single link to p, and once one friend
// is found inside it the rest of its subtree is skipped.
template <int D, class Shape = MedianShape>
__device__ __forceinline__ void fof_point(const TreeView& t, const float p[D], int64_t pos,
                                          int32_t me, float l2, int32_t base,
                                          int32_t* __restrict__ parent,
                                          uint32_t* __restrict__ conn, uint32_t* stk, int ld) {
  constexpr int S = rec_stride(D);
  const Shape sh(t);
  int sp = 1;
  stk[0] = 0;
  int32_t myroot = base + me;  // an ancestor of p's set root (see uf_union_from)
  int guard = -1;  // stack depth where the current one-component region began
  while (sp > 0) {
    --sp;
    if (guard >= 0 && sp < guard) guard = -1;
    const uint32_t node = stk[sp * ld];
    int64_t b, e;
    sh.range(node, b, e);
    // links go towards later tree positions only: a node that ends at or
    // before p's position is left to the points inside it
    if (e <= pos) continue;
    float lo[D], hi[D];
    load_box<D>(t.box, node, lo, hi);
    if (box_mindist<D>(lo, hi, p) > l2) continue;
    const bool in_region = guard >= 0;
    const bool one = in_region || flag_ld(conn + node) != 0;
    if (one && pos >= b && pos < e) continue;  // p is already in this component
    if (box_maxdist<D>(lo, hi, p) <= l2) {
      if (one) {
        uf_union_from(parent, myroot, base + __float_as_int(t.rec[b * S + D]));
        if (in_region) {
          sp = guard;
          guard = -1;
        }
      } else {
        for (int64_t i = b; i < e; ++i)
          uf_union_from(parent, myroot, base + __float_as_int(t.rec[i * S + D]));
        flag_st(conn + node, 1u);
      }
      continue;
    }
    if (sh.is_leaf(node)) {
      for (int64_t i = b; i < e; ++i) {
        float x[D];
        int32_t id = 0;
        load_rec<D>(t.rec, i, x, id);
        if (sq_dist<D>(x, p) > l2) continue;
        if (one) {
          uf_union_from(parent, myroot, base + id);
          if (in_region) {
            sp = guard;
            guard = -1;
          }
          break;
        }
        if (i > pos) uf_union_from(parent, myroot, base + id);
      }
      continue;
    }
    if (one && !in_region) guard = sp;
    const uint32_t c0 = sh.left(node);
    stk[sp++ * ld] = c0 + 1;
    stk[sp++ * ld] = c0;
  }
}

// Marks nodes whose box diagonal is within the linking length: all their
// points are mutual friends.
template <int D>
__device__ __forceinline__ void fof_mark_clique(const float* __restrict__ box, int64_t node,
                                                float l2, uint32_t* __restrict__ conn) {
  float lo[D], hi[D];
  load_box<D>(box, (uint32_t)node, lo, hi);
  conn[node] = box_diag2<D>(lo, hi) <= l2 ? 1u : 0u;
}

// Joins the point at tree position pos with the first point of the largest
// clique node above it (so every maximal clique becomes one component).
template <int D>
__device__ __forceinline__ void fof_join_clique(const TreeView& t, int64_t pos, int32_t me,
                                                int32_t base, int32_t* __restrict__ parent,
                                                const uint32_t* __restrict__ conn) {
  constexpr int S = rec_stride(D);
  const int64_t first_leaf = (int64_t(1) << t.levels) - 1;
  // leaf holding pos: largest j with node_begin(n, L, j) <= pos
  int64_t j = ((pos + 1) << t.levels) / t.n;
  while (j > 0 && node_begin(t.n, t.levels, j) > pos) --j;
  while (node_begin(t.n, t.levels, j + 1) <= pos) ++j;
  int64_t v = first_leaf + j;
  if (!conn[v]) return;
  while (v > 0 && conn[(v - 1) >> 1]) v = (v - 1) >> 1;
  const int lev = node_level((uint32_t)v);
  const int64_t b = node_begin(t.n, lev, v - ((int64_t(1) << lev) - 1));
  const int32_t first = __float_as_int(t.rec[b * S + D]);
  if (first != me) uf_union(parent, base + me, base + first);
}

// Root of x without shortcuts (safe while other lanes write final labels).
__device__ __forceinline__ int32_t uf_root(const int32_t* parent, int32_t x) {
  int32_t cur = x;
  for (;;) {
    const int32_t next = uf_ld(parent + cur);
    if (next >= cur) return cur;
    cur = next;
  }
}

template <int D>
kdt_status knn_packet_launch(const TreeView& v, int leaf, const float* d_q, int64_t nq, int k,
                             int32_t* d_idx, float* d_d2, int mode, const int32_t* order,
                             hipStream_t stream);
// Periodic boundaries (opts->period): kNN (k <= KDT_MAX_K) and ball queries
// on the D-torus, arguments as kdt_knn / kdt_range.
kdt_status knn_torus(const kdt_tree* tr, const float* d_q, int64_t nq, int k, int32_t* d_idx,
                     float* d_d2, int mode, bool sort_q, const int32_t* given,
                     const float* period, hipStream_t stream);
kdt_status range_torus(const kdt_tree* tr, const float* d_q, int64_t nq, float r,
                       int32_t* d_count, int64_t* d_off, int32_t* d_idx, int64_t capacity,
                       int64_t* required, bool sort_q, const int32_t* given, const float* period,
                       bool counts_given, hipStream_t stream);

// k above KDT_MAX_K: exact neighbours from a per-query ball that holds at
// least k points, its keys sorted per query (arguments as kdt_knn; period
// NULL for open boundaries).
kdt_status knn_large(const kdt_tree* tr, const float* d_q, int64_t nq, int k, int32_t* d_idx,
                     float* d_d2, int mode, bool sort_q, const int32_t* given,
                     const float* period, hipStream_t stream);

// kdt_knn's options after its argument checks.
struct KnnArgs {
  bool empty = false;  // nq == 0: nothing to do
  bool sort_q = true;
  int traversal = 0;
  // external queries: the caller's order or NULL; self queries: the
  // tree-order row marker (self_rows) or NULL
  const int32_t* given = nullptr;
  const float* period = nullptr;
};
// Checks kdt_knn's arguments (`who` names the entry point in messages).
kdt_status knn_check(const kdt_tree* tree, const float* d_q, int64_t nq, int32_t k,
                     const float* d_d2, int32_t kth_only, const kdt_query_opts* opts,
                     const char* who, KnnArgs* a);
// kNN with k <= KDT_MAX_K and open boundaries.  With a workspace (ws_bytes
// bytes of device memory) the query order, the only scratch of this path,
// is carved from it and nothing is allocated; KDT_ECAPACITY if it is too
// small.  ws == NULL: scratch from the stream-ordered pool.
kdt_status knn_in_workspace(const kdt_tree* t, const float* d_q, int64_t nq, int k,
                            int32_t* d_idx, float* d_d2, int mode, const KnnArgs& a, void* ws,
                            size_t ws_bytes, hipStream_t stream);

template <int D>
kdt_status range_packet_launch(const TreeView& v, int leaf, const float* d_q, int64_t nq, float r2,
                               const int32_t* order, int32_t* d_count, uint32_t split_budget,
                               hipStream_t stream, const FillOut* fill = nullptr);
template <int D>
kdt_status fof_packet_launch(const TreeView& v, int leaf, float l2, int32_t* parent, uint32_t* conn,
                             hipStream_t stream);

}  // namespace kdt
