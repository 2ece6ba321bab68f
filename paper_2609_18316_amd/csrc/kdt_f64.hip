// Float64 coordinates: the double-precision real kind of Sec. 2.4 (the
// paper's library picks float32 or float64 coordinates when it is compiled;
// here both live in one library and the float64 variant has entry points of
// its own).
//
// Build: the tree's shape (its splits and the tree order) is built by the
// float32 build from the coordinates rounded to float32 (clamped to the
// float32 range) -- any partition of the points gives correct queries, and
// the shape only steers the work.  The float64 coordinates are then stored in
// tree order and every node gets the tight float64 box of its own points,
// leaves from their points and inner nodes from their children, so pruning
// is exact for the float64 points.
//
// Queries (kNN with k <= 64, closed-ball counts and CSR lists) take one
// traversal per lane, depth first, nearer child first, with the node stack in
// LDS.  Squared distances are float64 sums over the axes in order, each
// operation rounded on its own; a node is pruned when its box distance is
// above the current k-th key's distance (kNN) or above fl64(r * r) (balls),
// and taken whole when its farthest corner is within the ball (Algorithm 3).
// Rounding is monotone, so a box bound computed this way never exceeds the
// computed distance of a point inside the box: no point that belongs to the
// answer is pruned.  Keys are (d2, index) pairs compared lexicographically,
// as in the float32 path; the candidate list is a sorted register array.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdint>

#include "kdt.h"
#include "kdt_internal.h"
#include "kdt_query.h"

namespace kdt {
namespace {

constexpr int kF64Block = 64;  // one wave per workgroup: the LDS stack is 4 B x depth per lane

struct View64 {
  const double* rec;   // [n][D] tree-ordered coordinates
  const double* box;   // [n_nodes][2][D] lo then hi
  const int32_t* perm; // [n] input index of each tree position
  int64_t n;
  int32_t levels;
  const int4* nodes;   // stored nodes (sliding-midpoint trees) or NULL
};

__device__ __forceinline__ TreeView shape_view(const View64& v) {
  TreeView t{};
  t.rec = nullptr;
  t.box = nullptr;
  t.n = v.n;
  t.levels = v.levels;
  t.nodes = v.nodes;
  return t;
}

View64 view64(const kdt_tree* t) {
  return View64{t->rec64, t->box64, t->perm, t->n, t->levels, t->nodes};
}

__global__ void k_to_f32(const double* __restrict__ x, int64_t m, float* __restrict__ y,
                         int32_t* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double v = x[i];
  if (!isfinite(v)) {
    atomicOr(bad, 1);
    y[i] = 0.0f;
    return;
  }
  y[i] = (float)fmin(fmax(v, -(double)FLT_MAX), (double)FLT_MAX);
}

template <int D>
__global__ void k_gather64(const double* __restrict__ x, const int32_t* __restrict__ perm,
                           int64_t n, double* __restrict__ rec) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t i = perm[t];
#pragma unroll
  for (int a = 0; a < D; ++a) rec[t * D + a] = x[i * D + a];
}

// Leaves: the tight box of their points (an empty range gives lo = +inf,
// hi = -inf, a box every bound prunes).
template <int D, typename Shape>
__global__ void k_leaf_boxes64(View64 v, int64_t n_nodes, double* __restrict__ box) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= n_nodes) return;
  const Shape shape(shape_view(v));
  if (!shape.is_leaf((uint32_t)node)) return;
  int64_t b, e;
  shape.range((uint32_t)node, b, e);
  double lo[D], hi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) lo[a] = INFINITY, hi[a] = -INFINITY;
  for (int64_t r = b; r < e; ++r)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double c = v.rec[r * D + a];
      lo[a] = fmin(lo[a], c);
      hi[a] = fmax(hi[a], c);
    }
#pragma unroll
  for (int a = 0; a < D; ++a) box[node * 2 * D + a] = lo[a], box[node * 2 * D + D + a] = hi[a];
}

// Inner nodes of one level: the union of their children's boxes.
template <int D, typename Shape>
__global__ void k_inner_boxes64(View64 v, int64_t first, int64_t count, int level,
                                double* __restrict__ box) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t node = first + i;
  if (v.nodes && v.nodes[node].w != level) return;
  const Shape shape(shape_view(v));
  if (shape.is_leaf((uint32_t)node)) return;
  const int64_t c = shape.left((uint32_t)node);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    box[node * 2 * D + a] = fmin(box[c * 2 * D + a], box[(c + 1) * 2 * D + a]);
    box[node * 2 * D + D + a] =
        fmax(box[c * 2 * D + D + a], box[(c + 1) * 2 * D + D + a]);
  }
}

template <int D>
__device__ __forceinline__ double box_min64(const double* __restrict__ box, uint32_t node,
                                            const double q[D]) {
  const double* lo = box + (size_t)node * 2 * D;
  const double* hi = lo + D;
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    double t = 0.0;
    if (q[a] < lo[a])
      t = lo[a] - q[a];
    else if (q[a] > hi[a])
      t = q[a] - hi[a];
    s += t * t;
  }
  return s;
}

template <int D>
__device__ __forceinline__ double box_max64(const double* __restrict__ box, uint32_t node,
                                            const double q[D]) {
  const double* lo = box + (size_t)node * 2 * D;
  const double* hi = lo + D;
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double t = fmax(fabs(q[a] - lo[a]), fabs(hi[a] - q[a]));
    s += t * t;
  }
  return s;
}

template <int D>
__device__ __forceinline__ double sq_dist64(const double* __restrict__ p, const double q[D]) {
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double t = p[a] - q[a];
    s += t * t;
  }
  return s;
}

// The query of lane slot i: its coordinates and the output row.
template <int D>
__device__ __forceinline__ int64_t load_query64(const View64& v, const double* __restrict__ q,
                                                const int32_t* __restrict__ order, int64_t i,
                                                double qq[D]) {
  if (q) {
    const int64_t row = order ? order[i] : i;
#pragma unroll
    for (int a = 0; a < D; ++a) qq[a] = q[row * D + a];
    return row;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) qq[a] = v.rec[i * D + a];
  return order ? i : v.perm[i];  // self queries: tree order when order is set
}

template <int D, int KC, typename Shape>
__global__ __launch_bounds__(kF64Block) void k_knn64(View64 v, const double* __restrict__ q,
                                                     int64_t nq, int k,
                                                     const int32_t* __restrict__ order,
                                                     int32_t* __restrict__ out_idx,
                                                     double* __restrict__ out_d2, int depth) {
  extern __shared__ uint32_t stk[];  // [depth][kF64Block]
  const int64_t i = (int64_t)blockIdx.x * kF64Block + threadIdx.x;
  if (i >= nq) return;
  double qq[D];
  const int64_t row = load_query64<D>(v, q, order, i, qq);
  const Shape shape(shape_view(v));
  double kd[KC];
  int32_t ki[KC];
#pragma unroll
  for (int j = 0; j < KC; ++j) kd[j] = INFINITY, ki[j] = INT_MAX;
  double wd = INFINITY;  // the k-th key
  int32_t wi = INT_MAX;
  int sp = 0;
  uint32_t node = 0;
  bool have = true;
  while (have) {
    if (shape.is_leaf(node)) {
      int64_t b, e;
      shape.range(node, b, e);
      for (int64_t r = b; r < e; ++r) {
        double d = sq_dist64<D>(v.rec + r * D, qq);
        int32_t id = v.perm[r];
        if (!(d < wd || (d == wd && id < wi))) continue;
#pragma unroll
        for (int j = 0; j < KC; ++j) {
          const bool lt = d < kd[j] || (d == kd[j] && id < ki[j]);
          const double td = kd[j];
          const int32_t ti = ki[j];
          kd[j] = lt ? d : td;
          ki[j] = lt ? id : ti;
          d = lt ? td : d;
          id = lt ? ti : id;
        }
#pragma unroll
        for (int j = 0; j < KC; ++j)
          if (j == k - 1) wd = kd[j], wi = ki[j];
      }
    } else {
      const uint32_t l = shape.left(node), r = l + 1;
      const double dl = box_min64<D>(v.box, l, qq), dr = box_min64<D>(v.box, r, qq);
      const uint32_t nearc = dl <= dr ? l : r, farc = dl <= dr ? r : l;
      const double dn = fmin(dl, dr), df = fmax(dl, dr);
      if (df <= wd) stk[(sp++) * kF64Block + threadIdx.x] = farc;
      if (dn <= wd) {
        node = nearc;
        continue;
      }
    }
    // pop the next node still within reach
    have = false;
    while (sp > 0) {
      const uint32_t c = stk[(--sp) * kF64Block + threadIdx.x];
      if (box_min64<D>(v.box, c, qq) <= wd) {
        node = c;
        have = true;
        break;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < KC; ++j)
    if (j < k) {
      const bool pad = ki[j] == INT_MAX;
      if (out_idx) out_idx[row * k + j] = pad ? -1 : ki[j];
      out_d2[row * k + j] = pad ? INFINITY : kd[j];
    }
}

// Closed-ball counts (FILL false) or lists (FILL true: the input indices of
// row `row` written from offsets[row] on, in traversal order).
template <int D, bool FILL, typename Shape>
__global__ __launch_bounds__(kF64Block) void k_range64(View64 v, const double* __restrict__ q,
                                                       int64_t nq, double r2,
                                                       const int32_t* __restrict__ order,
                                                       int32_t* __restrict__ count,
                                                       const int64_t* __restrict__ offsets,
                                                       int32_t* __restrict__ out, int depth) {
  extern __shared__ uint32_t stk[];
  const int64_t i = (int64_t)blockIdx.x * kF64Block + threadIdx.x;
  if (i >= nq) return;
  double qq[D];
  const int64_t row = load_query64<D>(v, q, order, i, qq);
  const Shape shape(shape_view(v));
  int64_t c = 0;
  int64_t at = FILL ? offsets[row] : 0;
  int sp = 0;
  stk[(sp++) * kF64Block + threadIdx.x] = 0;
  while (sp > 0) {
    const uint32_t node = stk[(--sp) * kF64Block + threadIdx.x];
    if (box_min64<D>(v.box, node, qq) > r2) continue;
    int64_t b, e;
    if (box_max64<D>(v.box, node, qq) <= r2) {
      shape.range(node, b, e);
      if (FILL)
        for (int64_t t = b; t < e; ++t) out[at++] = v.perm[t];
      c += e - b;
      continue;
    }
    if (shape.is_leaf(node)) {
      shape.range(node, b, e);
      for (int64_t t = b; t < e; ++t)
        if (sq_dist64<D>(v.rec + t * D, qq) <= r2) {
          if (FILL) out[at++] = v.perm[t];
          ++c;
        }
      continue;
    }
    const uint32_t l = shape.left(node);
    stk[(sp++) * kF64Block + threadIdx.x] = l + 1;
    stk[(sp++) * kF64Block + threadIdx.x] = l;
  }
  if (!FILL) count[row] = (int32_t)c;
}

__global__ void k_zero64(int32_t* p, int64_t* q) {
  if (p) *p = 0;
  if (q) *q = 0;
}

bool dim_ok64(int d) { return d == 2 || d == 3 || d == 4 || d == 8 || d == 16; }

template <typename F>
kdt_status by_dim(int d, F&& f) {
  switch (d) {
    case 2: return f(std::integral_constant<int, 2>());
    case 3: return f(std::integral_constant<int, 3>());
    case 4: return f(std::integral_constant<int, 4>());
    case 8: return f(std::integral_constant<int, 8>());
    case 16: return f(std::integral_constant<int, 16>());
  }
  return KDT_EUNSUPPORTED;
}

// Stack entries a traversal can hold: the depth-first kNN keeps one pending
// sibling per level, the ball traversal two children per level.
int stack_depth(const kdt_tree* t) { return 2 * (t->levels + 1) + 2; }

// The query order (Hilbert curve over the root box, d <= 4; tree leaf
// otherwise), taken from the float32 rounding of the queries.
kdt_status order64(const kdt_tree* t, const double* d_q, int64_t nq, PoolBuffers& buf,
                   int32_t** order, hipStream_t stream) {
  float* qf = nullptr;
  int32_t* bad = nullptr;
  int32_t* ord = nullptr;
  if (!buf.get(&qf, (size_t)nq * t->d) || !buf.get(&bad, 1) || !buf.get(&ord, (size_t)nq)) {
    kdt_set_error("float64 queries: device allocation failed for the query order");
    return KDT_ENOMEM;
  }
  const int64_t m = nq * t->d;
  k_to_f32<<<(unsigned)((m + 255) / 256), 256, 0, stream>>>(d_q, m, qf, bad);
  const kdt_status st = kdt_query_order(t, qf, nq, 0, ord, stream);
  if (st != KDT_OK) return st;
  *order = ord;
  return KDT_OK;
}

}  // namespace

}  // namespace kdt

using namespace kdt;

extern "C" kdt_status kdt_build_f64(const double* d_pts, int64_t n, int32_t d,
                                    const kdt_build_opts* opts, hipStream_t stream,
                                    kdt_tree** out) {
  kdt_clear_error();
  if (!out || !d_pts || n < 1 || n > INT32_MAX) {
    kdt_set_error("kdt_build_f64: NULL pointer or n=%lld outside [1, 2^31-1]", (long long)n);
    return KDT_EINVAL;
  }
  *out = nullptr;
  if (!dim_ok64(d)) {
    kdt_set_error("kdt_build_f64: dimension %d is not one of 2, 3, 4, 8, 16", d);
    return KDT_EUNSUPPORTED;
  }
  const bool check = opts ? opts->check_finite != 0 : true;
  PoolBuffers buf(stream);
  float* xf = nullptr;
  int32_t* bad = nullptr;
  if (!buf.get(&xf, (size_t)n * d) || !buf.get(&bad, 1)) {
    kdt_set_error("kdt_build_f64: device allocation failed (%lld points)", (long long)n);
    return KDT_ENOMEM;
  }
  k_zero64<<<1, 1, 0, stream>>>(bad, nullptr);
  const int64_t m = n * d;
  k_to_f32<<<(unsigned)((m + 255) / 256), 256, 0, stream>>>(d_pts, m, xf, bad);
  if (check) {
    int32_t h = 0;
    if (hipMemcpyAsync(&h, bad, sizeof(h), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
      kdt_set_error("kdt_build_f64: reading the finiteness flag failed");
      return KDT_EDEVICE;
    }
    if (h) {
      kdt_set_error("kdt_build_f64: non-finite coordinate (NaN or Inf)");
      return KDT_EINVAL;
    }
  }
  kdt_build_opts o{};
  if (opts) o = *opts;
  o.check_finite = 0;  // the float32 copy is finite by construction
  kdt_tree* t = nullptr;
  kdt_status st = kdt_build(xf, n, d, &o, stream, &t);
  if (st != KDT_OK) return st;
  const size_t b_rec = sizeof(double) * (size_t)n * d;
  const size_t b_box = sizeof(double) * (size_t)t->n_nodes * 2 * d;
  void* block = nullptr;
  if (dev_alloc(&block, ((b_rec + 255) & ~size_t(255)) + b_box, stream) != hipSuccess) {
    kdt_free(t);
    kdt_set_error("kdt_build_f64: cannot allocate the float64 tree (%lld points)", (long long)n);
    return KDT_ENOMEM;
  }
  t->f64_block = block;
  t->rec64 = static_cast<double*>(block);
  t->box64 = reinterpret_cast<double*>(static_cast<char*>(block) + ((b_rec + 255) & ~size_t(255)));
  const View64 v = view64(t);
  st = by_dim(d, [&](auto dd) -> kdt_status {
    constexpr int D = decltype(dd)::value;
    k_gather64<D><<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(d_pts, t->perm, n, t->rec64);
    const unsigned gn = (unsigned)((t->n_nodes + 255) / 256);
    if (t->nodes) {
      k_leaf_boxes64<D, StoredShape><<<gn, 256, 0, stream>>>(v, t->n_nodes, t->box64);
      for (int l = t->levels - 1; l >= 0; --l)
        k_inner_boxes64<D, StoredShape><<<gn, 256, 0, stream>>>(v, 0, t->n_nodes, l, t->box64);
    } else {
      k_leaf_boxes64<D, MedianShape><<<gn, 256, 0, stream>>>(v, t->n_nodes, t->box64);
      for (int l = t->levels - 1; l >= 0; --l) {
        const int64_t first = (int64_t(1) << l) - 1, count = int64_t(1) << l;
        k_inner_boxes64<D, MedianShape><<<(unsigned)((count + 255) / 256), 256, 0, stream>>>(
            v, first, count, l, t->box64);
      }
    }
    return hipGetLastError() == hipSuccess ? KDT_OK : KDT_EDEVICE;
  });
  if (st != KDT_OK) {
    kdt_free(t);
    kdt_set_error("kdt_build_f64: kernel launch failed");
    return st;
  }
  *out = t;
  return KDT_OK;
}

extern "C" kdt_status kdt_knn_f64(const kdt_tree* tree, const double* d_q, int64_t nq, int32_t k,
                                  int32_t* d_idx, double* d_d2, const kdt_query_opts* opts,
                                  hipStream_t stream) {
  kdt_clear_error();
  if (tree && tree->rec64 && nq == 0 && k >= 1 && k <= KDT_MAX_K) return KDT_OK;
  if (!tree || !tree->rec64 || !d_d2 || nq < 0 || nq > INT32_MAX) {
    kdt_set_error("kdt_knn_f64: NULL tree or output, a tree not built by kdt_build_f64, or nq "
                  "outside [0, 2^31-1]");
    return KDT_EINVAL;
  }
  if (k < 1) {
    kdt_set_error("kdt_knn_f64: k=%d below 1", k);
    return KDT_EINVAL;
  }
  if (k > KDT_MAX_K) {
    kdt_set_error("kdt_knn_f64: k=%d above %d", k, KDT_MAX_K);
    return KDT_EUNSUPPORTED;
  }
  if (opts && opts->period) {
    kdt_set_error("kdt_knn_f64: periodic boundaries are not available for float64 coordinates");
    return KDT_EUNSUPPORTED;
  }
  if (!d_q && nq != tree->n) {
    kdt_set_error("kdt_knn_f64: self queries need nq == n (%lld)", (long long)tree->n);
    return KDT_EINVAL;
  }
  const int32_t* rows = nullptr;
  const kdt_status rs = self_rows(tree, d_q, opts, "kdt_knn_f64", &rows);
  if (rs != KDT_OK) return rs;
  PoolBuffers buf(stream);
  // self queries: the tree-order row marker (or NULL)
  const int32_t* order = d_q ? (opts ? opts->order : nullptr) : rows;
  int32_t* own = nullptr;
  if (d_q && !order && (!opts || opts->sort_queries) && nq > 1) {
    const kdt_status st = order64(tree, d_q, nq, buf, &own, stream);
    if (st != KDT_OK) return st;
    order = own;
  }
  const View64 v = view64(tree);
  const int depth = stack_depth(tree);
  const size_t smem = sizeof(uint32_t) * (size_t)depth * kF64Block;
  const unsigned g = (unsigned)((nq + kF64Block - 1) / kF64Block);
  const kdt_status st = by_dim(tree->d, [&](auto dd) -> kdt_status {
    constexpr int D = decltype(dd)::value;
    auto go = [&](auto kc) {
      constexpr int KC = decltype(kc)::value;
      if (tree->nodes)
        k_knn64<D, KC, StoredShape><<<g, kF64Block, smem, stream>>>(
            v, d_q, nq, k, order, d_idx, d_d2, depth);
      else
        k_knn64<D, KC, MedianShape><<<g, kF64Block, smem, stream>>>(
            v, d_q, nq, k, order, d_idx, d_d2, depth);
    };
    if (k <= 8)
      go(std::integral_constant<int, 8>());
    else if (k <= 16)
      go(std::integral_constant<int, 16>());
    else if (k <= 32)
      go(std::integral_constant<int, 32>());
    else
      go(std::integral_constant<int, 64>());
    return hipGetLastError() == hipSuccess ? KDT_OK : KDT_EDEVICE;
  });
  if (st != KDT_OK) kdt_set_error("kdt_knn_f64: kernel launch failed");
  return st;
}

extern "C" kdt_status kdt_range_f64(const kdt_tree* tree, const double* d_q, int64_t nq, double r,
                                    int32_t* d_count, int64_t* d_offsets, int32_t* d_idx,
                                    int64_t capacity, int64_t* required,
                                    const kdt_query_opts* opts, hipStream_t stream) {
  kdt_clear_error();
  if (tree && tree->rec64 && nq == 0 && r >= 0.0 && capacity >= 0) {
    if (required) *required = 0;
    if (d_offsets) k_zero64<<<1, 1, 0, stream>>>(nullptr, d_offsets);
    return hipGetLastError() == hipSuccess ? KDT_OK : KDT_EDEVICE;
  }
  if (!tree || !tree->rec64 || !d_count || nq < 0 || nq > INT32_MAX || !(r >= 0.0) ||
      capacity < 0 || (d_idx && !d_offsets)) {
    kdt_set_error("kdt_range_f64: NULL tree or counts, a tree not built by kdt_build_f64, nq "
                  "outside [0, 2^31-1], r not >= 0, negative capacity or lists without offsets");
    return KDT_EINVAL;
  }
  if (opts && opts->period) {
    kdt_set_error("kdt_range_f64: periodic boundaries are not available for float64 coordinates");
    return KDT_EUNSUPPORTED;
  }
  if (!d_q && nq != tree->n) {
    kdt_set_error("kdt_range_f64: self queries need nq == n (%lld)", (long long)tree->n);
    return KDT_EINVAL;
  }
  const int32_t* rows = nullptr;
  const kdt_status rs = self_rows(tree, d_q, opts, "kdt_range_f64", &rows);
  if (rs != KDT_OK) return rs;
  if (required) *required = 0;
  PoolBuffers buf(stream);
  const int32_t* order = opts ? opts->order : nullptr;
  int32_t* own = nullptr;
  if (d_q && !order && (!opts || opts->sort_queries) && nq > 1) {
    const kdt_status st = order64(tree, d_q, nq, buf, &own, stream);
    if (st != KDT_OK) return st;
    order = own;
  }
  if (!d_q) order = rows;  // self queries: the tree-order row marker (or NULL)
  const View64 v = view64(tree);
  const double r2 = r * r;
  const int depth = stack_depth(tree);
  const size_t smem = sizeof(uint32_t) * (size_t)depth * kF64Block;
  const unsigned g = (unsigned)((nq + kF64Block - 1) / kF64Block);
  auto launch = [&](bool fill, int32_t* out) {
    return by_dim(tree->d, [&](auto dd) -> kdt_status {
      constexpr int D = decltype(dd)::value;
      if (tree->nodes) {
        if (fill)
          k_range64<D, true, StoredShape><<<g, kF64Block, smem, stream>>>(
              v, d_q, nq, r2, order, d_count, d_offsets, out, depth);
        else
          k_range64<D, false, StoredShape><<<g, kF64Block, smem, stream>>>(
              v, d_q, nq, r2, order, d_count, d_offsets, out, depth);
      } else {
        if (fill)
          k_range64<D, true, MedianShape><<<g, kF64Block, smem, stream>>>(
              v, d_q, nq, r2, order, d_count, d_offsets, out, depth);
        else
          k_range64<D, false, MedianShape><<<g, kF64Block, smem, stream>>>(
              v, d_q, nq, r2, order, d_count, d_offsets, out, depth);
      }
      return hipGetLastError() == hipSuccess ? KDT_OK : KDT_EDEVICE;
    });
  };
  kdt_status st = launch(false, nullptr);
  if (st != KDT_OK) {
    kdt_set_error("kdt_range_f64: kernel launch failed");
    return st;
  }
  if (!d_offsets) return KDT_OK;
  // offsets: exclusive running sum of the counts, then the total
  void* tmp = nullptr;
  if (!buf.get((char**)&tmp, scan_scratch_bytes(nq))) {
    kdt_set_error("kdt_range_f64: device allocation failed for the list offsets");
    return KDT_ENOMEM;
  }
  if (exclusive_scan<int64_t>(d_count, d_offsets, nq, d_offsets + nq, tmp, stream) != KDT_OK) {
    kdt_set_error("kdt_range_f64: offset scan failed");
    return KDT_EDEVICE;
  }
  int64_t total = 0;
  if (hipMemcpyAsync(&total, d_offsets + nq, sizeof(total), hipMemcpyDeviceToHost, stream) !=
          hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    kdt_set_error("kdt_range_f64: reading the list size failed");
    return KDT_EDEVICE;
  }
  if (required) *required = total;
  if (!d_idx) return KDT_OK;
  if (total > capacity) {
    kdt_set_error("kdt_range_f64: the lists need %lld entries, capacity is %lld",
                  (long long)total, (long long)capacity);
    return KDT_ECAPACITY;
  }
  if (total == 0) return KDT_OK;
  int32_t* unsorted = nullptr;
  if (!buf.get(&unsorted, (size_t)total)) {
    kdt_set_error("kdt_range_f64: device allocation failed for the lists");
    return KDT_ENOMEM;
  }
  st = launch(true, unsorted);
  if (st != KDT_OK) {
    kdt_set_error("kdt_range_f64: kernel launch failed");
    return st;
  }
  // every row ascending by input index
  st = sort_list_rows(unsorted, d_idx, d_offsets, nq, total, tree->n, stream);
  if (st != KDT_OK) return st;
  // the scratch goes back to the pool in stream order; the caller's arrays
  // are complete when the stream reaches this point
  return KDT_OK;
}
