// kdt_torus.hip -- kNN and ball queries on the D-torus: the periodic boundary
// conditions of Sec. 2.1 (the metric replaced by that of a D-toroid) and
// Sec. 2.4 (a compile-time option there, a template here), on gfx950.
//
// Every coordinate lies in [0, L_a).  Along each axis the distance goes the
// shorter way round, min(|x - q|, L - |x - q|), squared and summed in axis
// order in float32 without contraction, so results are exact against the
// oracle's definition.  The tree is the ordinary one: a node is skipped when
// even the shorter way round to its box is too far, and a node counts whole
// for a ball when its open-space farthest corner is inside (the torus
// distance never exceeds the open one).  kNN and ball lists take one
// traversal per lane; ball counts the wave-shared count traversal with a
// torus ball as its query shape (trees with leaves of at most 64 points).
// Also friends-of-friends groups on the torus (kdt_fof_torus).
#include <hip/hip_runtime.h>

#include <cmath>

#include "kdt_torus.h"

namespace kdt {

constexpr int kTBlock = 128;

// One query per lane: the tree's own points (q == NULL; row = input index,
// or s -- tree order -- when order is set) or q[order[s]] (q[s] without an
// order).
template <int D>
__device__ __forceinline__ int64_t torus_query(const TreeView& t, const float* __restrict__ q,
                                               const int32_t* __restrict__ order, int64_t s,
                                               float p[D]) {
  if (q == nullptr) {
    int32_t id = 0;
    load_rec<D>(t.rec, s, p, id);
    return order ? s : id;
  }
  const int64_t row = order ? order[s] : s;
#pragma unroll
  for (int a = 0; a < D; ++a) p[a] = q[row * D + a];
  return row;
}

template <int D, int KC, bool KTH>
__global__ __launch_bounds__(kTBlock) void k_torus_knn(TreeView t, const float* __restrict__ q,
                                                       int64_t nq, int k,
                                                       const int32_t* __restrict__ order,
                                                       Torus<D> T, int mode,
                                                       int32_t* __restrict__ oidx,
                                                       float* __restrict__ od2) {
  extern __shared__ uint32_t torus_stk[];
  const int64_t s = xcd_block<kXcdRunLane>() * kTBlock + threadIdx.x;
  if (s >= nq) return;
  float p[D];
  const int64_t row = torus_query<D>(t, q, order, s, p);
  if constexpr (KTH) {
    TopD<KC> best;
    best.init(k);
    knn_one<D>(t, p, best, torus_stk + threadIdx.x, kTBlock, TorusMetric<D>{T});
    knn_write_kth<KC>(best, mode, row, od2);
  } else {
    TopK<KC> best;
    best.init(k);
    knn_one<D>(t, p, best, torus_stk + threadIdx.x, kTBlock, TorusMetric<D>{T});
    knn_write<KC>(best, k, mode, row, oidx, od2);
  }
}

// Closed torus balls: counts (FILL = false) or the input indices of the
// points inside, from offsets[row] on (FILL = true).  Both children are
// pushed: at most levels + 2 stack entries.
template <int D, bool FILL>
__global__ __launch_bounds__(kTBlock) void k_torus_range(TreeView t, const float* __restrict__ q,
                                                         int64_t nq, float r2,
                                                         const int32_t* __restrict__ order,
                                                         Torus<D> T, int32_t* __restrict__ count,
                                                         const int64_t* __restrict__ offsets,
                                                         int32_t* __restrict__ out) {
  extern __shared__ uint32_t torus_col[];
  uint32_t* col = torus_col + threadIdx.x;
  const int64_t s = xcd_block<kXcdRunLane>() * kTBlock + threadIdx.x;
  if (s >= nq) return;
  float p[D];
  const int64_t row = torus_query<D>(t, q, order, s, p);
  const uint32_t first_leaf = (1u << t.levels) - 1u;
  int64_t c = 0;
  int64_t pos = FILL ? offsets[row] : 0;
  int sp = 0;
  col[kTBlock * sp++] = 0;
  while (sp > 0) {
    const uint32_t node = col[kTBlock * --sp];
    float lo[D], hi[D];
    load_box<D>(t.box, node, lo, hi);
    if (torus_box_mindist<D>(lo, hi, p, T) > r2) continue;
    const int lev = node_level(node);
    const int64_t j = (int64_t)node - ((int64_t(1) << lev) - 1);
    const int64_t b = node_begin(t.n, lev, j), e = node_begin(t.n, lev, j + 1);
    const bool whole = box_maxdist<D>(lo, hi, p) <= r2;
    if (whole || node >= first_leaf) {
      if (whole && !FILL) {
        c += e - b;
        continue;
      }
      for (int64_t i = b; i < e; ++i) {
        float x[D];
        int32_t id = 0;
        load_rec<D>(t.rec, i, x, id);
        if (whole || torus_sq_dist<D>(x, p, T) <= r2) {
          if (FILL) out[pos++] = id;
          ++c;
        }
      }
      continue;
    }
    col[kTBlock * sp++] = 2 * node + 2;
    col[kTBlock * sp++] = 2 * node + 1;
  }
  if (!FILL) count[row] = (int32_t)c;
}

// flag[0] <- 1 if some query coordinate lies outside [0, L_a).
template <int D>
__global__ void k_torus_check(const float* __restrict__ q, int64_t nq, Torus<D> T,
                              int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  bool bad = false;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float v = q[i * D + a];
    bad |= !(v >= 0.0f && v < T.L[a]);
  }
  if (bad) flag[0] = 1;
}

__global__ void k_torus_flag_clear(int32_t* flag) { flag[0] = 0; }

// Periods finite and positive, every tree point (its root box) and every
// query inside [0, L).  Waits on the stream.
template <int D>
static kdt_status torus_setup(const kdt_tree* tr, const float* d_q, int64_t nq,
                              const float* period, PoolBuffers& buf, Torus<D>* T,
                              hipStream_t stream, const char* who) {
  for (int a = 0; a < D; ++a) {
    if (!(period[a] > 0.0f) || !std::isfinite(period[a])) {
      kdt_set_error("%s: period %d is not finite and > 0", who, a);
      return KDT_EINVAL;
    }
    T->L[a] = period[a];
  }
  float root[2 * pad4(D)];
  int32_t bad = 0;
  int32_t* flag = nullptr;
  if (d_q && !buf.get(&flag, 1)) {
    kdt_set_error("%s: device allocation failed for the period check", who);
    return KDT_ENOMEM;
  }
  if (d_q) {
    k_torus_flag_clear<<<1, 1, 0, stream>>>(flag);
    k_torus_check<D><<<(unsigned)((nq + 255) / 256), 256, 0, stream>>>(d_q, nq, *T, flag);
  }
  if (hipMemcpyAsync(root, tr->box, sizeof(root), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      (d_q && hipMemcpyAsync(&bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, stream) !=
                  hipSuccess) ||
      hipStreamSynchronize(stream) != hipSuccess) {
    kdt_set_error("%s: reading the period check failed", who);
    return KDT_EDEVICE;
  }
  for (int a = 0; a < D; ++a)
    if (!(root[a] >= 0.0f && root[pad4(D) + a] < T->L[a])) {
      kdt_set_error("%s: tree points outside [0, period) on axis %d", who, a);
      return KDT_EINVAL;
    }
  if (bad) {
    kdt_set_error("%s: a query lies outside [0, period)", who);
    return KDT_EINVAL;
  }
  return KDT_OK;
}

template <int D>
static kdt_status torus_knn_impl(const kdt_tree* tr, const float* d_q, int64_t nq, int k,
                                 int32_t* d_idx, float* d_d2, int mode, bool sort_q,
                                 const int32_t* given, const float* period, hipStream_t stream) {
  PoolBuffers buf(stream);
  Torus<D> T;
  kdt_status st = torus_setup<D>(tr, d_q, nq, period, buf, &T, stream, "kdt_knn");
  if (st != KDT_OK) return st;
  TreeView v;
  v.rec = tr->rec;
  v.box = tr->box;
  v.n = tr->n;
  v.levels = tr->levels;
  const int32_t* order = given;
  if (d_q && !given && sort_q && nq > 1) {
    int32_t* own = nullptr;
    if (!buf.get(&own, (size_t)nq)) {
      kdt_set_error("kdt_knn: device allocation failed for the query order");
      return KDT_ENOMEM;
    }
    st = kdt_query_order(tr, d_q, nq, 0, own, stream);
    if (st != KDT_OK) return st;
    order = own;
  }
  if (!d_q) order = given;  // self queries: the tree-order row marker (or NULL)
  const unsigned grid = (unsigned)((nq + kTBlock - 1) / kTBlock);
  const size_t smem = sizeof(uint32_t) * (size_t)(tr->levels + 1) * kTBlock;
#define KDT_TORUS(KC)                                                                          \
  if (mode == 0)                                                                               \
    k_torus_knn<D, KC, false><<<grid, kTBlock, smem, stream>>>(v, d_q, nq, k, order, T, mode, \
                                                               d_idx, d_d2);                   \
  else                                                                                         \
    k_torus_knn<D, KC, true><<<grid, kTBlock, smem, stream>>>(v, d_q, nq, k, order, T, mode,  \
                                                              d_idx, d_d2);
  if (k <= 8) {
    KDT_TORUS(8)
  } else if (k <= 16) {
    KDT_TORUS(16)
  } else if (k <= 32) {
    KDT_TORUS(32)
  } else {
    KDT_TORUS(64)
  }
#undef KDT_TORUS
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_knn: torus kernel launch failed");
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

template <int D>
static kdt_status torus_range_impl(const kdt_tree* tr, const float* d_q, int64_t nq, float r,
                                   int32_t* d_count, int64_t* d_off, int32_t* d_idx,
                                   int64_t capacity, int64_t* required, bool sort_q,
                                   const int32_t* given, const float* period,
                                   bool counts_given, hipStream_t stream) {
  PoolBuffers buf(stream);
  Torus<D> T;
  kdt_status st = torus_setup<D>(tr, d_q, nq, period, buf, &T, stream, "kdt_range");
  if (st != KDT_OK) return st;
  TreeView v;
  v.rec = tr->rec;
  v.box = tr->box;
  v.n = tr->n;
  v.levels = tr->levels;
  const int32_t* order = given;
  if (d_q && !given && sort_q && nq > 1) {
    int32_t* own = nullptr;
    if (!buf.get(&own, (size_t)nq)) {
      kdt_set_error("kdt_range: device allocation failed for the query order");
      return KDT_ENOMEM;
    }
    st = kdt_query_order(tr, d_q, nq, 0, own, stream);
    if (st != KDT_OK) return st;
    order = own;
  }
  if (!d_q) order = given;  // self queries: the tree-order row marker (or NULL)
  const float r2 = r * r;
  const unsigned grid = (unsigned)((nq + kTBlock - 1) / kTBlock);
  const size_t smem = sizeof(uint32_t) * (size_t)(tr->levels + 2) * kTBlock;
  if (counts_given) {
    // the counts and offsets of the sizing call are in d_count and d_off
  } else if (tr->leaf <= 64) {
    int cap = 0;
    const TreeView vc = count_view(v, tr->leaf, &cap);
    st = torus_range_packet_launch<D>(vc, cap, d_q, nq, r2, T, order, d_count, 0u, stream);
    if (st != KDT_OK) return st;
  } else {
    k_torus_range<D, false><<<grid, kTBlock, smem, stream>>>(v, d_q, nq, r2, order, T, d_count,
                                                              nullptr, nullptr);
  }
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_range: torus count kernel launch failed");
    return KDT_EDEVICE;
  }
  if (!d_off) return KDT_OK;
  void* tmp = nullptr;
  if (!counts_given && !buf.get((char**)&tmp, scan_scratch_bytes(nq))) {
    kdt_set_error("kdt_range: device allocation failed for the list offsets");
    return KDT_ENOMEM;
  }
  if (!counts_given &&
      exclusive_scan<int64_t>(d_count, d_off, nq, d_off + nq, tmp, stream) != KDT_OK) {
    kdt_set_error("kdt_range: torus offset scan failed");
    return KDT_EDEVICE;
  }
  int64_t total = 0;
  if (hipMemcpyAsync(&total, d_off + nq, sizeof(int64_t), hipMemcpyDeviceToHost, stream) !=
          hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    kdt_set_error("kdt_range: reading the list size failed");
    return KDT_EDEVICE;
  }
  if (required) *required = total;
  if (!d_idx || total == 0) return KDT_OK;
  if (total > capacity) {
    kdt_set_error("list capacity %lld is below the %lld entries needed", (long long)capacity,
                  (long long)total);
    return KDT_ECAPACITY;
  }
  if (total > INT32_MAX) {
    kdt_set_error("lists above 2^31-1 entries are not supported");
    return KDT_EUNSUPPORTED;
  }
  int32_t* unsorted = nullptr;
  if (!buf.get(&unsorted, (size_t)total)) {
    kdt_set_error("device allocation failed for the lists");
    return KDT_ENOMEM;
  }
  if (tr->leaf <= 64) {
    // the wave-shared traversal of the counts, writing the lists
    int32_t* cur = nullptr;
    if (!buf.get(&cur, (size_t)nq)) {
      kdt_set_error("device allocation failed for the list cursors");
      return KDT_ENOMEM;
    }
    const FillOut fo{unsorted, d_off, cur};
    int cap = 0;
    const TreeView vc = count_view(v, tr->leaf, &cap);
    st = torus_range_packet_launch<D>(vc, cap, d_q, nq, r2, T, order, d_count, 0u, stream,
                                      &fo);
    if (st != KDT_OK) return st;
  } else {
    k_torus_range<D, true><<<grid, kTBlock, smem, stream>>>(v, d_q, nq, r2, order, T, d_count,
                                                             d_off, unsorted);
  }
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_range: torus list kernel launch failed");
    return KDT_EDEVICE;
  }
  return sort_list_rows(unsorted, d_idx, d_off, nq, total, tr->n, stream);
}

// Friends-of-friends on the torus (Sec. 4.1 with the periodic metric).
//
// A node whose open-space box diagonal is at most l is a clique: every two of
// its points are friends (the torus distance never exceeds the open one, and
// the rounded diagonal bounds every rounded pair distance).  First every
// point joins the first point of the highest clique node above it; then one
// lane per point in tree order searches its ball of radius l and links
// friends at later tree positions (nodes ending at or before its own are not
// entered: the other end of each such pair links it).  Inside a clique node,
// already one component, one friend suffices: the whole node when it lies in
// the ball, else the first friend found.  The union-find is the lock-free one
// of the open grouping, whose roots are the smallest input indices.  Trees
// with leaves of at most 64 points link through the wave-shared grouping
// traversal instead (the open grouping's, with the torus metric), which
// also takes one link per clique node and flags nodes it joined whole.
template <int D>
__global__ void k_torus_clique_mark(const float* __restrict__ box, int64_t n_nodes, float l2,
                                    uint32_t* __restrict__ clique) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_nodes) return;
  float lo[D], hi[D];
  load_box<D>(box, (uint32_t)v, lo, hi);
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float g = hi[a] - lo[a];
    const float g2 = g * g;
    s = s + g2;
  }
  clique[v] = s <= l2 ? 1 : 0;
}

template <int D>
__global__ void k_torus_clique_join(TreeView t, const uint32_t* __restrict__ clique,
                                    int32_t* __restrict__ parent) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= t.n) return;
  int64_t j = 0;
  for (int lev = 0; lev <= t.levels; ++lev) {
    const uint32_t node = (uint32_t)(((int64_t(1) << lev) - 1) + j);
    if (clique[node]) {
      const int64_t b = node_begin(t.n, lev, j);
      if (b != i) {
        constexpr int S = rec_stride(D);
        const int32_t me = __float_as_int(t.rec[i * S + D]);
        const int32_t first = __float_as_int(t.rec[b * S + D]);
        uf_union(parent, me, first);
      }
      return;
    }
    if (lev < t.levels) j = i >= node_begin(t.n, lev + 1, 2 * j + 1) ? 2 * j + 1 : 2 * j;
  }
}

// Both children are pushed: at most levels + 2 stack entries.
template <int D>
__global__ __launch_bounds__(kTBlock) void k_torus_fof_link(TreeView t, float l2, Torus<D> T,
                                                            const uint32_t* __restrict__ clique,
                                                            int32_t* __restrict__ parent) {
  extern __shared__ uint32_t torus_fcol[];
  uint32_t* col = torus_fcol + threadIdx.x;
  const int64_t s = xcd_block<kXcdRunFof>() * kTBlock + threadIdx.x;
  if (s >= t.n) return;
  float p[D];
  int32_t me = 0;
  load_rec<D>(t.rec, s, p, me);
  const uint32_t first_leaf = (1u << t.levels) - 1u;
  int sp = 0;
  col[kTBlock * sp++] = 0;
  while (sp > 0) {
    const uint32_t node = col[kTBlock * --sp];
    const int lev = node_level(node);
    const int64_t j = (int64_t)node - ((int64_t(1) << lev) - 1);
    const int64_t b = node_begin(t.n, lev, j), e = node_begin(t.n, lev, j + 1);
    if (e <= s + 1) continue;  // every point at or before this one
    float lo[D], hi[D];
    load_box<D>(t.box, node, lo, hi);
    if (torus_box_mindist<D>(lo, hi, p, T) > l2) continue;
    const bool whole = box_maxdist<D>(lo, hi, p) <= l2;
    const bool one = clique[node] != 0;  // one component already
    if (whole || one || node >= first_leaf) {
      for (int64_t i = b > s ? b : s + 1; i < e; ++i) {
        float x[D];
        int32_t id = 0;
        load_rec<D>(t.rec, i, x, id);
        if (whole || torus_sq_dist<D>(x, p, T) <= l2) {
          uf_union(parent, me, id);
          if (one) break;
        }
      }
      continue;
    }
    col[kTBlock * sp++] = 2 * node + 2;
    col[kTBlock * sp++] = 2 * node + 1;
  }
}

__global__ void k_torus_fof_init(int32_t* __restrict__ parent, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) parent[i] = (int32_t)i;
}

// Every element pointed at its root (written by its own lane only).
__global__ void k_torus_fof_final(int32_t* __restrict__ parent, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) uf_st(parent + i, uf_root(parent, (int32_t)i));
}

template <int D>
static kdt_status torus_fof_impl(const kdt_tree* tr, float l, const float* period,
                                 int32_t* d_labels, int64_t* n_groups, hipStream_t stream) {
  PoolBuffers buf(stream);
  Torus<D> T;
  kdt_status st = torus_setup<D>(tr, nullptr, 0, period, buf, &T, stream, "kdt_fof_torus");
  if (st != KDT_OK) return st;
  TreeView v;
  v.rec = tr->rec;
  v.box = tr->box;
  v.n = tr->n;
  v.levels = tr->levels;
  const int64_t n = tr->n;
  const unsigned g = (unsigned)((n + 255) / 256);
  uint32_t* clique = nullptr;
  if (!buf.get(&clique, (size_t)tr->n_nodes)) {
    kdt_set_error("kdt_fof_torus: device allocation failed");
    return KDT_ENOMEM;
  }
  const float l2 = l * l;
  k_torus_fof_init<<<g, 256, 0, stream>>>(d_labels, n);
  k_torus_clique_mark<D><<<(unsigned)((tr->n_nodes + 255) / 256), 256, 0, stream>>>(
      tr->box, tr->n_nodes, l2, clique);
  k_torus_clique_join<D><<<g, 256, 0, stream>>>(v, clique, d_labels);
  if (tr->leaf <= 64) {
    st = torus_fof_packet_launch<D>(v, tr->leaf, l2, T, d_labels, clique, stream);
    if (st != KDT_OK) return st;
  } else {
    const size_t smem = sizeof(uint32_t) * (size_t)(tr->levels + 2) * kTBlock;
    k_torus_fof_link<D><<<(unsigned)((n + kTBlock - 1) / kTBlock), kTBlock, smem, stream>>>(
        v, l2, T, clique, d_labels);
  }
  k_torus_fof_final<<<g, 256, 0, stream>>>(d_labels, n);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_fof_torus: kernel launch failed");
    return KDT_EDEVICE;
  }
  if (!n_groups) return KDT_OK;
  int64_t* d_out = nullptr;
  char* tmp = nullptr;
  int64_t h = 0;
  if (!buf.get(&d_out, 1) || !buf.get(&tmp, scan_scratch_bytes(n))) {
    kdt_set_error("kdt_fof_torus: device allocation failed");
    return KDT_ENOMEM;
  }
  if (count_roots(d_labels, n, d_out, tmp, stream) != KDT_OK ||
      hipMemcpyAsync(&h, d_out, sizeof(h), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    kdt_set_error("kdt_fof_torus: counting groups failed");
    return KDT_EDEVICE;
  }
  *n_groups = h;
  return KDT_OK;
}

kdt_status knn_torus(const kdt_tree* tr, const float* d_q, int64_t nq, int k, int32_t* d_idx,
                     float* d_d2, int mode, bool sort_q, const int32_t* given,
                     const float* period, hipStream_t stream) {
  switch (tr->d) {
    case 2: return torus_knn_impl<2>(tr, d_q, nq, k, d_idx, d_d2, mode, sort_q, given, period, stream);
    case 3: return torus_knn_impl<3>(tr, d_q, nq, k, d_idx, d_d2, mode, sort_q, given, period, stream);
    case 4: return torus_knn_impl<4>(tr, d_q, nq, k, d_idx, d_d2, mode, sort_q, given, period, stream);
    case 8: return torus_knn_impl<8>(tr, d_q, nq, k, d_idx, d_d2, mode, sort_q, given, period, stream);
    case 16: return torus_knn_impl<16>(tr, d_q, nq, k, d_idx, d_d2, mode, sort_q, given, period, stream);
  }
  kdt_set_error("kdt_knn: unsupported dimension %d", tr->d);
  return KDT_EUNSUPPORTED;
}

kdt_status range_torus(const kdt_tree* tr, const float* d_q, int64_t nq, float r,
                       int32_t* d_count, int64_t* d_off, int32_t* d_idx, int64_t capacity,
                       int64_t* required, bool sort_q, const int32_t* given, const float* period,
                       bool counts_given, hipStream_t stream) {
  switch (tr->d) {
    case 2: return torus_range_impl<2>(tr, d_q, nq, r, d_count, d_off, d_idx, capacity, required, sort_q, given, period, counts_given, stream);
    case 3: return torus_range_impl<3>(tr, d_q, nq, r, d_count, d_off, d_idx, capacity, required, sort_q, given, period, counts_given, stream);
    case 4: return torus_range_impl<4>(tr, d_q, nq, r, d_count, d_off, d_idx, capacity, required, sort_q, given, period, counts_given, stream);
    case 8: return torus_range_impl<8>(tr, d_q, nq, r, d_count, d_off, d_idx, capacity, required, sort_q, given, period, counts_given, stream);
    case 16: return torus_range_impl<16>(tr, d_q, nq, r, d_count, d_off, d_idx, capacity, required, sort_q, given, period, counts_given, stream);
  }
  kdt_set_error("kdt_range: unsupported dimension %d", tr->d);
  return KDT_EUNSUPPORTED;
}

}  // namespace kdt

using namespace kdt;

extern "C" kdt_status kdt_fof_torus(const kdt_tree* tree, float l, const float* period,
                                    int32_t* d_labels, int64_t* n_groups, hipStream_t stream) {
  kdt_clear_error();
  if (refuse_stored(tree, "kdt_fof_torus") || refuse_f64(tree, "kdt_fof_torus"))
    return KDT_EUNSUPPORTED;
  if (!tree || !d_labels || !period || !(l >= 0.0f) || !std::isfinite(l)) {
    kdt_set_error("kdt_fof_torus: NULL tree, labels or period, or l not finite and >= 0");
    return KDT_EINVAL;
  }
  switch (tree->d) {
    case 2: return torus_fof_impl<2>(tree, l, period, d_labels, n_groups, stream);
    case 3: return torus_fof_impl<3>(tree, l, period, d_labels, n_groups, stream);
    case 4: return torus_fof_impl<4>(tree, l, period, d_labels, n_groups, stream);
    case 8: return torus_fof_impl<8>(tree, l, period, d_labels, n_groups, stream);
    case 16: return torus_fof_impl<16>(tree, l, period, d_labels, n_groups, stream);
  }
  kdt_set_error("kdt_fof_torus: unsupported dimension %d", tree->d);
  return KDT_EUNSUPPORTED;
}
