// kdt_query.hip -- batched kNN (Sec. 2.3, Algorithm 2) and ball queries
// (Algorithm 3) over a balanced k-d tree on gfx950.
//
// One lane per query.  The paper's best-first node queue is replaced by a
// depth-first stack that descends into the nearer child first and prunes a
// node when its box is farther than the current k-th candidate (strict '>').
// Candidates live in a sorted register list keyed by (d2, index), so the
// result -- the k smallest keys -- is exactly the one the best-first order
// gives.  Queries of one wave are made spatially coherent either by running
// in tree order (self queries) or by sorting external queries by the leaf
// they fall in.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kdt_query.h"

namespace kdt {

constexpr int kQBlock = 128;

// ---------------------------------------------------------------------------
// kNN
// ---------------------------------------------------------------------------

// The per-lane stack lives in LDS, (levels + 1) entries per lane (the tree
// depth bounds it: one pending sibling per level), sized at launch.  KTH:
// only the k-th distance is written (modes 1 and 2), kept in a TopD list.
template <int D, int KC, bool KTH, class Shape = MedianShape>
__global__ __launch_bounds__(kQBlock) void k_knn_lane(TreeView t, const float* __restrict__ q,
                                                      int64_t nq, int k,
                                                      const int32_t* __restrict__ order, int mode,
                                                      int32_t* __restrict__ oidx,
                                                      float* __restrict__ od2) {
  extern __shared__ uint32_t stk_dyn[];
  const int64_t s = xcd_block<kXcdRunLane>() * kQBlock + threadIdx.x;
  if (s >= nq) return;
  float p[D];
  int64_t row;
  if (q == nullptr) {
    // self queries: row = input index, or s (tree order) when order is set
    int32_t id = 0;
    load_rec<D>(t.rec, s, p, id);
    row = order ? s : id;
  } else {
    row = order ? order[s] : s;
#pragma unroll
    for (int a = 0; a < D; ++a) p[a] = q[row * D + a];
  }
  if constexpr (KTH) {
    TopD<KC> best;
    best.init(k);
    knn_one<D, TopD<KC>, OpenMetric<D>, Shape>(t, p, best, stk_dyn + threadIdx.x, kQBlock);
    knn_write_kth<KC>(best, mode, row, od2);
  } else {
    TopK<KC> best;
    best.init(k);
    knn_one<D, TopK<KC>, OpenMetric<D>, Shape>(t, p, best, stk_dyn + threadIdx.x, kQBlock);
    knn_write<KC>(best, k, mode, row, oidx, od2);
  }
}

// ---------------------------------------------------------------------------
// Ball queries: counts, then CSR lists
// ---------------------------------------------------------------------------

template <int D, bool FILL, class Shape = MedianShape>
__global__ __launch_bounds__(kQBlock) void k_range(TreeView t, const float* __restrict__ q,
                                                   int64_t nq, float r2,
                                                   const int32_t* __restrict__ order,
                                                   int32_t* __restrict__ count,
                                                   const int64_t* __restrict__ offsets,
                                                   int32_t* __restrict__ out) {
  extern __shared__ uint32_t stk_dyn32[];
  uint32_t* col = stk_dyn32 + threadIdx.x;
  const int64_t s = xcd_block<kXcdRunLane>() * kQBlock + threadIdx.x;
  if (s >= nq) return;
  float p[D];
  int64_t row;
  if (q == nullptr) {
    // self queries: row = input index, or s (tree order) when order is set
    int32_t id = 0;
    load_rec<D>(t.rec, s, p, id);
    row = order ? s : id;
  } else {
    row = order ? order[s] : s;
#pragma unroll
    for (int a = 0; a < D; ++a) p[a] = q[row * D + a];
  }
  const Shape sh(t);
  int64_t c = 0;
  int64_t pos = FILL ? offsets[row] : 0;
  int sp = 0;
  col[kQBlock * sp++] = 0;
  while (sp > 0) {
    const uint32_t node = col[kQBlock * --sp];
    float lo[D], hi[D];
    load_box<D>(t.box, node, lo, hi);
    if (box_mindist<D>(lo, hi, p) > r2) continue;
    int64_t b, e;
    sh.range(node, b, e);
    if (box_maxdist<D>(lo, hi, p) <= r2) {
      if (FILL) {
        for (int64_t i = b; i < e; ++i) {
          float x[D];
          int32_t id = 0;
          load_rec<D>(t.rec, i, x, id);
          out[pos++] = id;
        }
      }
      c += e - b;
      continue;
    }
    if (sh.is_leaf(node)) {
      for (int64_t i = b; i < e; ++i) {
        float x[D];
        int32_t id = 0;
        load_rec<D>(t.rec, i, x, id);
        if (sq_dist<D>(x, p) <= r2) {
          if (FILL) out[pos++] = id;
          ++c;
        }
      }
      continue;
    }
    const uint32_t c0 = sh.left(node);
    col[kQBlock * sp++] = c0 + 1;
    col[kQBlock * sp++] = c0;
  }
  if (!FILL) count[row] = (int32_t)c;
}

// ---------------------------------------------------------------------------
// Query ordering: a Hilbert key over the root box, or the leaf reached by
// descending towards the nearer child.
// ---------------------------------------------------------------------------

template <int D, class Shape = MedianShape>
__global__ void k_query_leaf(TreeView t, const float* __restrict__ q, int64_t nq,
                             uint32_t* __restrict__ key, int32_t* __restrict__ val) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nq) return;
  float p[D];
#pragma unroll
  for (int a = 0; a < D; ++a) p[a] = q[s * D + a];
  const Shape sh(t);
  uint32_t node = 0;
  while (!sh.is_leaf(node)) {
    const uint32_t c0 = sh.left(node);
    float lo[D], hi[D];
    load_box<D>(t.box, c0, lo, hi);
    const float d0 = box_mindist<D>(lo, hi, p);
    load_box<D>(t.box, c0 + 1, lo, hi);
    const float d1 = box_mindist<D>(lo, hi, p);
    node = d0 <= d1 ? c0 : c0 + 1;
  }
  key[s] = node;
  val[s] = (int32_t)s;
}

// Hilbert key of a query over the root box: B = 30 / D bits per axis
// (queries outside the box take the nearest cell), mapped to the Hilbert
// curve index with Skilling's transpose method (J. Skilling, "Programming
// the Hilbert curve", AIP Conf. Proc. 707, 2004): undo the excess work of
// the inverse transform level by level, Gray-encode, then read the index
// bits axis-interleaved from the top.  Consecutive keys are face-adjacent
// cells, so 64 consecutive queries occupy one compact region -- what a wave
// that shares one traversal needs -- and no tree walk is involved.
template <int D>
__global__ void k_query_hilbert(TreeView t, const float* __restrict__ q, int64_t nq,
                                uint32_t* __restrict__ key, int32_t* __restrict__ val) {
  constexpr int B = 30 / D;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nq) return;
  float lo[D], hi[D];
  load_box<D>(t.box, 0, lo, hi);
  uint32_t X[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float ext = hi[a] - lo[a];
    const float u = ext > 0.0f ? (q[s * D + a] - lo[a]) / ext * (float)(1u << B) : 0.0f;
    X[a] = u <= 0.0f ? 0u : (u >= (float)((1u << B) - 1) ? (1u << B) - 1 : (uint32_t)u);
  }
#pragma unroll
  for (uint32_t Q = 1u << (B - 1); Q > 1; Q >>= 1) {
    const uint32_t P = Q - 1;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        const uint32_t x = (X[0] ^ X[i]) & P;
        X[0] ^= x;
        X[i] ^= x;
      }
    }
  }
#pragma unroll
  for (int i = 1; i < D; ++i) X[i] ^= X[i - 1];
  uint32_t flip = 0;
#pragma unroll
  for (uint32_t Q = 1u << (B - 1); Q > 1; Q >>= 1)
    if (X[D - 1] & Q) flip ^= Q - 1;
  uint32_t k = 0;
#pragma unroll
  for (int b = B - 1; b >= 0; --b)
#pragma unroll
    for (int a = 0; a < D; ++a) k = (k << 1) | (((X[a] ^ flip) >> b) & 1u);
  key[s] = k;
  val[s] = (int32_t)s;
}


#define KDT_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      kdt_set_error("%s failed: %s", #call, hipGetErrorString(e_));          \
      return KDT_EDEVICE;                                                    \
    }                                                                        \
  } while (0)

static TreeView view_of(const kdt_tree* t) {
  TreeView v;
  v.rec = t->rec;
  v.box = t->box;
  v.n = t->n;
  v.levels = t->levels;
  v.nodes = t->nodes;
  v.visits = visit_counters();
  return v;
}

// Sorts external queries along the tree's space (a Hilbert key for D <= 4,
// else the leaf they fall in); returns the order array (caller frees with
// hipFreeAsync).
// kind 0: a Hilbert key over the root box for D <= 4 (cheap: no tree walk;
// what one traversal per lane and the ball counts use), else the tree leaf;
// kind 1: the tree leaf (a wave's queries then sit in one subtree; what the
// wave-packet kNN uses).  Ball counts on the clustered workload took 25.5 ms
// in leaf order against 48 ms in Hilbert order before heavy traversals were
// split over several launches; with that splitting Hilbert order is the
// faster one (3.3 against 4.1 ms, and its key costs 0.24 against 0.69 ms).
// Writes the permutation to `dst` if given, else to a new buffer *out.
// With a workspace `ws` (ws_bytes bytes of device memory), every buffer is
// carved from it -- nothing is allocated -- and *out points into it.
template <int D>
static kdt_status order_queries(const kdt_tree* t, const float* d_q, int64_t nq, int kind,
                                int32_t** out, hipStream_t stream, int32_t* dst = nullptr,
                                void* ws = nullptr, size_t ws_bytes = 0) {
  *out = nullptr;
  if (nq > INT32_MAX) {
    kdt_set_error("query reordering supports at most 2^31-1 queries");
    return KDT_EINVAL;
  }
  PoolBuffers buf(stream);
  uint32_t *k0 = nullptr, *k1 = nullptr;
  int32_t *v0 = nullptr, *v1 = nullptr;
  // up to 4 dimensions a Hilbert key over the root box; above, the leaf
  // reached by descending towards the nearer child
  const bool hilbert = D <= 4 && kind == 0;
  // leaf keys are node ids: below 2^(L+1) in a median tree, n_nodes in a stored one
  int node_bits = 1;
  while (node_bits < 31 && (int64_t(1) << node_bits) < t->n_nodes) ++node_bits;
  const int end_bit = hilbert ? (30 / D) * D : t->nodes ? node_bits : std::max(1, t->levels + 1);
  // The sort (kdt_sort.hip) ping-pongs between two key and two index arrays,
  // one pass per 8 key bits; the keys are written into the buffer that makes
  // the last pass land in the caller's array, so nothing is copied.
  const int passes = nq > 1 ? (end_bit + 7) / 8 : 0;
  const int last = passes & 1;
  const size_t tmp_bytes = radix_sort_scratch_bytes(nq);
  void* tmp = nullptr;
  if (ws) {
    const size_t a = ((size_t)nq * 4 + 255) / 256 * 256;  // one key or index array
    const size_t need = 4 * a + tmp_bytes;
    if (need > ws_bytes) {
      kdt_set_error("ordering %lld queries needs %zu bytes of scratch, %zu available",
                    (long long)nq, need, ws_bytes);
      return KDT_ECAPACITY;
    }
    char* w = static_cast<char*>(ws);
    k0 = reinterpret_cast<uint32_t*>(w);
    k1 = reinterpret_cast<uint32_t*>(w + a);
    v0 = reinterpret_cast<int32_t*>(w + 2 * a);
    v1 = reinterpret_cast<int32_t*>(w + 3 * a);
    tmp = w + 4 * a;
  } else if (!buf.get(&k0, (size_t)nq) || !buf.get(&k1, (size_t)nq) ||
             !buf.get(&v0, (size_t)nq) || (!dst && !buf.get(&v1, (size_t)nq)) ||
             !buf.get((char**)&tmp, tmp_bytes)) {
    kdt_set_error("device allocation failed for query ordering");
    return KDT_ENOMEM;
  }
  int32_t* vals[2] = {v0, v1};
  if (dst) vals[last] = dst, vals[last ^ 1] = v0;
  uint32_t* keys[2] = {k0, k1};
  if (hilbert)
    k_query_hilbert<D><<<(unsigned)((nq + 255) / 256), 256, 0, stream>>>(view_of(t), d_q, nq,
                                                                         keys[0], vals[0]);
  else if (t->nodes)
    k_query_leaf<D, StoredShape><<<(unsigned)((nq + 255) / 256), 256, 0, stream>>>(
        view_of(t), d_q, nq, keys[0], vals[0]);
  else
    k_query_leaf<D><<<(unsigned)((nq + 255) / 256), 256, 0, stream>>>(view_of(t), d_q, nq,
                                                                      keys[0], vals[0]);
  KDT_HIP(hipGetLastError());
  const int cur = radix_sort_pairs(keys, vals, nq, 0, end_bit, tmp, stream);
  KDT_HIP(hipGetLastError());
  int32_t* sorted = vals[cur];
  if (dst) return KDT_OK;  // the last pass wrote dst (vals[last])
  if (!ws) {
    // the other index array goes back to the pool; the sorted one is the caller's
    buf.keep(sorted);
  }
  *out = sorted;
  return KDT_OK;
}

template <int D>
static kdt_status knn_dispatch(const kdt_tree* t, const float* d_q, int64_t nq, int k,
                               int32_t* d_idx, float* d_d2, int mode, const int32_t* order,
                               hipStream_t stream) {
  TreeView v = view_of(t);
  // the k-th distance alone (smoothing lengths) reads the tree at 32-point
  // nodes, as the counts do, when k is above 16: 2^24 self queries at k = 32
  // took 19.0 ms on 16-point leaves, 18.6 ms on 32-point nodes of the same
  // tree; at k = 8 the tree's own 24-point leaves are faster (8.7 against
  // 9.9 ms)
  if (mode != 0 && !t->nodes && k > 16) {
    int cap = 0;
    v = count_view(v, t->leaf, &cap);
  }
  const unsigned grid = (unsigned)((nq + kQBlock - 1) / kQBlock);
  const size_t smem = sizeof(uint32_t) * (size_t)(t->levels + 1) * kQBlock;
#define KDT_LANE_S(KC, SH)                                                                    \
  if (mode == 0)                                                                              \
    k_knn_lane<D, KC, false, SH><<<grid, kQBlock, smem, stream>>>(v, d_q, nq, k, order, mode, \
                                                                  d_idx, d_d2);               \
  else                                                                                        \
    k_knn_lane<D, KC, true, SH><<<grid, kQBlock, smem, stream>>>(v, d_q, nq, k, order, mode,  \
                                                                 d_idx, d_d2);
#define KDT_LANE(KC)            \
  if (t->nodes) {               \
    KDT_LANE_S(KC, StoredShape) \
  } else {                      \
    KDT_LANE_S(KC, MedianShape) \
  }
  if (k <= 8) {
    KDT_LANE(8)
  } else if (k <= 16) {
    KDT_LANE(16)
  } else if (k <= 32) {
    KDT_LANE(32)
  } else {
    KDT_LANE(64)
  }
#undef KDT_LANE
#undef KDT_LANE_S
  KDT_HIP(hipGetLastError());
  return KDT_OK;
}

// ws: optional workspace for the query order (then nothing is allocated).
template <int D>
static kdt_status knn_impl(const kdt_tree* t, const float* d_q, int64_t nq, int k, int32_t* d_idx,
                           float* d_d2, int mode, bool sort_q, int traversal,
                           const int32_t* given, hipStream_t stream, void* ws = nullptr,
                           size_t ws_bytes = 0) {
  if (traversal == 0) traversal = tuned(D, t->n, k).qpw == 64 ? 2 : 1;  // the tuning table
  if (t->leaf > 64) traversal = 1;  // the wave kernel marks at most 64 points per leaf
  if (t->nodes) traversal = 1;      // stored trees: one traversal per lane
  int32_t* order = nullptr;
  if (d_q && !given && sort_q && nq > 1) {
    kdt_status st = order_queries<D>(t, d_q, nq, traversal == 1 ? 0 : 1, &order, stream, nullptr,
                                     ws, ws_bytes);
    if (st != KDT_OK) return st;
  }
  // self queries: `given` is the tree-order row marker (or NULL)
  const int32_t* use = d_q ? (given ? given : order) : given;
  kdt_status st = traversal == 1
                      ? knn_dispatch<D>(t, d_q, nq, k, d_idx, d_d2, mode, use, stream)
                      : knn_packet_launch<D>(view_of(t), t->leaf, d_q, nq, k, d_idx, d_d2, mode,
                                             use, stream);
  if (order && !ws) (void)hipFreeAsync(order, stream);
  return st;
}

template <int D>
static kdt_status range_impl(const kdt_tree* t, const float* d_q, int64_t nq, float r,
                             int32_t* d_count, int64_t* d_off, int32_t* d_idx, int64_t capacity,
                             int64_t* required, bool sort_q, const int32_t* given,
                             int traversal, uint32_t split_budget, bool counts_given,
                             hipStream_t stream) {
  int32_t* own = nullptr;
  if (d_q && !given && sort_q && nq > 1) {
    kdt_status st = order_queries<D>(t, d_q, nq, 0, &own, stream);
    if (st != KDT_OK) return st;
  }
  // self queries: `given` is the tree-order row marker (or NULL)
  const int32_t* order = d_q ? (given ? given : own) : given;
  const TreeView v = view_of(t);
  const float r2 = r * r;
  const unsigned grid = (unsigned)((nq + kQBlock - 1) / kQBlock);
  // both children are pushed: at most levels + 2 entries
  const size_t rsmem = sizeof(uint32_t) * (size_t)(t->levels + 2) * kQBlock;
  kdt_status st = KDT_OK;
  if (counts_given) {
    // the counts and offsets of the sizing call are in d_count and d_off
  } else if (t->nodes) {
    k_range<D, false, StoredShape><<<grid, kQBlock, rsmem, stream>>>(v, d_q, nq, r2, order,
                                                                     d_count, nullptr, nullptr);
  } else if (t->leaf <= 64 && traversal != 1) {
    int cap = 0;
    const TreeView vc = count_view(v, t->leaf, &cap);
    st = range_packet_launch<D>(vc, cap, d_q, nq, r2, order, d_count, split_budget, stream);
  } else {
    k_range<D, false><<<grid, kQBlock, rsmem, stream>>>(v, d_q, nq, r2, order, d_count, nullptr,
                                                        nullptr);
  }
  if (st != KDT_OK) {
    if (own) (void)hipFreeAsync(own, stream);
    return st;
  }
  if (d_off) {
    PoolBuffers buf(stream);
    void* tmp = nullptr;
    int64_t total = 0;
    if (!counts_given && !buf.get((char**)&tmp, scan_scratch_bytes(nq))) {
      kdt_set_error("device allocation failed for the list offsets");
      st = KDT_ENOMEM;
    } else if (!counts_given &&
               exclusive_scan<int64_t>(d_count, d_off, nq, d_off + nq, tmp, stream) != KDT_OK) {
      kdt_set_error("kdt_range: offset scan failed");
      st = KDT_EDEVICE;
    } else {
      if (hipMemcpyAsync(&total, d_off + nq, sizeof(int64_t), hipMemcpyDeviceToHost, stream) !=
              hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess) {
        kdt_set_error("reading the list size failed");
        st = KDT_EDEVICE;
      }
    }
    if (st == KDT_OK) {
      if (required) *required = total;
      if (d_idx && total > capacity) {
        kdt_set_error("list capacity %lld is below the %lld entries needed",
                      (long long)capacity, (long long)total);
        st = KDT_ECAPACITY;
      } else if (d_idx && total > INT32_MAX) {
        kdt_set_error("lists above 2^31-1 entries are not supported");
        st = KDT_EUNSUPPORTED;
      } else if (d_idx && total > 0) {
        int32_t* unsorted = nullptr;
        if (!buf.get(&unsorted, (size_t)total)) {
          kdt_set_error("device allocation failed for the lists");
          st = KDT_ENOMEM;
        } else {
          int32_t* cur = nullptr;
          if (t->nodes) {
            k_range<D, true, StoredShape><<<grid, kQBlock, rsmem, stream>>>(
                v, d_q, nq, r2, order, d_count, d_off, unsorted);
          } else if (t->leaf <= 64 && traversal != 1) {
            // the wave-shared traversal of the counts, writing the lists
            if (!buf.get(&cur, (size_t)nq)) {
              kdt_set_error("device allocation failed for the list cursors");
              st = KDT_ENOMEM;
            } else {
              const FillOut fo{unsorted, d_off, cur};
              int cap = 0;
              const TreeView vc = count_view(v, t->leaf, &cap);
              st = range_packet_launch<D>(vc, cap, d_q, nq, r2, order, d_count, split_budget,
                                          stream, &fo);
            }
          } else {
            k_range<D, true><<<grid, kQBlock, rsmem, stream>>>(v, d_q, nq, r2, order, d_count,
                                                               d_off, unsorted);
          }
          if (st == KDT_OK && hipGetLastError() != hipSuccess) {
            kdt_set_error("kdt_range: list kernel launch failed");
            st = KDT_EDEVICE;
          }
          if (st == KDT_OK) st = sort_list_rows(unsorted, d_idx, d_off, nq, total, t->n, stream);
        }
      }
    }
  }
  if (own) (void)hipFreeAsync(own, stream);
  if (st == KDT_OK) KDT_HIP(hipGetLastError());
  return st;
}


template <int D>
static kdt_status order_into(const kdt_tree* t, const float* d_q, int64_t nq, int kind,
                             int32_t* d_order, hipStream_t stream) {
  int32_t* unused = nullptr;
  return order_queries<D>(t, d_q, nq, kind, &unused, stream, d_order);
}

}  // namespace kdt

using namespace kdt;

extern "C" kdt_status kdt_query_order(const kdt_tree* tree, const float* d_q, int64_t nq,
                                      int32_t kind, int32_t* d_order, hipStream_t stream) {
  kdt_clear_error();
  if (!tree || nq < 0 || nq > INT32_MAX || (kind != 0 && kind != 1)) {
    kdt_set_error("kdt_query_order: NULL tree, nq outside [0, 2^31-1] or kind not 0 or 1");
    return KDT_EINVAL;
  }
  if (nq == 0) return KDT_OK;
  if (!d_q || !d_order) {
    kdt_set_error("kdt_query_order: NULL queries or order");
    return KDT_EINVAL;
  }
  switch (tree->d) {
    case 2: return order_into<2>(tree, d_q, nq, kind, d_order, stream);
    case 3: return order_into<3>(tree, d_q, nq, kind, d_order, stream);
    case 4: return order_into<4>(tree, d_q, nq, kind, d_order, stream);
    case 8: return order_into<8>(tree, d_q, nq, kind, d_order, stream);
    case 16: return order_into<16>(tree, d_q, nq, kind, d_order, stream);
  }
  kdt_set_error("kdt_query_order: unsupported dimension %d", tree->d);
  return KDT_EUNSUPPORTED;
}

namespace kdt {

kdt_status knn_check(const kdt_tree* tree, const float* d_q, int64_t nq, int32_t k,
                     const float* d_d2, int32_t kth_only, const kdt_query_opts* opts,
                     const char* who, KnnArgs* a) {
  if (!tree || nq < 0) {
    kdt_set_error("%s: NULL tree or negative nq", who);
    return KDT_EINVAL;
  }
  if (k < 1 || k > KDT_MAX_K_SORTED) {
    kdt_set_error("%s: k=%d outside [1, %d]", who, k, KDT_MAX_K_SORTED);
    return k < 1 ? KDT_EINVAL : KDT_EUNSUPPORTED;
  }
  if (kth_only < 0 || kth_only > 2) {
    kdt_set_error("%s: kth_only must be 0, 1 or 2", who);
    return KDT_EINVAL;
  }
  a->empty = nq == 0;  // no queries: nothing is read or written
  if (a->empty) return KDT_OK;
  if (!d_d2) {
    kdt_set_error("%s: NULL d_d2", who);
    return KDT_EINVAL;
  }
  if (!d_q && nq != tree->n) {
    kdt_set_error("%s: self queries need nq == n (%lld)", who, (long long)tree->n);
    return KDT_EINVAL;
  }
  a->sort_q = opts ? opts->sort_queries != 0 : true;
  a->traversal = opts ? opts->traversal : 0;
  const int32_t* rows = nullptr;
  const kdt_status rs = self_rows(tree, d_q, opts, who, &rows);
  if (rs != KDT_OK) return rs;
  a->given = d_q ? (opts ? opts->order : nullptr) : rows;
  a->period = opts ? opts->period : nullptr;
  if (a->traversal < 0 || a->traversal > 2) {
    kdt_set_error("%s: traversal must be 0, 1 or 2", who);
    return KDT_EINVAL;
  }
  return KDT_OK;
}

kdt_status knn_in_workspace(const kdt_tree* t, const float* d_q, int64_t nq, int k,
                            int32_t* d_idx, float* d_d2, int mode, const KnnArgs& a, void* ws,
                            size_t ws_bytes, hipStream_t stream) {
#define KDT_WS(DD)                                                                            \
  return knn_impl<DD>(t, d_q, nq, k, d_idx, d_d2, mode, a.sort_q, a.traversal, a.given, stream, \
                      ws, ws_bytes)
  switch (t->d) {
    case 2: KDT_WS(2);
    case 3: KDT_WS(3);
    case 4: KDT_WS(4);
    case 8: KDT_WS(8);
    case 16: KDT_WS(16);
  }
#undef KDT_WS
  kdt_set_error("unsupported dimension %d", t->d);
  return KDT_EUNSUPPORTED;
}

}  // namespace kdt

extern "C" kdt_status kdt_knn(const kdt_tree* tree, const float* d_q, int64_t nq, int32_t k,
                              int32_t* d_idx, float* d_d2, int32_t kth_only,
                              const kdt_query_opts* opts, hipStream_t stream) {
  kdt_clear_error();
  if (refuse_f64(tree, "kdt_knn")) return KDT_EUNSUPPORTED;
  KnnArgs a;
  const kdt_status chk = knn_check(tree, d_q, nq, k, d_d2, kth_only, opts, "kdt_knn", &a);
  if (chk != KDT_OK || a.empty) return chk;
  if ((k > KDT_MAX_K || a.period) && refuse_stored(tree, "kdt_knn with k > 64 or a period"))
    return KDT_EUNSUPPORTED;
  if (k > KDT_MAX_K)
    return knn_large(tree, d_q, nq, k, d_idx, d_d2, kth_only, a.sort_q, a.given, a.period, stream);
  if (a.period)
    return knn_torus(tree, d_q, nq, k, d_idx, d_d2, kth_only, a.sort_q, a.given, a.period, stream);
  return knn_in_workspace(tree, d_q, nq, k, d_idx, d_d2, kth_only, a, nullptr, 0, stream);
}

extern "C" kdt_status kdt_range(const kdt_tree* tree, const float* d_q, int64_t nq, float r,
                                int32_t* d_count, int64_t* d_offsets, int32_t* d_idx,
                                int64_t capacity, int64_t* required, const kdt_query_opts* opts,
                                hipStream_t stream) {
  kdt_clear_error();
  if (refuse_f64(tree, "kdt_range")) return KDT_EUNSUPPORTED;
  if (!tree || nq < 0 || !(r >= 0.0f) || !std::isfinite(r)) {
    kdt_set_error("kdt_range: NULL tree, negative nq, or r not finite and >= 0");
    return KDT_EINVAL;
  }
  if (!d_count && nq > 0) {
    kdt_set_error("kdt_range: NULL d_count");
    return KDT_EINVAL;
  }
  if (!d_q && nq > 0 && nq != tree->n) {
    kdt_set_error("kdt_range: self queries need nq == n (%lld)", (long long)tree->n);
    return KDT_EINVAL;
  }
  if (d_idx && !d_offsets) {
    kdt_set_error("kdt_range: lists need d_offsets");
    return KDT_EINVAL;
  }
  if (opts && opts->split_budget < 0) {
    kdt_set_error("kdt_range: split_budget must be >= 0");
    return KDT_EINVAL;
  }
  const bool counts_given = opts && opts->counts_given;
  if (opts && (opts->counts_given < 0 || opts->counts_given > 1 ||
               (counts_given && (!d_idx || !d_offsets)))) {
    kdt_set_error("kdt_range: counts_given must be 0 or 1, and 1 needs lists (d_idx, d_offsets)");
    return KDT_EINVAL;
  }
  const uint32_t budget = opts ? (uint32_t)opts->split_budget : 0u;
  if (nq > INT32_MAX && d_offsets) {
    kdt_set_error("kdt_range: list mode supports at most 2^31-1 queries");
    return KDT_EUNSUPPORTED;
  }
  if (nq == 0) {
    if (required) *required = 0;
    if (d_offsets) {
      int64_t z = 0;
      if (hipMemcpyAsync(d_offsets, &z, sizeof(z), hipMemcpyHostToDevice, stream) != hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess) {
        kdt_set_error("kdt_range: writing empty offsets failed");
        return KDT_EDEVICE;
      }
    }
    return KDT_OK;
  }
  const bool sort_q = opts ? opts->sort_queries != 0 : true;
  const int32_t* rows = nullptr;
  const kdt_status rs = self_rows(tree, d_q, opts, "kdt_range", &rows);
  if (rs != KDT_OK) return rs;
  const int32_t* given = d_q ? (opts ? opts->order : nullptr) : rows;
  if (opts && opts->period && refuse_stored(tree, "kdt_range with a period"))
    return KDT_EUNSUPPORTED;
  if (opts && opts->period)
    return range_torus(tree, d_q, nq, r, d_count, d_offsets, d_idx, capacity, required, sort_q,
                       given, opts->period, counts_given, stream);
  const int trav = opts ? opts->traversal : 0;
  switch (tree->d) {
    case 2: return range_impl<2>(tree, d_q, nq, r, d_count, d_offsets, d_idx, capacity, required, sort_q, given, trav, budget, counts_given, stream);
    case 3: return range_impl<3>(tree, d_q, nq, r, d_count, d_offsets, d_idx, capacity, required, sort_q, given, trav, budget, counts_given, stream);
    case 4: return range_impl<4>(tree, d_q, nq, r, d_count, d_offsets, d_idx, capacity, required, sort_q, given, trav, budget, counts_given, stream);
    case 8: return range_impl<8>(tree, d_q, nq, r, d_count, d_offsets, d_idx, capacity, required, sort_q, given, trav, budget, counts_given, stream);
    case 16: return range_impl<16>(tree, d_q, nq, r, d_count, d_offsets, d_idx, capacity, required, sort_q, given, trav, budget, counts_given, stream);
  }
  kdt_set_error("kdt_range: unsupported dimension %d", tree->d);
  return KDT_EUNSUPPORTED;
}
