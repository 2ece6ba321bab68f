// kdt_box.hip -- axis-aligned box queries on gfx950: the rectangular ranges
// that Sec. 2.3 names beside the ball query.  For each query box [lo, hi]
// (closed on every axis) the number of tree points inside and, optionally,
// their input indices in CSR form, ascending.  A node whose tight box misses
// the query box is skipped, a node whose box lies inside it is taken whole,
// leaves test their points.  Counts use the wave-shared traversal of the ball
// counts with a box as the query shape (packed leaf scans, heavy traversals
// split over several launches); the lists, and trees with leaves of more than
// 64 points, one traversal per lane.  Only comparisons are involved, so the
// result is exact.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kdt_packet.h"

namespace kdt {

constexpr int kBoxBlock = 128;

// Counts (FILL = false) or writes the input indices of the points inside each
// query box, from offsets[row] on (FILL = true).  The node-id stack lives in
// LDS, levels + 2 entries per lane.
template <int D, bool FILL>
__global__ __launch_bounds__(kBoxBlock) void k_box(TreeView t, const float* __restrict__ qlo,
                                                   const float* __restrict__ qhi, int64_t nq,
                                                   const int32_t* __restrict__ order,
                                                   int32_t* __restrict__ count,
                                                   const int64_t* __restrict__ offsets,
                                                   int32_t* __restrict__ out) {
  extern __shared__ uint32_t box_stk[];
  uint32_t* col = box_stk + threadIdx.x;
  const int64_t s = (int64_t)blockIdx.x * kBoxBlock + threadIdx.x;
  if (s >= nq) return;
  const int64_t row = order ? order[s] : s;
  float ql[D], qh[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    ql[a] = qlo[row * D + a];
    qh[a] = qhi[row * D + a];
  }
  const uint32_t first_leaf = (1u << t.levels) - 1u;
  int64_t c = 0;
  int64_t pos = FILL ? offsets[row] : 0;
  int sp = 0;
  col[kBoxBlock * sp++] = 0;
  while (sp > 0) {
    const uint32_t node = col[kBoxBlock * --sp];
    float lo[D], hi[D];
    load_box<D>(t.box, node, lo, hi);
    bool miss = false, inside = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      miss |= hi[a] < ql[a] || lo[a] > qh[a];
      inside &= ql[a] <= lo[a] && hi[a] <= qh[a];
    }
    if (miss) continue;
    const int lev = node_level(node);
    const int64_t j = (int64_t)node - ((int64_t(1) << lev) - 1);
    const int64_t b = node_begin(t.n, lev, j), e = node_begin(t.n, lev, j + 1);
    if (inside) {
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
    if (node >= first_leaf) {
      for (int64_t i = b; i < e; ++i) {
        float x[D];
        int32_t id = 0;
        load_rec<D>(t.rec, i, x, id);
        bool in = true;
#pragma unroll
        for (int a = 0; a < D; ++a) in &= ql[a] <= x[a] && x[a] <= qh[a];
        if (in) {
          if (FILL) out[pos++] = id;
          ++c;
        }
      }
      continue;
    }
    col[kBoxBlock * sp++] = 2 * node + 2;
    col[kBoxBlock * sp++] = 2 * node + 1;
  }
  if (!FILL) count[row] = (int32_t)c;
}

// Box centres for ordering the queries along the tree (a non-finite centre,
// from an infinite or NaN bound, becomes 0: the order only affects speed).
template <int D>
__global__ void k_box_centres(const float* __restrict__ lo, const float* __restrict__ hi,
                              int64_t nq, float* __restrict__ c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq * D) return;
  const float m = 0.5f * lo[i] + 0.5f * hi[i];
  c[i] = isfinite(m) ? m : 0.0f;
}

template <int D>
static kdt_status box_impl(const kdt_tree* tr, const float* d_lo, const float* d_hi, int64_t nq,
                           int32_t* d_count, int64_t* d_off, int32_t* d_idx, int64_t capacity,
                           int64_t* required, bool sort_q, const int32_t* given, int traversal,
                           uint32_t split_budget, hipStream_t stream) {
  TreeView v;
  v.rec = tr->rec;
  v.box = tr->box;
  v.n = tr->n;
  v.levels = tr->levels;
  PoolBuffers buf(stream);
  const int32_t* order = given;
  if (!order && sort_q && nq > 1) {
    float* centres = nullptr;
    int32_t* own = nullptr;
    if (!buf.get(&centres, (size_t)nq * D) || !buf.get(&own, (size_t)nq)) {
      kdt_set_error("device allocation failed for the box query order");
      return KDT_ENOMEM;
    }
    k_box_centres<D><<<(unsigned)((nq * D + 255) / 256), 256, 0, stream>>>(d_lo, d_hi, nq, centres);
    const kdt_status st = kdt_query_order(tr, centres, nq, 0, own, stream);
    if (st != KDT_OK) return st;
    order = own;
  }
  const unsigned grid = (unsigned)((nq + kBoxBlock - 1) / kBoxBlock);
  const size_t smem = sizeof(uint32_t) * (size_t)(tr->levels + 2) * kBoxBlock;
  if (tr->leaf <= 64 && traversal != 1) {
    int cap = 0;
    const TreeView vc = count_view(v, tr->leaf, &cap);
    const kdt_status st =
        box_packet_launch<D>(vc, cap, d_lo, d_hi, nq, order, d_count, split_budget, stream);
    if (st != KDT_OK) return st;
  } else {
    k_box<D, false><<<grid, kBoxBlock, smem, stream>>>(v, d_lo, d_hi, nq, order, d_count,
                                                        nullptr, nullptr);
    if (hipGetLastError() != hipSuccess) {
      kdt_set_error("kdt_box: count kernel launch failed");
      return KDT_EDEVICE;
    }
  }
  if (!d_off) return KDT_OK;
  void* tmp = nullptr;
  if (!buf.get((char**)&tmp, scan_scratch_bytes(nq))) {
    kdt_set_error("device allocation failed for the box list offsets");
    return KDT_ENOMEM;
  }
  int64_t total = 0;
  if (exclusive_scan<int64_t>(d_count, d_off, nq, d_off + nq, tmp, stream) != KDT_OK) {
    kdt_set_error("kdt_box: offset scan failed");
    return KDT_EDEVICE;
  }
  if (hipMemcpyAsync(&total, d_off + nq, sizeof(int64_t), hipMemcpyDeviceToHost, stream) !=
          hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    kdt_set_error("kdt_box: reading the list size failed");
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
    kdt_set_error("device allocation failed for the box lists");
    return KDT_ENOMEM;
  }
  if (tr->leaf <= 64 && traversal != 1) {
    // the wave-shared traversal of the counts, writing the lists
    int32_t* cur = nullptr;
    if (!buf.get(&cur, (size_t)nq)) {
      kdt_set_error("device allocation failed for the box list cursors");
      return KDT_ENOMEM;
    }
    const FillOut fo{unsorted, d_off, cur};
    int cap = 0;
    const TreeView vc = count_view(v, tr->leaf, &cap);
    const kdt_status st = box_packet_launch<D>(vc, cap, d_lo, d_hi, nq, order, d_count,
                                               split_budget, stream, &fo);
    if (st != KDT_OK) return st;
  } else {
    k_box<D, true><<<grid, kBoxBlock, smem, stream>>>(v, d_lo, d_hi, nq, order, d_count, d_off,
                                                       unsorted);
  }
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_box: list kernel launch failed");
    return KDT_EDEVICE;
  }
  const kdt_status ss = sort_list_rows(unsorted, d_idx, d_off, nq, total, tr->n, stream);
  if (ss != KDT_OK) return ss;
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_box: list kernel launch failed");
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

}  // namespace kdt

using namespace kdt;

extern "C" kdt_status kdt_box(const kdt_tree* tree, const float* d_lo, const float* d_hi,
                              int64_t nq, int32_t* d_count, int64_t* d_offsets, int32_t* d_idx,
                              int64_t capacity, int64_t* required, const kdt_query_opts* opts,
                              hipStream_t stream) {
  kdt_clear_error();
  if (refuse_stored(tree, "kdt_box") || refuse_f64(tree, "kdt_box")) return KDT_EUNSUPPORTED;
  if (!tree || nq < 0) {
    kdt_set_error("kdt_box: NULL tree or negative nq");
    return KDT_EINVAL;
  }
  if (nq > 0 && (!d_lo || !d_hi || !d_count)) {
    kdt_set_error("kdt_box: NULL lo, hi or d_count");
    return KDT_EINVAL;
  }
  if (d_idx && !d_offsets) {
    kdt_set_error("kdt_box: lists need d_offsets");
    return KDT_EINVAL;
  }
  if (nq > INT32_MAX && d_offsets) {
    kdt_set_error("kdt_box: list mode supports at most 2^31-1 queries");
    return KDT_EUNSUPPORTED;
  }
  if (nq == 0) {
    if (required) *required = 0;
    if (d_offsets) {
      int64_t z = 0;
      if (hipMemcpyAsync(d_offsets, &z, sizeof(z), hipMemcpyHostToDevice, stream) != hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess) {
        kdt_set_error("kdt_box: writing empty offsets failed");
        return KDT_EDEVICE;
      }
    }
    return KDT_OK;
  }
  if (opts && (opts->split_budget < 0 || opts->traversal < 0 || opts->traversal > 2)) {
    kdt_set_error("kdt_box: traversal must be 0, 1 or 2 and split_budget >= 0");
    return KDT_EINVAL;
  }
  if (opts && opts->period) {
    kdt_set_error("kdt_box: periodic boundaries are not supported for box queries");
    return KDT_EUNSUPPORTED;
  }
  const bool sort_q = opts ? opts->sort_queries != 0 : true;
  const int32_t* given = opts ? opts->order : nullptr;
  const int trav = opts ? opts->traversal : 0;
  const uint32_t budget = opts ? (uint32_t)opts->split_budget : 0u;
  switch (tree->d) {
    case 2: return box_impl<2>(tree, d_lo, d_hi, nq, d_count, d_offsets, d_idx, capacity, required, sort_q, given, trav, budget, stream);
    case 3: return box_impl<3>(tree, d_lo, d_hi, nq, d_count, d_offsets, d_idx, capacity, required, sort_q, given, trav, budget, stream);
    case 4: return box_impl<4>(tree, d_lo, d_hi, nq, d_count, d_offsets, d_idx, capacity, required, sort_q, given, trav, budget, stream);
    case 8: return box_impl<8>(tree, d_lo, d_hi, nq, d_count, d_offsets, d_idx, capacity, required, sort_q, given, trav, budget, stream);
    case 16: return box_impl<16>(tree, d_lo, d_hi, nq, d_count, d_offsets, d_idx, capacity, required, sort_q, given, trav, budget, stream);
  }
  kdt_set_error("kdt_box: unsupported dimension %d", tree->d);
  return KDT_EUNSUPPORTED;
}
