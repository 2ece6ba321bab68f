// kdt_knn_packet.hip -- wave-coherent kNN traversal (Sec. 2.3, Algorithm 2
// semantics) for gfx950.
//
// A wave of 64 spatially coherent queries (tree order for self queries, leaf
// order for external ones) walks the tree together.  The node stack is held in
// the wave's lane registers (entry i lives in lane i, popped with readlane), so
// it costs no memory.  A node is entered when at least one lane's box distance
// is within its current k-th candidate (wave ballot); a visited leaf is copied
// once into the wave's LDS slice and every point is then read back as a
// broadcast, so one coalesced load serves 64 queries.  Each lane keeps its own
// register top-k keyed by (d2, index): the result is exactly the k smallest
// keys, the same as any exact traversal.
#include <hip/hip_runtime.h>

#include "kdt_query.h"

namespace kdt {

constexpr int kPWaves = 4;  // waves per workgroup (independent packets)

template <int D, int KC>
__global__ __launch_bounds__(64 * kPWaves) void k_knn_packet(TreeView t, const float* __restrict__ q,
                                                             int64_t nq, int k,
                                                             const int32_t* __restrict__ order,
                                                             int mode, int32_t* __restrict__ oidx,
                                                             float* __restrict__ od2, int leaf_cap) {
  extern __shared__ __align__(16) float lds[];
  constexpr int S = rec_stride(D);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* leafbuf = lds + (size_t)wave * leaf_cap * S;
  const int64_t s0 = ((int64_t)blockIdx.x * kPWaves + wave) * 64;
  if (s0 >= nq) return;  // whole wave idle
  const int64_t s = s0 + lane;
  const bool active = s < nq;
  float p[D];
  int64_t row = 0;
  if (active) {
    if (q == nullptr) {
      int32_t id = 0;
      load_rec<D>(t.rec, s, p, id);
      row = id;
    } else {
      row = order ? order[s] : s;
#pragma unroll
      for (int a = 0; a < D; ++a) p[a] = q[row * D + a];
    }
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a) p[a] = 0.0f;
  }
  TopK<KC> best;
  best.init(k);
  const uint32_t first_leaf = (1u << t.levels) - 1u;
  uint32_t stackv = 0;  // lane i holds stack entry i
  int sp = 1;
  uint64_t mask = 0;    // this lane's pending candidates in the staged leaf
  // One flat loop (the candidate list is then live across a single loop
  // header): a round either inserts one pending candidate per lane, or pops
  // and visits the next node.
  for (;;) {
    if (__any(mask != 0)) {
      const bool has = mask != 0;
      const int i = has ? __ffsll((unsigned long long)mask) - 1 : 0;
      mask &= mask - 1;
      const float* r = leafbuf + i * S;
      float x[D];
#pragma unroll
      for (int a = 0; a < D; ++a) x[a] = r[a];
      const uint64_t key = make_key(sq_dist<D>(x, p), __float_as_int(r[D]));
      best.insert(has ? key : kEmptyKey);
      continue;
    }
    if (sp == 0) break;
    --sp;
    const uint32_t node = (uint32_t)__builtin_amdgcn_readlane((int)stackv, sp);
    float lo[D], hi[D];
    load_box<D>(t.box, node, lo, hi);
    const bool need = active && box_mindist<D>(lo, hi, p) <= best.worst_d2();
    if (!__any(need)) continue;
    if (node >= first_leaf) {
      const int64_t j = node - first_leaf;
      const int64_t b = node_begin(t.n, t.levels, j), e = node_begin(t.n, t.levels, j + 1);
      const int cnt = (int)(e - b);
      wave_sync();  // every lane is done with the previous leaf
      const float4* src = reinterpret_cast<const float4*>(t.rec + b * S);
      float4* dst = reinterpret_cast<float4*>(leafbuf);
      for (int i = lane; i < cnt * (S / 4); i += 64) dst[i] = src[i];
      wave_sync();
      // Mark the leaf points (at most 64) that beat this lane's current k-th
      // candidate; the rounds above then insert them, so the wave pays for
      // the largest per-lane count of insertions rather than for every point
      // some lane wants.
      const uint64_t w = best.worst();
#pragma unroll 1
      for (int i = 0; i < cnt; ++i) {
        const float* r = leafbuf + i * S;
        float x[D];
#pragma unroll
        for (int a = 0; a < D; ++a) x[a] = r[a];
        const uint64_t key = make_key(sq_dist<D>(x, p), __float_as_int(r[D]));
        mask |= (uint64_t)(key < w) << i;
      }
      if (!active) mask = 0;
    } else {
      const uint32_t c0 = 2 * node + 1, c1 = c0 + 1;
      load_box<D>(t.box, c0, lo, hi);
      const float d0 = box_mindist<D>(lo, hi, p);
      load_box<D>(t.box, c1, lo, hi);
      const float d1 = box_mindist<D>(lo, hi, p);
      const float wd = best.worst_d2();
      const bool n0 = active && d0 <= wd, n1 = active && d1 <= wd;
      const uint64_t b0 = __ballot(n0), b1 = __ballot(n1);
      const int pref0 = __popcll(__ballot(n0 && d0 <= d1));
      const int pref1 = __popcll(__ballot(n1 && d1 < d0));
      const bool first0 = pref0 >= pref1;
      const uint32_t nn = first0 ? c0 : c1, ff = first0 ? c1 : c0;
      const bool need_n = first0 ? b0 != 0 : b1 != 0;
      const bool need_f = first0 ? b1 != 0 : b0 != 0;
      if (need_f) {
        stackv = lane == sp ? ff : stackv;
        ++sp;
      }
      if (need_n) {
        stackv = lane == sp ? nn : stackv;
        ++sp;
      }
    }
  }
  if (active) knn_write<KC>(best, k, mode, row, oidx, od2);
}

template <int D>
kdt_status knn_packet_launch(const TreeView& v, int leaf, const float* d_q, int64_t nq, int k,
                             int32_t* d_idx, float* d_d2, int mode, const int32_t* order,
                             hipStream_t stream) {
  const unsigned grid = (unsigned)((nq + 64 * kPWaves - 1) / (64 * kPWaves));
  const size_t smem = sizeof(float) * (size_t)leaf * rec_stride(D) * kPWaves;
  if (k <= 8)
    k_knn_packet<D, 8><<<grid, 64 * kPWaves, smem, stream>>>(v, d_q, nq, k, order, mode, d_idx, d_d2, leaf);
  else if (k <= 16)
    k_knn_packet<D, 16><<<grid, 64 * kPWaves, smem, stream>>>(v, d_q, nq, k, order, mode, d_idx, d_d2, leaf);
  else if (k <= 32)
    k_knn_packet<D, 32><<<grid, 64 * kPWaves, smem, stream>>>(v, d_q, nq, k, order, mode, d_idx, d_d2, leaf);
  else
    k_knn_packet<D, 64><<<grid, 64 * kPWaves, smem, stream>>>(v, d_q, nq, k, order, mode, d_idx, d_d2, leaf);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_knn: packet kernel launch failed");
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

template kdt_status knn_packet_launch<2>(const TreeView&, int, const float*, int64_t, int, int32_t*, float*, int, const int32_t*, hipStream_t);
template kdt_status knn_packet_launch<3>(const TreeView&, int, const float*, int64_t, int, int32_t*, float*, int, const int32_t*, hipStream_t);
template kdt_status knn_packet_launch<4>(const TreeView&, int, const float*, int64_t, int, int32_t*, float*, int, const int32_t*, hipStream_t);
template kdt_status knn_packet_launch<8>(const TreeView&, int, const float*, int64_t, int, int32_t*, float*, int, const int32_t*, hipStream_t);
template kdt_status knn_packet_launch<16>(const TreeView&, int, const float*, int64_t, int, int32_t*, float*, int, const int32_t*, hipStream_t);

}  // namespace kdt
