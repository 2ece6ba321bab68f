// kdt_packet.hip -- single-tree kernels of the wave-coherent traversals
// (kNN, Sec. 2.3 / Algorithm 2; ball counts, Algorithm 3) for gfx950.
#include <hip/hip_runtime.h>

#include "kdt_packet.h"
#include "kdt_torus.h"

namespace kdt {

constexpr int kPWaves = 4;  // waves per workgroup (independent packets)
// Ball-count work splitting: passes; node visits per wave before it hands the
// rest of its stack on, in the first pass (where most waves are light and a
// hand-off costs atomics) and in the later ones; task slots per pass;
// workgroups of a task pass.
constexpr int kRangePasses = 8;
constexpr uint32_t kRangeBudgetFirst = 512;
constexpr uint32_t kRangeBudget = 32;
constexpr uint32_t kRangeTaskCap = 1u << 20;
constexpr unsigned kRangeTaskBlocks = 8192;
// The first pass hands work on only once fewer than this many of its waves
// are left (about what the chip holds at once).
constexpr int64_t kRangeTailWaves = 8192;

// LDS of a workgroup: a leaf slice per wave.
template <int D>
size_t packet_lds_bytes(int leaf) {
  return sizeof(float) * (size_t)leaf * rec_stride(D) * kPWaves;
}

template <int D>
__device__ __forceinline__ float* wave_slice(float* lds, int wave, int leaf_cap) {
  return lds + (size_t)wave * leaf_cap * rec_stride(D);
}

template <int D>
__device__ __forceinline__ bool load_query(const TreeView& t, const float* __restrict__ q,
                                           int64_t nq, const int32_t* __restrict__ order,
                                           int64_t s, float p[D], int64_t& row) {
  if (s >= nq) {
#pragma unroll
    for (int a = 0; a < D; ++a) p[a] = 0.0f;
    return false;
  }
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
  return true;
}

// MODE 0 writes k (index, d2) pairs per row, 1 the k-th d2, 2 the k-th
// distance (a compile-time choice, so each output form is its own kernel).
template <int D, int KC, int MODE>
__global__ __launch_bounds__(64 * kPWaves) void k_knn_packet(TreeView t, const float* __restrict__ q,
                                                             int64_t nq, int k,
                                                             const int32_t* __restrict__ order,
                                                             int32_t* __restrict__ oidx,
                                                             float* __restrict__ od2, int leaf_cap) {
  extern __shared__ __align__(16) float lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t s0 = (xcd_block<kXcdRunPacket>() * kPWaves + wave) * 64;
  if (s0 >= nq) return;  // whole wave idle
  float p[D];
  int64_t row = 0;
  const bool active = load_query<D>(t, q, nq, order, s0 + lane, p, row);
  TopK<KC> best;
  best.init(k);
  packet_knn<D, KC>(t, p, active, best, lds + (size_t)wave * knn_wave_floats<D>(leaf_cap),
                    leaf_cap);
  if (active) knn_write<KC>(best, k, MODE, row, oidx, od2);
}

// Where the queries of a count come from: balls (centres, or the tree's own
// points, and one squared radius) or boxes (corners).
template <int D>
struct BallQueries {
  using Shape = BallShape<D>;
  const float* q;  // [nq][D], or nullptr: the tree's own points
  float r2;
  __device__ __forceinline__ bool load(const TreeView& t, int64_t nq, const int32_t* order,
                                       int64_t s, Shape& sh, int64_t& row) const {
    sh.r2 = r2;
    return load_query<D>(t, q, nq, order, s, sh.p, row);
  }
};

template <int D>
struct TorusBallQueries {
  using Shape = TorusBallShape<D>;
  const float* q;  // [nq][D], or nullptr: the tree's own points
  float r2;
  Torus<D> T;
  __device__ __forceinline__ bool load(const TreeView& t, int64_t nq, const int32_t* order,
                                       int64_t s, Shape& sh, int64_t& row) const {
    sh.r2 = r2;
    sh.T = T;
    return load_query<D>(t, q, nq, order, s, sh.p, row);
  }
};

template <int D, class Metric>
struct VarBallQueries {
  using Shape = VarBallShape<D, Metric>;
  const float* q;   // [rows][D]
  const float* r2;  // [rows]
  Metric m;
  __device__ __forceinline__ bool load(const TreeView& t, int64_t nq, const int32_t* order,
                                       int64_t s, Shape& sh, int64_t& row) const {
    sh.m = m;
    const bool ok = load_query<D>(t, q, nq, order, s, sh.p, row);
    sh.r2 = ok ? r2[row] : 0.0f;
    return ok;
  }
};

template <int D>
struct BoxQueries {
  using Shape = BoxShape<D>;
  const float* lo;  // [nq][D]
  const float* hi;
  __device__ __forceinline__ bool load(const TreeView&, int64_t nq, const int32_t* order,
                                       int64_t s, Shape& sh, int64_t& row) const {
    if (s >= nq) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        sh.lo[a] = 1.0f;  // an empty box
        sh.hi[a] = 0.0f;
      }
      return false;
    }
    row = order ? order[s] : s;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      sh.lo[a] = lo[row * D + a];
      sh.hi[a] = hi[row * D + a];
    }
    return true;
  }
};

template <int D, class Q>
__host__ __device__ constexpr size_t count_wave_floats(int leaf) {
  return range_wave_floats<D, Q::Shape::kFloats>(leaf);
}

// First pass of the counts: one 64-query group per wave from the root; writes
// each count (partial if the wave handed subtrees on), or with FILL the
// lists.
template <int D, class Q, bool FILL>
__global__ __launch_bounds__(64 * kPWaves) void k_count_packet(TreeView t, Q src, int64_t nq,
                                                               const int32_t* __restrict__ order,
                                                               int32_t* __restrict__ count,
                                                               int leaf_cap, PacketSpill spill,
                                                               FillOut fo) {
  extern __shared__ __align__(16) float lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t s0 = (xcd_block<kXcdRunPacket>() * kPWaves + wave) * 64;
  if (s0 >= nq) return;
  typename Q::Shape sh;
  int64_t row = 0;
  const bool active = src.load(t, nq, order, s0 + lane, sh, row);
  const int64_t c = packet_range_count<D, typename Q::Shape, FILL>(
      t, sh, active, lds + (size_t)wave * count_wave_floats<D, Q>(leaf_cap), leaf_cap, 0u, ~0ull,
      (uint32_t)(s0 / 64), spill, row, fo);
  if (!FILL && active) count[row] = (int32_t)c;
  wave_done(spill);
}

// A later pass: each wave takes tasks left by the previous pass (a fixed
// count, read at start, so every wave's loop ends) and adds its counts.
template <int D, class Q, bool FILL>
__global__ __launch_bounds__(64 * kPWaves) void k_count_tasks(
    TreeView t, Q src, int64_t nq, const int32_t* __restrict__ order,
    int32_t* __restrict__ count, int leaf_cap, const PacketTask* __restrict__ in,
    const uint32_t* __restrict__ in_count, uint32_t in_cap, PacketSpill spill, FillOut fo) {
  extern __shared__ __align__(16) float lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t n = min(*in_count, in_cap);
  float* slice = lds + (size_t)wave * count_wave_floats<D, Q>(leaf_cap);
  for (uint32_t k = blockIdx.x * kPWaves + wave; k < n; k += gridDim.x * kPWaves) {
    const PacketTask task = in[k];
    if (task.node == kNoNode) continue;
    typename Q::Shape sh;
    int64_t row = 0;
    const bool active = src.load(t, nq, order, (int64_t)task.group * 64 + lane, sh, row);
    const uint64_t mask = ((uint64_t)task.hi << 32) | task.lo;
    const int64_t c = packet_range_count<D, typename Q::Shape, FILL>(
        t, sh, active, slice, leaf_cap, task.node, mask, task.group, spill, row, fo);
    if (!FILL && active && c != 0) atomicAdd(count + row, (int32_t)c);
  }
}

__global__ void k_zero_tasks(uint32_t* c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0u;
}

__global__ void k_zero_i32(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <int D>
__global__ __launch_bounds__(64 * kPWaves) void k_fof_packet(TreeView t, float l2,
                                                             int32_t* __restrict__ parent,
                                                             uint32_t* __restrict__ conn,
                                                             int leaf_cap) {
  extern __shared__ __align__(16) float lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t s0 = (xcd_block<kXcdRunFof>() * kPWaves + wave) * 64;
  if (s0 >= t.n) return;
  const int64_t pos = s0 + lane;
  const bool active = pos < t.n;
  float p[D];
  int32_t me = 0;
  if (active) {
    load_rec<D>(t.rec, pos, p, me);
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a) p[a] = 0.0f;
  }
  packet_fof<D>(t, p, pos, me, active, l2, 0, parent, conn, wave_slice<D>(lds, wave, leaf_cap));
}

template <int D>
kdt_status fof_packet_launch(const TreeView& v, int leaf, float l2, int32_t* parent, uint32_t* conn,
                             hipStream_t stream) {
  const unsigned grid = (unsigned)((v.n + 64 * kPWaves - 1) / (64 * kPWaves));
  k_fof_packet<D><<<grid, 64 * kPWaves, packet_lds_bytes<D>(leaf), stream>>>(v, l2, parent, conn,
                                                                            leaf);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_fof: packet kernel launch failed");
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

template <int D>
__global__ __launch_bounds__(64 * kPWaves) void k_fof_torus_packet(TreeView t, float l2,
                                                                   Torus<D> T,
                                                                   int32_t* __restrict__ parent,
                                                                   uint32_t* __restrict__ conn,
                                                                   int leaf_cap) {
  extern __shared__ __align__(16) float lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t s0 = (xcd_block<kXcdRunFof>() * kPWaves + wave) * 64;
  if (s0 >= t.n) return;
  const int64_t pos = s0 + lane;
  const bool active = pos < t.n;
  float p[D];
  int32_t me = 0;
  if (active) {
    load_rec<D>(t.rec, pos, p, me);
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a) p[a] = 0.0f;
  }
  packet_fof<D>(t, p, pos, me, active, l2, 0, parent, conn, wave_slice<D>(lds, wave, leaf_cap),
                TorusMetric<D>{T});
}

template <int D>
kdt_status torus_fof_packet_launch(const TreeView& v, int leaf, float l2, const Torus<D>& T,
                                   int32_t* parent, uint32_t* conn, hipStream_t stream) {
  const unsigned grid = (unsigned)((v.n + 64 * kPWaves - 1) / (64 * kPWaves));
  k_fof_torus_packet<D><<<grid, 64 * kPWaves, packet_lds_bytes<D>(leaf), stream>>>(
      v, l2, T, parent, conn, leaf);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_fof_torus: packet kernel launch failed");
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

template <int D>
kdt_status knn_packet_launch(const TreeView& v, int leaf, const float* d_q, int64_t nq, int k,
                             int32_t* d_idx, float* d_d2, int mode, const int32_t* order,
                             hipStream_t stream) {
  const unsigned grid = (unsigned)((nq + 64 * kPWaves - 1) / (64 * kPWaves));
  const size_t smem = sizeof(float) * knn_wave_floats<D>(leaf) * kPWaves;
#define KDT_LAUNCH(KC, M)                                                                      \
  k_knn_packet<D, KC, M><<<grid, 64 * kPWaves, smem, stream>>>(v, d_q, nq, k, order, d_idx, d_d2, \
                                                               leaf)
#define KDT_BY_MODE(KC)          \
  if (mode == 0) KDT_LAUNCH(KC, 0); \
  else if (mode == 1) KDT_LAUNCH(KC, 1); \
  else KDT_LAUNCH(KC, 2);
  if (k <= 8) {
    KDT_BY_MODE(8)
  } else if (k <= 16) {
    KDT_BY_MODE(16)
  } else if (k <= 32) {
    KDT_BY_MODE(32)
  } else {
    KDT_BY_MODE(64)
  }
#undef KDT_BY_MODE
#undef KDT_LAUNCH
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_knn: packet kernel launch failed");
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

// The wave-shared counts (balls or boxes), with heavy traversals split over
// kRangePasses launches: the first kRangePasses - 1 hand off what exceeds their
// budget of node visits, the last finishes everything.
//
// With `fill` the same launches write the CSR lists instead (fill->cur zeroed
// here first); d_count is then not written.
template <int D, class Q>
static kdt_status count_packet_launch(const TreeView& v, int leaf, Q src, int64_t nq,
                                      const int32_t* order, int32_t* d_count,
                                      uint32_t split_budget, hipStream_t stream,
                                      const char* who, const FillOut* fill = nullptr) {
  const unsigned grid = (unsigned)((nq + 64 * kPWaves - 1) / (64 * kPWaves));
  const size_t smem = sizeof(float) * count_wave_floats<D, Q>(leaf) * kPWaves;
  PoolBuffers buf(stream);
  PacketTask* tasks = nullptr;
  uint32_t* counts = nullptr;
  // counts[0 .. kRangePasses - 1): tasks per pass; then the first pass's
  // finished-wave counters
  if (!buf.get(&tasks, (size_t)kRangeTaskCap * (kRangePasses - 1)) ||
      !buf.get(&counts, kRangePasses + kDoneShards)) {
    kdt_set_error("%s: device allocation failed for the task lists", who);
    return KDT_ENOMEM;
  }
  k_zero_tasks<<<1, 64, 0, stream>>>(counts, kRangePasses + kDoneShards);
  // a caller's budget applies to every wave of every launch
  const uint32_t first = split_budget ? split_budget : kRangeBudgetFirst;
  const uint32_t later = split_budget ? split_budget : kRangeBudget;
  const int64_t waves = (nq + 63) / 64;
  const uint32_t tail_from = split_budget                ? 0u
                             : waves > kRangeTailWaves ? (uint32_t)(waves - kRangeTailWaves)
                                                       : 0u;
  const FillOut fo = fill ? *fill : FillOut{nullptr, nullptr, nullptr};
  if (fill) k_zero_i32<<<(unsigned)((nq + 255) / 256), 256, 0, stream>>>(fill->cur, nq);
  const PacketSpill sp0{tasks, counts, kRangeTaskCap, first, counts + kRangePasses, tail_from};
  if (fill)
    k_count_packet<D, Q, true><<<grid, 64 * kPWaves, smem, stream>>>(v, src, nq, order, d_count,
                                                                     leaf, sp0, fo);
  else
    k_count_packet<D, Q, false><<<grid, 64 * kPWaves, smem, stream>>>(v, src, nq, order, d_count,
                                                                      leaf, sp0, fo);
  for (int pass = 1; pass < kRangePasses; ++pass) {
    const bool last = pass == kRangePasses - 1;
    const PacketSpill out = last ? PacketSpill{nullptr, nullptr, 0u, 0u, nullptr, 0u}
                                : PacketSpill{tasks + (size_t)pass * kRangeTaskCap, counts + pass,
                                             kRangeTaskCap, later, nullptr, 0u};
    const PacketTask* in = tasks + (size_t)(pass - 1) * kRangeTaskCap;
    if (fill)
      k_count_tasks<D, Q, true><<<kRangeTaskBlocks, 64 * kPWaves, smem, stream>>>(
          v, src, nq, order, d_count, leaf, in, counts + pass - 1, kRangeTaskCap, out, fo);
    else
      k_count_tasks<D, Q, false><<<kRangeTaskBlocks, 64 * kPWaves, smem, stream>>>(
          v, src, nq, order, d_count, leaf, in, counts + pass - 1, kRangeTaskCap, out, fo);
  }
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("%s: packet kernel launch failed", who);
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

template <int D>
kdt_status range_packet_launch(const TreeView& v, int leaf, const float* d_q, int64_t nq, float r2,
                               const int32_t* order, int32_t* d_count, uint32_t split_budget,
                               hipStream_t stream, const FillOut* fill) {
  return count_packet_launch<D>(v, leaf, BallQueries<D>{d_q, r2}, nq, order, d_count,
                                split_budget, stream, "kdt_range", fill);
}

template <int D>
kdt_status box_packet_launch(const TreeView& v, int leaf, const float* d_lo, const float* d_hi,
                             int64_t nq, const int32_t* order, int32_t* d_count,
                             uint32_t split_budget, hipStream_t stream, const FillOut* fill) {
  return count_packet_launch<D>(v, leaf, BoxQueries<D>{d_lo, d_hi}, nq, order, d_count,
                                split_budget, stream, "kdt_box", fill);
}

template <int D>
kdt_status torus_range_packet_launch(const TreeView& v, int leaf, const float* d_q, int64_t nq,
                                     float r2, const Torus<D>& T, const int32_t* order,
                                     int32_t* d_count, uint32_t split_budget,
                                     hipStream_t stream, const FillOut* fill) {
  return count_packet_launch<D>(v, leaf, TorusBallQueries<D>{d_q, r2, T}, nq, order, d_count,
                                split_budget, stream, "kdt_range", fill);
}

template <int D, class Metric>
kdt_status var_ball_count_launch(const TreeView& v, int leaf, const float* d_q, const float* d_r2,
                                 int64_t nq, const int32_t* order, const Metric& m,
                                 int32_t* d_count, hipStream_t stream) {
  return count_packet_launch<D>(v, leaf, VarBallQueries<D, Metric>{d_q, d_r2, m}, nq, order,
                                d_count, 0u, stream, "kdt_knn");
}

#define KDT_INST(D)                                                                                \
  template kdt_status knn_packet_launch<D>(const TreeView&, int, const float*, int64_t, int,       \
                                           int32_t*, float*, int, const int32_t*, hipStream_t);    \
  template kdt_status range_packet_launch<D>(const TreeView&, int, const float*, int64_t, float,   \
                                             const int32_t*, int32_t*, uint32_t, hipStream_t,    \
                                             const FillOut*);                                    \
  template kdt_status box_packet_launch<D>(const TreeView&, int, const float*, const float*,       \
                                           int64_t, const int32_t*, int32_t*, uint32_t,          \
                                           hipStream_t, const FillOut*);                         \
  template kdt_status fof_packet_launch<D>(const TreeView&, int, float, int32_t*, uint32_t*,       \
                                           hipStream_t);                                         \
  template kdt_status torus_range_packet_launch<D>(const TreeView&, int, const float*, int64_t,    \
                                                   float, const Torus<D>&, const int32_t*,       \
                                                   int32_t*, uint32_t, hipStream_t,              \
                                                   const FillOut*);                              \
  template kdt_status torus_fof_packet_launch<D>(const TreeView&, int, float, const Torus<D>&,     \
                                                 int32_t*, uint32_t*, hipStream_t);              \
  template kdt_status var_ball_count_launch<D, OpenMetric<D>>(                                     \
      const TreeView&, int, const float*, const float*, int64_t, const int32_t*,                  \
      const OpenMetric<D>&, int32_t*, hipStream_t);                                               \
  template kdt_status var_ball_count_launch<D, TorusMetric<D>>(                                    \
      const TreeView&, int, const float*, const float*, int64_t, const int32_t*,                  \
      const TorusMetric<D>&, int32_t*, hipStream_t);
KDT_INST(2)
KDT_INST(3)
KDT_INST(4)
KDT_INST(8)
KDT_INST(16)
#undef KDT_INST

}  // namespace kdt
