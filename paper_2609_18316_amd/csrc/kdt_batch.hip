// kdt_batch.hip -- many independent point sets of uneven size in one batch.
//
// A batch plan fixes every shape on the host: the forest schedule (each level
// kernel of the build covers the nodes of every set at that level, so a level
// costs one launch for the whole batch), all buffers, and persistent
// work-queue kernels for the queries: workgroups take packets of 128
// consecutive points from a device counter until the batch is exhausted; each
// lane finds its set and runs the same traversal as the single-tree kernels.
// The pipeline (build, kNN of every point, friends-of-friends) is captured
// once into a hipGraph and replayed.  Mode 0 is the baseline: the single-tree
// entry points called once per set, eagerly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "kdt_packet.h"

namespace kdt {

constexpr int kBQ = 128;

__device__ __forceinline__ int find_set(const SetDesc* __restrict__ sets, int n_sets, int64_t row) {
  int lo = 0, hi = n_sets - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sets[mid].off <= row) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int D>
__device__ __forceinline__ TreeView set_view(const SetDesc& sd, const float* rec, const float* box) {
  TreeView t;
  t.rec = rec + sd.off * rec_stride(D);
  t.box = box + sd.node_base * 2 * pad4(D);
  t.n = sd.n;
  t.levels = sd.levels;
  return t;
}

__device__ __forceinline__ int64_t next_packet(unsigned long long* ctr, int64_t* slot) {
  if (threadIdx.x == 0) *slot = (int64_t)atomicAdd(ctr, 1ull);
  __syncthreads();
  const int64_t p = *slot;
  __syncthreads();
  return p;
}

template <int D, int KC>
__global__ __launch_bounds__(kBQ) void k_knn_forest(const SetDesc* __restrict__ sets, int n_sets,
                                                    const float* __restrict__ rec,
                                                    const float* __restrict__ box, int64_t total,
                                                    int k, int32_t* __restrict__ oidx,
                                                    float* __restrict__ od2,
                                                    unsigned long long* __restrict__ ctr) {
  __shared__ uint32_t stk[kMaxDepth][kBQ];
  __shared__ int64_t slot;
  const int64_t n_packets = (total + kBQ - 1) / kBQ;
  for (;;) {
    const int64_t pk = next_packet(ctr, &slot);
    if (pk >= n_packets) break;
    const int64_t row = pk * kBQ + threadIdx.x;
    if (row < total) {
      const SetDesc sd = sets[find_set(sets, n_sets, row)];
      const TreeView t = set_view<D>(sd, rec, box);
      float q[D];
      int32_t id = 0;
      load_rec<D>(t.rec, row - sd.off, q, id);
      TopK<KC> best;
      best.init(k);
      knn_one<D>(t, q, best, &stk[0][threadIdx.x], kBQ);
      knn_write<KC>(best, k, 0, sd.off + id, oidx, od2);
    }
  }
}

// Persistent wave-level work queue over packets of 64 consecutive points of
// one set (packets never straddle sets, so a wave always walks one tree).
template <int D, int KC>
__global__ __launch_bounds__(256) void k_knn_forest_packet(
    const SetDesc* __restrict__ sets, int n_sets, const int64_t* __restrict__ pbase,
    const float* __restrict__ rec, const float* __restrict__ box, int k, int leaf_cap,
    int32_t* __restrict__ oidx, float* __restrict__ od2, unsigned long long* __restrict__ ctr) {
  extern __shared__ __align__(16) float lds[];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  float* slice = lds + (size_t)wave * knn_wave_floats<D>(leaf_cap);
  const int64_t n_packets = pbase[n_sets];
  for (;;) {
    unsigned long long got = 0;
    if (lane == 0) got = atomicAdd(ctr, 1ull);
    const int64_t pk = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(got >> 32)) << 32) |
                                 (uint32_t)__builtin_amdgcn_readfirstlane((int)got));
    if (pk >= n_packets) break;
    int lo = 0, hi = n_sets - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pbase[mid] <= pk) lo = mid;
      else hi = mid - 1;
    }
    const SetDesc sd = sets[lo];
    const TreeView t = set_view<D>(sd, rec, box);
    const int64_t pos = (pk - pbase[lo]) * 64 + lane;
    const bool active = pos < sd.n;
    float q[D];
    int32_t id = 0;
    if (active) {
      load_rec<D>(t.rec, pos, q, id);
    } else {
#pragma unroll
      for (int a = 0; a < D; ++a) q[a] = 0.0f;
    }
    TopK<KC> best;
    best.init(k);
    packet_knn<D, KC>(t, q, active, best, slice, leaf_cap);
    if (active) knn_write<KC>(best, k, 0, sd.off + id, oidx, od2);
  }
}

// Friends-of-friends links over the same wave-level packet queue.
template <int D>
__global__ __launch_bounds__(256) void k_fof_forest_packet(
    const SetDesc* __restrict__ sets, int n_sets, const int64_t* __restrict__ pbase,
    const float* __restrict__ rec, const float* __restrict__ box,
    const float* __restrict__ lengths, int leaf_cap, int32_t* __restrict__ parent,
    uint32_t* __restrict__ conn, unsigned long long* __restrict__ ctr) {
  extern __shared__ __align__(16) float lds[];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  float* slice = lds + (size_t)wave * leaf_cap * rec_stride(D);
  const int64_t n_packets = pbase[n_sets];
  for (;;) {
    unsigned long long got = 0;
    if (lane == 0) got = atomicAdd(ctr, 1ull);
    const int64_t pk = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(got >> 32)) << 32) |
                                 (uint32_t)__builtin_amdgcn_readfirstlane((int)got));
    if (pk >= n_packets) break;
    int lo = 0, hi = n_sets - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pbase[mid] <= pk) lo = mid;
      else hi = mid - 1;
    }
    const SetDesc sd = sets[lo];
    const TreeView t = set_view<D>(sd, rec, box);
    const float l = lengths[lo];
    const float l2 = l * l;
    const int64_t pos = (pk - pbase[lo]) * 64 + lane;
    const bool active = pos < sd.n;
    float q[D];
    int32_t me = 0;
    if (active) {
      load_rec<D>(t.rec, pos, q, me);
    } else {
#pragma unroll
      for (int a = 0; a < D; ++a) q[a] = 0.0f;
    }
    packet_fof<D>(t, q, pos, me, active, l2, (int32_t)sd.off, parent, conn + sd.node_base, slice);
  }
}

__global__ void k_iota_i32(int32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

template <int D>
__global__ void k_fof_forest_mark(const SetDesc* __restrict__ sets, int n_sets,
                                  const float* __restrict__ box, int64_t n_nodes,
                                  const float* __restrict__ lengths, uint32_t* __restrict__ conn) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_nodes) return;
  int lo = 0, hi = n_sets - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sets[mid].node_base <= v) lo = mid;
    else hi = mid - 1;
  }
  const float l = lengths[lo];
  fof_mark_clique<D>(box, v, l * l, conn);
}

template <int D>
__global__ void k_fof_forest_join(const SetDesc* __restrict__ sets, int n_sets,
                                  const float* __restrict__ rec, const float* __restrict__ box,
                                  int64_t total, int32_t* __restrict__ parent,
                                  const uint32_t* __restrict__ conn) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= total) return;
  const SetDesc sd = sets[find_set(sets, n_sets, row)];
  const TreeView t = set_view<D>(sd, rec, box);
  const int64_t pos = row - sd.off;
  fof_join_clique<D>(t, pos, __float_as_int(t.rec[pos * rec_stride(D) + D]), (int32_t)sd.off,
                     parent, conn + sd.node_base);
}

template <int D>
__global__ __launch_bounds__(kBQ) void k_fof_forest(const SetDesc* __restrict__ sets, int n_sets,
                                                    const float* __restrict__ rec,
                                                    const float* __restrict__ box, int64_t total,
                                                    const float* __restrict__ lengths,
                                                    int32_t* __restrict__ parent,
                                                    uint32_t* __restrict__ conn,
                                                    unsigned long long* __restrict__ ctr) {
  __shared__ uint32_t stk[kMaxDepth][kBQ];
  __shared__ int64_t slot;
  const int64_t n_packets = (total + kBQ - 1) / kBQ;
  for (;;) {
    const int64_t pk = next_packet(ctr, &slot);
    if (pk >= n_packets) break;
    const int64_t row = pk * kBQ + threadIdx.x;
    if (row < total) {
      const int s = find_set(sets, n_sets, row);
      const SetDesc sd = sets[s];
      const TreeView t = set_view<D>(sd, rec, box);
      const float l = lengths[s];
      const float l2 = l * l;
      float q[D];
      int32_t me = 0;
      const int64_t pos = row - sd.off;
      load_rec<D>(t.rec, pos, q, me);
      fof_point<D>(t, q, pos, me, l2, (int32_t)sd.off, parent, conn + sd.node_base,
                   &stk[0][threadIdx.x], kBQ);
    }
  }
}

__global__ void k_fof_forest_final(const SetDesc* __restrict__ sets, int n_sets,
                                   const int32_t* __restrict__ parent, int64_t total,
                                   int32_t* __restrict__ labels) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const SetDesc sd = sets[find_set(sets, n_sets, i)];
  labels[i] = uf_root(parent, (int32_t)i) - (int32_t)sd.off;
}

}  // namespace kdt

using namespace kdt;

struct kdt_batch_plan {
  Plan plan;
  PlanDev dev;
  int d = 0, k = 0, leaf = 0;  // leaf: the largest N_leaf of the sets
  std::vector<int> leaves;     // N_leaf of each set
  bool knn_packets = false;  // wave-packet kNN instead of one query per lane
  std::vector<int64_t> offsets;
  BuildScratch w;
  void* tree_block = nullptr;
  BuildOut out{};
  int32_t* parent = nullptr;
  uint32_t* conn = nullptr;
  int64_t* pbase = nullptr;  // first packet of each set, [n_sets + 1]
  unsigned long long* ctr = nullptr;
  int knn_blocks = 0, fof_blocks = 0;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  const void* key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

// LDS of a 4-wave workgroup of the forest packet kernels (a leaf slice per
// wave).
template <int D>
static size_t forest_lds_bytes(int leaf) {
  return sizeof(float) * (size_t)leaf * rec_stride(D) * 4;
}

template <int D, int KC>
static int occupancy_blocks(const void* fn, size_t smem, int block) {
  int per_cu = 0, dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, smem);
  return std::max(1, per_cu) * std::max(1, cus);
}

template <int D>
static kdt_status forest_queries(kdt_batch_plan* bp, const float* d_l, int32_t* d_idx,
                                 float* d_d2, int32_t* d_labels, hipStream_t s) {
  const Plan& p = bp->plan;
  const int ns = (int)p.sets.size();
  const int64_t tot = p.total;
  k_zero_u64<<<1, 64, 0, s>>>(bp->ctr, 2);
  const int k = bp->k;
  if (bp->knn_packets) {
    const unsigned g = (unsigned)bp->knn_blocks;
    const size_t smem = sizeof(float) * knn_wave_floats<D>(bp->leaf) * 4;
    if (k <= 8)
      k_knn_forest_packet<D, 8><<<g, 256, smem, s>>>(bp->dev.sets, ns, bp->pbase, bp->out.rec, bp->out.box, k, bp->leaf, d_idx, d_d2, bp->ctr);
    else if (k <= 16)
      k_knn_forest_packet<D, 16><<<g, 256, smem, s>>>(bp->dev.sets, ns, bp->pbase, bp->out.rec, bp->out.box, k, bp->leaf, d_idx, d_d2, bp->ctr);
    else if (k <= 32)
      k_knn_forest_packet<D, 32><<<g, 256, smem, s>>>(bp->dev.sets, ns, bp->pbase, bp->out.rec, bp->out.box, k, bp->leaf, d_idx, d_d2, bp->ctr);
    else
      k_knn_forest_packet<D, 64><<<g, 256, smem, s>>>(bp->dev.sets, ns, bp->pbase, bp->out.rec, bp->out.box, k, bp->leaf, d_idx, d_d2, bp->ctr);
  } else if (k <= 8)
    k_knn_forest<D, 8><<<bp->knn_blocks, kBQ, 0, s>>>(bp->dev.sets, ns, bp->out.rec, bp->out.box,
                                                      tot, k, d_idx, d_d2, bp->ctr);
  else if (k <= 16)
    k_knn_forest<D, 16><<<bp->knn_blocks, kBQ, 0, s>>>(bp->dev.sets, ns, bp->out.rec, bp->out.box,
                                                       tot, k, d_idx, d_d2, bp->ctr);
  else if (k <= 32)
    k_knn_forest<D, 32><<<bp->knn_blocks, kBQ, 0, s>>>(bp->dev.sets, ns, bp->out.rec, bp->out.box,
                                                       tot, k, d_idx, d_d2, bp->ctr);
  else
    k_knn_forest<D, 64><<<bp->knn_blocks, kBQ, 0, s>>>(bp->dev.sets, ns, bp->out.rec, bp->out.box,
                                                       tot, k, d_idx, d_d2, bp->ctr);
  const unsigned g = (unsigned)((tot + 255) / 256);
  k_iota_i32<<<g, 256, 0, s>>>(bp->parent, tot);
  const unsigned gn = (unsigned)((p.n_nodes + 255) / 256);
  k_fof_forest_mark<D><<<gn, 256, 0, s>>>(bp->dev.sets, ns, bp->out.box, p.n_nodes, d_l, bp->conn);
  k_fof_forest_join<D><<<g, 256, 0, s>>>(bp->dev.sets, ns, bp->out.rec, bp->out.box, tot,
                                         bp->parent, bp->conn);
  if (bp->leaf <= 64) {
    k_fof_forest_packet<D><<<bp->fof_blocks, 256, forest_lds_bytes<D>(bp->leaf), s>>>(
        bp->dev.sets, ns, bp->pbase, bp->out.rec, bp->out.box, d_l, bp->leaf, bp->parent, bp->conn,
        bp->ctr + 1);
  } else {
    k_fof_forest<D><<<bp->fof_blocks, kBQ, 0, s>>>(bp->dev.sets, ns, bp->out.rec, bp->out.box, tot,
                                                   d_l, bp->parent, bp->conn, bp->ctr + 1);
  }
  k_fof_forest_final<<<g, 256, 0, s>>>(bp->dev.sets, ns, bp->parent, tot, d_labels);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_batch_launch: kernel launch failed");
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

static kdt_status forest_pipeline(kdt_batch_plan* bp, const float* d_pts, const float* d_l,
                                  int32_t* d_idx, float* d_d2, int32_t* d_labels, hipStream_t s) {
  kdt_status st = build_launch(bp->plan, bp->dev, d_pts, bp->w, bp->out, 0, s);
  if (st == KDT_OK) st = build_launch(bp->plan, bp->dev, d_pts, bp->w, bp->out, 1, s);
  if (st != KDT_OK) return st;
  switch (bp->d) {
    case 2: return forest_queries<2>(bp, d_l, d_idx, d_d2, d_labels, s);
    case 3: return forest_queries<3>(bp, d_l, d_idx, d_d2, d_labels, s);
    case 4: return forest_queries<4>(bp, d_l, d_idx, d_d2, d_labels, s);
    case 8: return forest_queries<8>(bp, d_l, d_idx, d_d2, d_labels, s);
    case 16: return forest_queries<16>(bp, d_l, d_idx, d_d2, d_labels, s);
  }
  return KDT_EUNSUPPORTED;
}

template <int D>
static void size_grids(kdt_batch_plan* bp) {
  const void* kf = nullptr;
  const size_t smem = bp->leaf <= 64 ? forest_lds_bytes<D>(bp->leaf) : 0;
  const size_t knn_smem = bp->leaf <= 64 ? sizeof(float) * knn_wave_floats<D>(bp->leaf) * 4 : 0;
  if (bp->knn_packets) {
    if (bp->k <= 8) kf = reinterpret_cast<const void*>(&k_knn_forest_packet<D, 8>);
    else if (bp->k <= 16) kf = reinterpret_cast<const void*>(&k_knn_forest_packet<D, 16>);
    else if (bp->k <= 32) kf = reinterpret_cast<const void*>(&k_knn_forest_packet<D, 32>);
    else kf = reinterpret_cast<const void*>(&k_knn_forest_packet<D, 64>);
    bp->knn_blocks = occupancy_blocks<D, 0>(kf, knn_smem, 256);
  } else {
    if (bp->k <= 8) kf = reinterpret_cast<const void*>(&k_knn_forest<D, 8>);
    else if (bp->k <= 16) kf = reinterpret_cast<const void*>(&k_knn_forest<D, 16>);
    else if (bp->k <= 32) kf = reinterpret_cast<const void*>(&k_knn_forest<D, 32>);
    else kf = reinterpret_cast<const void*>(&k_knn_forest<D, 64>);
    bp->knn_blocks = occupancy_blocks<D, 0>(kf, 0, kBQ);
  }
  if (bp->leaf <= 64)
    bp->fof_blocks = occupancy_blocks<D, 0>(reinterpret_cast<const void*>(&k_fof_forest_packet<D>), smem, 256);
  else
    bp->fof_blocks = occupancy_blocks<D, 0>(reinterpret_cast<const void*>(&k_fof_forest<D>), 0, kBQ);
}

static void release(kdt_batch_plan* bp) {
  if (bp->exec) (void)hipGraphExecDestroy(bp->exec);
  if (bp->graph) (void)hipGraphDestroy(bp->graph);
  if (bp->cap) (void)hipStreamDestroy(bp->cap);
  build_scratch_free(bp->w, kPlainAlloc);
  if (bp->tree_block) (void)hipFree(bp->tree_block);
  if (bp->parent) (void)hipFree(bp->parent);
  if (bp->conn) (void)hipFree(bp->conn);
  if (bp->pbase) (void)hipFree(bp->pbase);
  if (bp->ctr) (void)hipFree(bp->ctr);
  plan_release(bp->dev);
}

extern "C" kdt_status kdt_batch_plan_create(const int64_t* h_offsets, int32_t n_sets, int32_t d,
                                            int32_t k, const kdt_build_opts* bopts,
                                            const kdt_query_opts* qopts, kdt_batch_plan** out) {
  kdt_clear_error();
  if (!out || !h_offsets || n_sets < 1) {
    kdt_set_error("kdt_batch_plan_create: NULL argument or no sets");
    return KDT_EINVAL;
  }
  *out = nullptr;
  if (!(d == 2 || d == 3 || d == 4 || d == 8 || d == 16)) {
    kdt_set_error("kdt_batch_plan_create: dimension %d is not one of 2, 3, 4, 8, 16", d);
    return KDT_EUNSUPPORTED;
  }
  if (k < 1 || k > KDT_MAX_K) {
    kdt_set_error("kdt_batch_plan_create: k=%d outside [1, %d]", k, KDT_MAX_K);
    return k < 1 ? KDT_EINVAL : KDT_EUNSUPPORTED;
  }
  if (bopts && bopts->split_rule != 0) {
    kdt_set_error("kdt_batch_plan_create: the batched forest is built with median splits only");
    return KDT_EUNSUPPORTED;
  }
  if (h_offsets[0] != 0 || h_offsets[n_sets] > INT32_MAX) {
    kdt_set_error("kdt_batch_plan_create: offsets must start at 0 and total below 2^31");
    return KDT_EINVAL;
  }
  const int given_leaf = bopts ? bopts->leaf_size : 0;
  if (given_leaf != 0 && (given_leaf < 2 || given_leaf > 256)) {
    kdt_set_error("kdt_batch_plan_create: leaf_size %d outside [2, 256]", given_leaf);
    return KDT_EINVAL;
  }
  // leaf_size 0: each set takes the tuned N_leaf of its own size
  std::vector<int> leaves((size_t)n_sets);
  for (int s = 0; s < n_sets; ++s)
    leaves[s] = given_leaf ? given_leaf : tuned(d, h_offsets[s + 1] - h_offsets[s], k).leaf;
  const int leaf = *std::max_element(leaves.begin(), leaves.end());
  kdt_batch_plan* bp = new (std::nothrow) kdt_batch_plan();
  if (!bp) {
    kdt_set_error("kdt_batch_plan_create: out of host memory");
    return KDT_ENOMEM;
  }
  bp->d = d;
  bp->k = k;
  bp->leaf = leaf;
  bp->leaves = leaves;
  // traversal 0 picks the measured default: wave packets (for the batch's
  // all-points kNN they beat one query per lane: the whole 256-set clustered
  // pipeline at k = 8 takes 57.1 ms with them, 65.4 ms without)
  const int trav = qopts ? qopts->traversal : 0;
  bp->knn_packets = leaf <= 64 && trav != 1;
  bp->offsets.assign(h_offsets, h_offsets + n_sets + 1);
  std::string err;
  if (!make_plan(h_offsets, n_sets, d, leaves.data(), bp->plan, err)) {
    delete bp;
    kdt_set_error("kdt_batch_plan_create: %s", err.c_str());
    return KDT_EINVAL;
  }
  kdt_status st = plan_upload(bp->plan, bp->dev, nullptr);
  if (st == KDT_OK) st = build_scratch_alloc(bp->plan, bp->dev, bp->w, kPlainAlloc);
  const int64_t tot = bp->plan.total;
  const size_t b_rec = sizeof(float) * (size_t)tot * rec_stride(d);
  const size_t b_box = sizeof(float) * (size_t)bp->plan.n_nodes * 2 * pad4(d);
  const size_t b_perm = sizeof(int32_t) * (size_t)tot;
  const size_t b_axis = sizeof(int32_t) * (size_t)bp->plan.n_nodes;
  const size_t b_split = sizeof(float) * (size_t)bp->plan.n_nodes;
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  if (st == KDT_OK &&
      (hipMalloc(&bp->tree_block, up(b_rec) + up(b_box) + up(b_perm) + up(b_axis) + up(b_split)) !=
           hipSuccess ||
       hipMalloc((void**)&bp->parent, sizeof(int32_t) * std::max<int64_t>(tot, 1)) != hipSuccess ||
       hipMalloc((void**)&bp->conn, sizeof(uint32_t) * std::max<int64_t>(bp->plan.n_nodes, 1)) !=
           hipSuccess ||
       hipMalloc((void**)&bp->ctr, 256) != hipSuccess)) {
    kdt_set_error("kdt_batch_plan_create: device allocation failed (%lld points)", (long long)tot);
    st = KDT_ENOMEM;
  }
  if (st == KDT_OK) {
    std::vector<int64_t> pb(n_sets + 1, 0);
    for (int i = 0; i < n_sets; ++i) pb[i + 1] = pb[i] + (h_offsets[i + 1] - h_offsets[i] + 63) / 64;
    if (hipMalloc((void**)&bp->pbase, sizeof(int64_t) * (n_sets + 1)) != hipSuccess ||
        hipMemcpy(bp->pbase, pb.data(), sizeof(int64_t) * (n_sets + 1), hipMemcpyHostToDevice) !=
            hipSuccess) {
      kdt_set_error("kdt_batch_plan_create: cannot upload the packet table");
      st = KDT_ENOMEM;
    }
  }
  if (st == KDT_OK && hipStreamCreateWithFlags(&bp->cap, hipStreamNonBlocking) != hipSuccess) {
    kdt_set_error("kdt_batch_plan_create: cannot create the capture stream");
    st = KDT_EDEVICE;
  }
  if (st != KDT_OK) {
    release(bp);
    delete bp;
    return st;
  }
  unsigned char* b = static_cast<unsigned char*>(bp->tree_block);
  bp->out.rec = reinterpret_cast<float*>(b);
  bp->out.box = reinterpret_cast<float*>(b + up(b_rec));
  bp->out.perm = reinterpret_cast<int32_t*>(b + up(b_rec) + up(b_box));
  bp->out.axis = reinterpret_cast<int32_t*>(b + up(b_rec) + up(b_box) + up(b_perm));
  bp->out.split = reinterpret_cast<float*>(b + up(b_rec) + up(b_box) + up(b_perm) + up(b_axis));
  switch (d) {
    case 2: size_grids<2>(bp); break;
    case 3: size_grids<3>(bp); break;
    case 4: size_grids<4>(bp); break;
    case 8: size_grids<8>(bp); break;
    case 16: size_grids<16>(bp); break;
  }
  build_init_once();
  *out = bp;
  return KDT_OK;
}

static kdt_status eager_per_set(kdt_batch_plan* bp, const float* d_pts, const float* d_l,
                                int32_t* d_idx, float* d_d2, int32_t* d_labels, hipStream_t s) {
  const int ns = (int)bp->offsets.size() - 1;
  std::vector<float> lens(ns);
  if (hipMemcpyAsync(lens.data(), d_l, sizeof(float) * ns, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    kdt_set_error("kdt_batch_launch: reading linking lengths failed");
    return KDT_EDEVICE;
  }
  std::vector<kdt_tree*> trees(ns, nullptr);
  kdt_status st = KDT_OK;
  for (int i = 0; i < ns && st == KDT_OK; ++i) {
    const int64_t off = bp->offsets[i], n = bp->offsets[i + 1] - off;
    kdt_build_opts bo{bp->leaves[i], 0, 0, 0};
    st = kdt_build(d_pts + off * bp->d, n, bp->d, &bo, s, &trees[i]);
    if (st == KDT_OK)
      st = kdt_knn(trees[i], nullptr, n, bp->k, d_idx + off * bp->k, d_d2 + off * bp->k, 0, nullptr, s);
    if (st == KDT_OK) st = kdt_fof(trees[i], lens[i], d_labels + off, nullptr, s);
  }
  for (kdt_tree* t : trees)
    if (t) kdt_free(t);
  return st;
}

extern "C" kdt_status kdt_batch_launch(kdt_batch_plan* bp, const float* d_pts, const float* d_l,
                                       int32_t* d_idx, float* d_d2, int32_t* d_labels,
                                       int32_t use_graph, hipStream_t stream) {
  kdt_clear_error();
  if (!bp || !d_pts || !d_l || !d_idx || !d_d2 || !d_labels) {
    kdt_set_error("kdt_batch_launch: NULL argument");
    return KDT_EINVAL;
  }
  if (use_graph == 0) return eager_per_set(bp, d_pts, d_l, d_idx, d_d2, d_labels, stream);
  if (use_graph == 2) return forest_pipeline(bp, d_pts, d_l, d_idx, d_d2, d_labels, stream);
  const void* key[5] = {d_pts, d_l, d_idx, d_d2, d_labels};
  if (!bp->exec || memcmp(key, bp->key, sizeof(key)) != 0) {
    if (bp->exec) {
      (void)hipGraphExecDestroy(bp->exec);
      bp->exec = nullptr;
    }
    if (bp->graph) {
      (void)hipGraphDestroy(bp->graph);
      bp->graph = nullptr;
    }
    if (hipStreamBeginCapture(bp->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      kdt_set_error("kdt_batch_launch: cannot start graph capture");
      return KDT_EDEVICE;
    }
    kdt_status st = forest_pipeline(bp, d_pts, d_l, d_idx, d_d2, d_labels, bp->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(bp->cap, &g);
    if (st != KDT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess || !g || hipGraphInstantiate(&bp->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      kdt_set_error("kdt_batch_launch: graph capture failed: %s", hipGetErrorString(e));
      return KDT_EDEVICE;
    }
    bp->graph = g;
    memcpy(bp->key, key, sizeof(key));
  }
  if (hipGraphLaunch(bp->exec, stream) != hipSuccess) {
    kdt_set_error("kdt_batch_launch: graph launch failed");
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

extern "C" kdt_status kdt_batch_plan_free(kdt_batch_plan* bp) {
  kdt_clear_error();
  if (!bp) return KDT_OK;
  (void)hipDeviceSynchronize();
  release(bp);
  delete bp;
  return KDT_OK;
}
