// kdt_packet.h -- wave-coherent traversals shared by the single-tree and the
// batched kernels (gfx950, wave64).
//
// A wave of 64 spatially coherent queries walks one tree together.  The node
// stack is held in the wave's lane registers (entry i lives in lane i, popped
// with readlane), so it costs no memory.  A node is entered when at least one
// lane needs it (wave ballot); its box sits at a wave-uniform address and is
// read with scalar loads, one load serving 64 queries.
#pragma once

#include "kdt_query.h"

namespace kdt {

// A visited leaf (wave-uniform) is copied once into the wave's LDS slice
// (`lds`, at least 64 records) with one coalesced load, then its points are
// read back as LDS broadcasts, several in flight.  (Reading the points with
// scalar loads straight from the records was measured slower at every d:
// each batch waits on the scalar cache, which the waves' leaves overflow --
// ball counts 22.5 against 17.1 ms on the clustered workload.)
template <int D>
struct LeafReader {
  static constexpr int S = rec_stride(D);
  const float* rec;
  float* lds;
  int64_t b = 0;  // first record of the open leaf
  __device__ __forceinline__ LeafReader(const float* r, float* l) : rec(r), lds(l) {}
  // Called by the whole wave with a wave-uniform leaf.
  __device__ __forceinline__ void open(int64_t first, int cnt) {
    b = first;
    wave_sync();  // every lane is done with the previous leaf
    const float4* src = reinterpret_cast<const float4*>(rec + first * S);
    float4* dst = reinterpret_cast<float4*>(lds);
    for (int i = lane_id(); i < cnt * (S / 4); i += 64) dst[i] = src[i];
    wave_sync();
  }
  // Point i of the open leaf (i wave-uniform: a broadcast).
  __device__ __forceinline__ void point(int i, float x[D]) const {
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = lds[i * S + a];
  }
  // The input index of point i of the open leaf.
  __device__ __forceinline__ int32_t index(int i) const { return __float_as_int(lds[i * S + D]); }
  // Point i of the open leaf and its index, i per lane.
  __device__ __forceinline__ void lane_point(int i, float x[D], int32_t& id) const {
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = lds[i * S + a];
    id = __float_as_int(lds[i * S + D]);
  }
};

// ---------------------------------------------------------------------------
// Matrix-core filter for the leaf scan of the wave kNN (d = 8, 16)
// ---------------------------------------------------------------------------
//
// In high dimension almost every leaf is visited and the scan -- 64 queries
// against up to 64 points -- is a dense contraction.  The filter computes
// every query-point dot product on the matrix cores and marks point i for
// query q.
//
// Everything is first moved to a centre c, the wave's first active query
// (wave-uniform): q' = fl(q - c), p' = fl(p - c), in float32.  Each operand
// value v is then split into two bf16 values, v_hi = bf16(v) (round to
// nearest even) and v_lo = bf16(v - v_hi) (v - v_hi is exact in float32),
// and the dot product is taken as three bf16 products accumulated in float32
// (v_mfma_f32_16x16x16_bf16: q_hi.p_hi + q_hi.p_lo + q_lo.p_hi, the 16
// coordinates of a block in one step; d = 8 pads with zeros).  With
// s = |q'|^2 + |p'|^2 (computed in float32), point i is marked when
//   !( (1 - 2^-13) s - 2 q'.p'  >  (1 + 2^-16) worst_q + 2^-100 )  or  !(s < 2^125),
// worst_q being the query's current k-th squared distance.
//
// Why no candidate is lost.  With u_b = 2^-8 (bf16) the split leaves
// |v - v_hi - v_lo| <= u_b^2 |v| and |v_lo| <= u_b (1 + u_b) |v|, so per axis
// |q'p' - (q_hi p_hi + q_hi p_lo + q_lo p_hi)| <= 3.01 * 2^-16 |q'||p'|, and
// over the axes 3.01 * 2^-16 |q'||p'| <= 1.51 * 2^-16 s.  The 48 products are
// exact in float32; their accumulation in any order adds at most 48 u of
// their absolute sum, 0.1 * 2^-16 s (u = 2^-24).  So 2 q'.p' is within
// 3.22 * 2^-16 s.  The rest of the test (norms, combination, the recentring
// that moves each axis of q' - p' by at most u (|q'_a| + |p'_a|), and the
// exact float32 distance of the insertion pass) stays within (3d + 14) u s
// and (d + 2) u worst, below 0.25 * 2^-16 s at d = 16.  The relative
// margins are 8 * 2^-16 of s and 2^-16 of worst, so more than twice the
// total.  Operands a matrix core flushes to zero (bf16 or float32 values
// below 2^-126) change the dot product by at most 2^-123 max(1, s), covered
// by the 2^-100 absolute term and the relative margin.  While s < 2^125 no
// partial sum overflows; at or above it, or with any value NaN (a split of
// an infinite value gives one), the point is marked without a test.  So
// every point that can enter the list is marked, and the insertion pass,
// which recomputes the exact distance from the original coordinates, keeps
// the results bit-identical.  The centre keeps s near the squared size of
// the region the wave works in, so far from the origin (coordinates of
// 1e18 and beyond) the filter still prunes instead of marking everything.
//
// MFMA lane layout (16x16x16 bf16, checked on the device): lane l supplies
// A[l % 16][4 (l / 16) + j] and B[4 (l / 16) + j][l % 16] for j = 0..3 and
// receives D[4 (l / 16) + r][l % 16] in register r.  Rows are leaf points,
// columns queries.

typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef short v4s_t __attribute__((ext_vector_type(4)));

// The bf16 bits of v rounded to nearest even (NaN to a quiet NaN, values
// past the bf16 range to infinity), as the high half of a float32.
__device__ __forceinline__ uint32_t bf16_rne_bits(float v) {
  const uint32_t u = __float_as_uint(v);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC00000u;
  return (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
}

// v = hi + lo + e with hi = bf16(v), lo = bf16(v - hi), |e| <= 2^-16 |v|.
__device__ __forceinline__ void split_bf16(float v, short& hi, short& lo) {
  const uint32_t h = bf16_rne_bits(v);
  const uint32_t l = bf16_rne_bits(v - __uint_as_float(h));
  hi = (short)(h >> 16);
  lo = (short)(l >> 16);
}

template <int D>
struct DotFilter {
  static constexpr bool kOn = D == 8 || D == 16;
  v4s_t bhi[4], blo[4];  // B operands: coordinates 4 (l / 16) + j of query 16 qj + l % 16, minus c
  float nq[4];           // |q - c|^2 of query 16 qj + l % 16
  float c[D];            // the centre (wave-uniform)
  float cs[4];           // c[4 (l / 16) + j]: the centre on this lane's operand slots (0 past d)
  float* np;             // LDS [64]: |p - c|^2 of the open leaf's points
  uint64_t* mb;          // LDS [4][4][16]: partial marks on their way to the query's lane

  // LDS of one wave: the leaf slice (also the query staging area), then np
  // and mb.  `leaf` is the tree's leaf size.
  __host__ __device__ static constexpr size_t slice_floats(int leaf) {
    return ((size_t)((leaf + 15) / 16 * 16) * rec_stride(D) > (size_t)64 * D
                ? (size_t)((leaf + 15) / 16 * 16) * rec_stride(D)
                : (size_t)64 * D);
  }
  __host__ __device__ static constexpr size_t wave_floats(int leaf) {
    return slice_floats(leaf) + 64 + 2 * 4 * 4 * 16;
  }

  // Called by the whole wave before any leaf is opened.
  __device__ __forceinline__ void init(const float p[D], bool active, float* lds, int leaf) {
    const int l = lane_id();
    float* stage = lds;
    np = lds + slice_floats(leaf);
    mb = reinterpret_cast<uint64_t*>(np + 64);
    const uint64_t am = __ballot(active);
    const int first = am ? __ffsll((unsigned long long)am) - 1 : 0;
    wave_sync();
#pragma unroll
    for (int a = 0; a < D; ++a) stage[l * D + a] = active ? p[a] : 0.0f;
    wave_sync();
#pragma unroll
    for (int a = 0; a < D; ++a)
      c[a] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(stage[first * D + a])));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 4 * (l >> 4) + j;
      cs[j] = k < D ? stage[first * D + k] : 0.0f;
    }
    float n2 = 0.0f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const float v = p[a] - c[a];
      n2 += v * v;
    }
    np[l] = active ? n2 : 0.0f;
    wave_sync();
#pragma unroll
    for (int qj = 0; qj < 4; ++qj) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 4 * (l >> 4) + j;
        const float v = k < D ? stage[(16 * qj + (l & 15)) * D + k] - cs[j] : 0.0f;
        short h, lo;
        split_bf16(v, h, lo);
        bhi[qj][j] = h;
        blo[qj][j] = lo;
      }
      nq[qj] = np[16 * qj + (l & 15)];
    }
    wave_sync();
  }

  // Marks of the open leaf (`leaf`: its LDS copy, `cnt` points) for this
  // lane's query, whose own threshold is `worst`.  Whole wave.
  __device__ __forceinline__ uint64_t marks(const float* leaf, int cnt, float worst) const {
    constexpr int S = rec_stride(D);
    const int l = lane_id();
    const float thr_own = worst * (1.0f + 0x1p-16f) + 0x1p-100f;
    float thr[4];
#pragma unroll
    for (int qj = 0; qj < 4; ++qj) thr[qj] = __shfl(thr_own, 16 * qj + (l & 15));
    float n2 = 0.0f;
    if (l < cnt) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const float v = leaf[l * S + a] - c[a];
        n2 += v * v;
      }
    }
    np[l] = n2;
    wave_sync();
    uint64_t m[4] = {0, 0, 0, 0};
#pragma unroll
    for (int pi = 0; pi < 4; ++pi) {
      if (16 * pi >= cnt) break;
      v4s_t ahi, alo;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 4 * (l >> 4) + j;
        const float v = k < D ? leaf[(16 * pi + (l & 15)) * S + k] - cs[j] : 0.0f;
        short h, lo;
        split_bf16(v, h, lo);
        ahi[j] = h;
        alo[j] = lo;
      }
      const int row0 = 16 * pi + 4 * (l >> 4);
      float npv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) npv[r] = np[row0 + r];
#pragma unroll
      for (int qj = 0; qj < 4; ++qj) {
        v4f_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo[qj], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi[qj], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi[qj], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float ns = nq[qj] + npv[r];
          const float lhs = ns * (1.0f - 0x1p-13f) - 2.0f * acc[r];
          // unordered compares (NaN) and norms too large to trust mark the point
          const bool mk = !(lhs > thr[qj]) || !(ns < 0x1p125f);
          m[qj] |= (uint64_t)mk << (row0 + r);
        }
      }
    }
#pragma unroll
    for (int qj = 0; qj < 4; ++qj) mb[(qj * 4 + (l >> 4)) * 16 + (l & 15)] = m[qj];
    wave_sync();
    uint64_t mine = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) mine |= mb[((l >> 4) * 4 + t) * 16 + (l & 15)];
    wave_sync();  // np and mb are rewritten by the next leaf
    return cnt < 64 ? mine & ((1ull << cnt) - 1) : mine;
  }
};

// LDS floats of one wave of the wave kNN.
template <int D>
__host__ __device__ constexpr size_t knn_wave_floats(int leaf) {
  // without the filter: the open leaf, then packed queries [64][D + 1]
  return DotFilter<D>::kOn ? DotFilter<D>::wave_floats(leaf)
                           : (size_t)leaf * rec_stride(D) + 64 * (D + 1);
}

// kNN of the 64 queries of a wave (Algorithm 2 semantics).  Each lane keeps its
// own register top-k keyed by (d2, index), so the result is exactly the k
// smallest keys, the same as any exact traversal.  Leaves must hold at most 64
// points.
// `lds` is the wave's slice of knn_wave_floats<D>(leaf_cap) floats.
//
// Below d = 8, a leaf that only a few lanes need (box within their k-th
// distance) is marked as (query, point) pairs of those lanes, packed in LDS
// as in the ball count; each lane's marks come back to it from the ballot of
// its slot.  A lane whose box test fails has no point within its k-th
// distance (the float box distance never exceeds a point's), so the marks are
// those of the scan over all lanes.
template <int D, int KC>
__device__ __forceinline__ void packet_knn(const TreeView& t, const float p[D], bool active,
                                           TopK<KC>& best, float* lds, int leaf_cap) {
  const int lane = lane_id();
  const uint32_t first_leaf = (1u << t.levels) - 1u;
  uint32_t stackv = 0;  // lane i holds stack entry i
  int sp = 1;
  uint64_t mask = 0;    // this lane's pending candidates in the open leaf
  LeafReader<D> leaf(t.rec, lds);
  DotFilter<D> filt;
  if constexpr (DotFilter<D>::kOn) filt.init(p, active, lds, leaf_cap);
  // One flat loop (the candidate list is then live across a single loop
  // header): a round either inserts one pending candidate per lane, or pops
  // and visits the next node.
  for (;;) {
    if (__any(mask != 0)) {
      const bool has = mask != 0;
      const int i = has ? __ffsll((unsigned long long)mask) - 1 : 0;
      mask &= mask - 1;
      float x[D];
      int32_t id = 0;
      leaf.lane_point(i, x, id);
      const uint64_t key = make_key(sq_dist<D>(x, p), id);
      best.insert(has && key < best.worst() ? key : kEmptyKey);
      continue;
    }
    if (sp == 0) break;
    --sp;
    const uint32_t node = (uint32_t)__builtin_amdgcn_readlane((int)stackv, sp);
    float lo[D], hi[D];
    load_box_uniform<D>(t.box, node, lo, hi);
    KDT_WAVE_VISIT(t, kVisitWaveNodes, 1);
    const bool need = active && box_mindist<D>(lo, hi, p) <= best.worst_d2();
    if (!__any(need)) continue;
    if (node >= first_leaf) {
      const int64_t j = node - first_leaf;
      const int64_t b = node_begin(t.n, t.levels, j), e = node_begin(t.n, t.levels, j + 1);
      const int cnt = (int)(e - b);
      leaf.open(b, cnt);
      KDT_WAVE_VISIT(t, kVisitWavePoints, cnt);
      // Mark the leaf points (at most 64) that beat this lane's current k-th
      // candidate; the rounds above then insert them, so the wave pays for
      // the largest per-lane count of insertions rather than for every point
      // some lane wants.
      // A float compare on d2 alone marks a superset of the candidates (it
      // keeps ties with the current k-th); the exact key test is repeated
      // before insertion.
      const float wd = best.worst_d2();
      if constexpr (DotFilter<D>::kOn) {
        mask = filt.marks(lds, cnt, wd);
        if (!active) mask = 0;
      } else {
        const uint64_t nm = __ballot(need);
        const int na = __popcll(nm);
        const int W = cnt <= 8 ? 8 : cnt <= 16 ? 16 : cnt <= 32 ? 32 : 64;
        const int G = 64 / W;
        const int steps = (na + G - 1) / G;
        if (2 * steps <= cnt) {  // a packed step costs about two broadcast steps
          float* cq = lds + (size_t)leaf_cap * rec_stride(D);  // [64][D + 1]: query, k-th d2
          const int me = lanes_below(nm);
          if (need) {
#pragma unroll
            for (int a = 0; a < D; ++a) cq[me * (D + 1) + a] = p[a];
            cq[me * (D + 1) + D] = wd;
          }
          wave_sync();
          const int slot = lane / W, i = lane % W;
          const uint64_t wmask = ~0ull >> (64 - W);
          float x[D];
          leaf.point(min(i, cnt - 1), x);
          uint64_t rem = nm;  // owners of the slots still to come, lowest first
          for (int s = 0; s < steps; ++s) {
            const int a = s * G + slot;
            const int ac = min(a, na - 1);
            float qv[D];
#pragma unroll
            for (int u = 0; u < D; ++u) qv[u] = cq[ac * (D + 1) + u];
            const float qw = cq[ac * (D + 1) + D];
            const uint64_t hm = __ballot(i < cnt && a < na && sq_dist<D>(x, qv) <= qw);
            for (int g = 0; g < G && rem != 0; ++g) {
              const int owner = __ffsll((unsigned long long)rem) - 1;
              rem &= rem - 1;
              const uint64_t bits = (hm >> (g * W)) & wmask;
              mask = lane == owner ? bits : mask;
            }
          }
          wave_sync();
        } else {
#pragma unroll uniform_batch<D>()
          for (int i = 0; i < cnt; ++i) {
            float x[D];
            leaf.point(i, x);
            mask |= (uint64_t)(sq_dist<D>(x, p) <= wd) << i;
          }
          if (!active) mask = 0;
        }
      }
    } else {
      const uint32_t c0 = 2 * node + 1, c1 = c0 + 1;
      KDT_WAVE_VISIT(t, kVisitWaveNodes, 2);
      load_box_uniform<D>(t.box, c0, lo, hi);
      const float d0 = box_mindist<D>(lo, hi, p);
      load_box_uniform<D>(t.box, c1, lo, hi);
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
}

// A subtree of the wave-shared ball count handed from
// one wave to a later pass: the 64-query group, the subtree's root and the
// lanes that still need it.
struct PacketTask {
  uint32_t group, node, lo, hi;
};
constexpr uint32_t kNoNode = 0xFFFFFFFFu;  // a reserved task slot left empty
constexpr uint32_t kSplitLevels = 2;       // subtrees of fewer leaves are never handed on

// Where a traversal that exceeds its budget of node visits leaves the rest of
// its stack (buf == nullptr: no budget).  With `done` set, it hands work on
// only once the finished waves reach tail_from: while enough waves are still
// to start, a heavy wave costs no time at the end of the launch, and a
// hand-off (its atomics and the extra passes) would.  Finished waves are
// counted in kDoneShards counters (workgroup b adds to b % kDoneShards), so
// that the count itself does not serialise the launch.
constexpr int kDoneShards = 32;
struct PacketSpill {
  PacketTask* buf;
  uint32_t* count;  // tasks reserved so far (may exceed cap: the excess is not written)
  uint32_t cap;
  uint32_t budget;
  uint32_t* done;  // [kDoneShards] finished waves of the launch, or nullptr
  uint32_t tail_from;
};

// A wave of a launch with a tail test reports that it has finished.
__device__ __forceinline__ void wave_done(const PacketSpill& spill) {
  if (spill.done && lane_id() == 0) atomicAdd(spill.done + blockIdx.x % kDoneShards, 1u);
}

// Called by a wave whose budget of node visits is used up (left == 0).  In
// the launch's tail it hands the bottom entries of its stack whose subtrees
// span at least 2^kSplitLevels leaves on as tasks (entries deepen from the
// bottom of the stack to its top, and entry i sits in lane i, so each lane
// writes one task) and keeps the smaller ones.  Resets the budget; returns
// true when nothing is left to do here.
__device__ __forceinline__ bool hand_off(const PacketSpill& spill, int levels, uint32_t group,
                                         uint32_t& stackv, uint32_t& stk_lo, uint32_t& stk_hi,
                                         int& sp, uint32_t& left) {
  const int lane = lane_id();
  const int big_level = levels - (int)kSplitLevels;
  bool tail = true;
  if (spill.done) {
    int d = lane < kDoneShards ? (int)__hip_atomic_load(spill.done + lane, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)
                               : 0;
#pragma unroll
    for (int o = kDoneShards / 2; o > 0; o >>= 1) d += __shfl_xor(d, o);  // lane 0: all shards
    tail = (uint32_t)__builtin_amdgcn_readfirstlane(d) >= spill.tail_from;
  }
  const int nbig = tail ? __popcll(__ballot(lane < sp && node_level(stackv) <= big_level)) : 0;
  left = spill.budget;
  if (nbig == 0) return false;
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(spill.count, (uint32_t)nbig);
  base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
  if ((uint64_t)base + (uint32_t)nbig > spill.cap) {
    // no room: leave the reserved slots empty and finish here
    if (lane < nbig && (uint64_t)base + lane < spill.cap)
      spill.buf[base + lane] = PacketTask{group, kNoNode, 0u, 0u};
    left = 0xFFFFFFFFu;
    return false;
  }
  if (lane < nbig) spill.buf[base + lane] = PacketTask{group, stackv, stk_lo, stk_hi};
  if (nbig == sp) return true;
  const int from = min(lane + nbig, 63);
  stackv = (uint32_t)__shfl((int)stackv, from);
  stk_lo = (uint32_t)__shfl((int)stk_lo, from);
  stk_hi = (uint32_t)__shfl((int)stk_hi, from);
  sp -= nbig;
  return false;
}

// Box counts by the wave-shared traversal (the ball counts' launch is declared
// with the other single-tree entry points).  Leaves must hold at most 64 points.
template <int D>
kdt_status box_packet_launch(const TreeView& v, int leaf, const float* d_lo, const float* d_hi,
                             int64_t nq, const int32_t* order, int32_t* d_count,
                             uint32_t split_budget, hipStream_t stream,
                             const FillOut* fill = nullptr);

// Query shapes of the wave-shared counts.  Each says whether it cuts a node
// box, holds a node box whole, and holds a point, and packs into kFloats
// floats for the packed leaf scan.
//
// A closed ball (Algorithm 3): centre p, squared radius r2 (the same for all
// queries of a launch).
template <int D>
struct BallShape {
  static constexpr int kFloats = D;
  float p[D];
  float r2;
  __device__ __forceinline__ bool cuts(const float lo[D], const float hi[D]) const {
    return box_mindist<D>(lo, hi, p) <= r2;
  }
  __device__ __forceinline__ bool holds_box(const float lo[D], const float hi[D]) const {
    return box_maxdist<D>(lo, hi, p) <= r2;
  }
  __device__ __forceinline__ bool holds(const float x[D]) const { return sq_dist<D>(x, p) <= r2; }
  __device__ __forceinline__ void pack(float* dst) const {
#pragma unroll
    for (int a = 0; a < D; ++a) dst[a] = p[a];
  }
  __device__ __forceinline__ BallShape unpack(const float* src) const {
    BallShape b;
#pragma unroll
    for (int a = 0; a < D; ++a) b.p[a] = src[a];
    b.r2 = r2;
    return b;
  }
};

// A closed ball with its own squared radius (packed with the centre), under
// a metric (open space or the D-torus): the per-query balls of kNN with k
// above the register lists.
template <int D, class Metric>
struct VarBallShape {
  static constexpr int kFloats = D + 1;
  float p[D];
  float r2;
  Metric m;
  __device__ __forceinline__ bool cuts(const float lo[D], const float hi[D]) const {
    return m.mindist(lo, hi, p) <= r2;
  }
  __device__ __forceinline__ bool holds_box(const float lo[D], const float hi[D]) const {
    return m.maxdist(lo, hi, p) <= r2;
  }
  __device__ __forceinline__ bool holds(const float x[D]) const { return m.dist(x, p) <= r2; }
  __device__ __forceinline__ void pack(float* dst) const {
#pragma unroll
    for (int a = 0; a < D; ++a) dst[a] = p[a];
    dst[D] = r2;
  }
  __device__ __forceinline__ VarBallShape unpack(const float* src) const {
    VarBallShape b;
#pragma unroll
    for (int a = 0; a < D; ++a) b.p[a] = src[a];
    b.r2 = src[D];
    b.m = m;
    return b;
  }
};

// Counts of per-query balls (centres q[row], squared radii r2v[row]) through
// the wave-shared count traversal, rows order[s] (or s) for s < nq
// (kdt_packet.hip; Metric is OpenMetric<D> or TorusMetric<D>).
template <int D, class Metric>
kdt_status var_ball_count_launch(const TreeView& v, int leaf, const float* d_q, const float* d_r2,
                                 int64_t nq, const int32_t* order, const Metric& m,
                                 int32_t* d_count, hipStream_t stream);

// A closed axis-aligned box [lo, hi] (the rectangular ranges of Sec. 2.3).
template <int D>
struct BoxShape {
  static constexpr int kFloats = 2 * D;
  float lo[D], hi[D];
  __device__ __forceinline__ bool cuts(const float nlo[D], const float nhi[D]) const {
    bool meet = true;
#pragma unroll
    for (int a = 0; a < D; ++a) meet &= nhi[a] >= lo[a] && nlo[a] <= hi[a];
    return meet;
  }
  __device__ __forceinline__ bool holds_box(const float nlo[D], const float nhi[D]) const {
    bool in = true;
#pragma unroll
    for (int a = 0; a < D; ++a) in &= lo[a] <= nlo[a] && nhi[a] <= hi[a];
    return in;
  }
  __device__ __forceinline__ bool holds(const float x[D]) const {
    bool in = true;
#pragma unroll
    for (int a = 0; a < D; ++a) in &= lo[a] <= x[a] && x[a] <= hi[a];
    return in;
  }
  __device__ __forceinline__ void pack(float* dst) const {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      dst[a] = lo[a];
      dst[D + a] = hi[a];
    }
  }
  __device__ __forceinline__ BoxShape unpack(const float* src) const {
    BoxShape b;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      b.lo[a] = src[a];
      b.hi[a] = src[D + a];
    }
    return b;
  }
};

// LDS floats of one wave of a count: the open leaf, then the packed queries
// [64][K] (K floats per query shape), their counts [64] and, for the fill,
// their hit masks [64] (uint64).
template <int D, int K = D>
__host__ __device__ constexpr size_t range_wave_floats(int leaf) {
  return (size_t)leaf * rec_stride(D) + 64 * (K + 1) + 128;
}

// Fill mode: a lane appends n indices to its row; returns the first slot.
__device__ __forceinline__ int64_t fill_reserve(const FillOut& fo, int64_t row, int n) {
  return fo.off[row] + atomicAdd(fo.cur + row, n);
}

// Fill mode: a lane's leaf hits (bit i: point i of the open leaf) into its row.
template <class Leaf>
__device__ __forceinline__ void fill_hits(const FillOut& fo, int64_t row, uint64_t hits,
                                          const Leaf& leaf) {
  if (!hits) return;
  int64_t at = fill_reserve(fo, row, __popcll(hits));
  while (hits) {
    const int i = __ffsll((unsigned long long)hits) - 1;
    hits &= hits - 1;
    fo.out[at++] = leaf.index(i);
  }
}

// Counts of the 64 query shapes of a wave (closed balls: Algorithm 3
// semantics; or closed boxes): a node that no lane's shape cuts is skipped, a
// node entirely inside a lane's shape adds its size to that lane, and leaves
// are scanned only for the lanes whose shape cuts them.  Each stack entry carries the mask of lanes that
// still need that subtree, so a lane that has counted a whole node never
// counts its descendants again.  Leaves must hold at most 64 points.
//
// Where the balls of a wave overlap a dense region, a leaf often cuts the
// surface of only a few of them.  Then the queries that need the leaf are
// packed into LDS and the wave tests (query, point) pairs instead: 64 / W
// queries per step, W the leaf size rounded up to a power of two, each lane
// holding one point; a query's count is the population of its lanes' ballot.
// The distances are the same float32 expressions either way.
//
// The traversal starts at `start` for the lanes of `start_mask`.  In a dense
// halo the balls of one wave can hold millions of points while most waves
// finish within a few hundred node visits, and that one wave would set the
// length of the whole launch.  So a wave that has visited `budget` nodes
// writes its remaining stack entries (entry i sits in lane i) as tasks for a
// later pass and returns its partial counts; the later passes add theirs, so
// every count is the same integer sum.
//
// FILL: the same traversal writes the CSR lists (FillOut) of the lanes'
// rows instead of only counting: a whole node is written for each lane that
// holds it by the whole wave (64 entries per step, its rows' slots reserved
// by that lane), a leaf's hits by each lane from its hit mask.
template <int D, class Shape, bool FILL = false>
__device__ __forceinline__ int64_t packet_range_count(const TreeView& t, const Shape& sh,
                                                      bool active, float* lds,
                                                      int leaf_cap, uint32_t start,
                                                      uint64_t start_mask, uint32_t group,
                                                      const PacketSpill& spill,
                                                      int64_t row = 0,
                                                      const FillOut& fo = FillOut{}) {
  constexpr int S = rec_stride(D);
  constexpr int K = Shape::kFloats;
  const int lane = lane_id();
  LeafReader<D> leaf(t.rec, lds);
  float* cq = lds + (size_t)leaf_cap * S;                  // packed queries [64][K]
  int32_t* cc = reinterpret_cast<int32_t*>(cq + 64 * K);  // their counts [64]
  uint64_t* cm = reinterpret_cast<uint64_t*>(cc + 64);    // their hit masks [64] (fill)
  const uint32_t first_leaf = (1u << t.levels) - 1u;
  int64_t count = 0;
  uint32_t stackv = start;                         // lane i: node of entry i
  uint32_t stk_lo = (uint32_t)start_mask;          // lane i: lane mask of entry i
  uint32_t stk_hi = (uint32_t)(start_mask >> 32);
  int sp = 1;
  uint32_t left = spill.buf ? spill.budget : 0xFFFFFFFFu;  // node visits before handing off
  while (sp > 0) {
    if (left == 0 && hand_off(spill, t.levels, group, stackv, stk_lo, stk_hi, sp, left))
      return count;
    --left;
    --sp;
    const uint32_t node = (uint32_t)__builtin_amdgcn_readlane((int)stackv, sp);
    const uint64_t live = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)stk_hi, sp) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)stk_lo, sp);
    const bool mine = active && ((live >> lane) & 1ull);
    float lo[D], hi[D];
    load_box_uniform<D>(t.box, node, lo, hi);
    KDT_WAVE_VISIT(t, kVisitWaveNodes, 1);
    const bool touch = mine && sh.cuts(lo, hi);
    if (!__any(touch)) continue;
    const bool full = touch && sh.holds_box(lo, hi);
    const int lev = node_level(node);
    const int64_t j = (int64_t)node - ((int64_t(1) << lev) - 1);
    const int64_t b = node_begin(t.n, lev, j), e = node_begin(t.n, lev, j + 1);
    if (full) count += e - b;
    if (FILL) {
      uint64_t fm = __ballot(full);
      if (fm) {
        constexpr int S2 = rec_stride(D);
        const int64_t at = full ? fill_reserve(fo, row, (int)(e - b)) : 0;
        while (fm) {
          const int l = __ffsll((unsigned long long)fm) - 1;
          fm &= fm - 1;
          const int64_t dst = ((int64_t)__builtin_amdgcn_readlane((int)(at >> 32), l) << 32) |
                              (uint32_t)__builtin_amdgcn_readlane((int)at, l);
          for (int64_t i = b + lane; i < e; i += 64)
            fo.out[dst + (i - b)] = __float_as_int(t.rec[i * S2 + D]);
        }
      }
    }
    const bool part = touch && !full;
    const uint64_t pm = __ballot(part);
    if (pm == 0) continue;
    if (node >= first_leaf) {
      const int cnt = (int)(e - b);
      leaf.open(b, cnt);
      KDT_WAVE_VISIT(t, kVisitWavePoints, cnt);
      const int na = __popcll(pm);
      const int W = cnt <= 8 ? 8 : cnt <= 16 ? 16 : cnt <= 32 ? 32 : 64;
      const int G = 64 / W;
      const int steps = (na + G - 1) / G;
      if (2 * steps <= cnt) {  // a packed step costs about two broadcast steps
        const int me = lanes_below(pm);
        if (part) sh.pack(cq + me * K);
        wave_sync();
        const int slot = lane / W, i = lane % W;
        const uint64_t wmask = ~0ull >> (64 - W);
        float x[D];
        leaf.point(min(i, cnt - 1), x);
        for (int s = 0; s < steps; ++s) {
          const int a = s * G + slot;
          const int ac = min(a, na - 1);
          const Shape qs = sh.unpack(cq + ac * K);
          const bool hit = i < cnt && a < na && qs.holds(x);
          const uint64_t hm = __ballot(hit);
          if (i == 0 && a < na) {
            cc[a] = __popcll((hm >> (slot * W)) & wmask);
            if (FILL) cm[a] = (hm >> (slot * W)) & wmask;
          }
        }
        wave_sync();
        if (part) count += cc[me];
        if (FILL && part) fill_hits(fo, row, cm[me], leaf);
      } else {
        int c = 0;
        uint64_t hits = 0;
#pragma unroll uniform_batch<D>()
        for (int i = 0; i < cnt; ++i) {
          float x[D];
          leaf.point(i, x);
          const bool h = sh.holds(x);
          c += h;
          if (FILL) hits |= (uint64_t)h << i;
        }
        if (part) count += c;
        if (FILL && part) fill_hits(fo, row, hits, leaf);
      }
    } else {
      const uint32_t mlo = (uint32_t)pm, mhi = (uint32_t)(pm >> 32);
#pragma unroll
      for (int c = 2; c >= 1; --c) {
        stackv = lane == sp ? 2 * node + c : stackv;
        stk_lo = lane == sp ? mlo : stk_lo;
        stk_hi = lane == sp ? mhi : stk_hi;
        ++sp;
      }
    }
  }
  return count;
}

// Friends-of-friends links of the 64 points of a wave (tree positions pos,
// indices me; union-find indices base + index).  A node whose points are known
// to form one component (conn flag) is skipped by every lane whose own root is
// already that component's, needs a single link when it lies entirely within l
// of the lane, and otherwise only its first friend.  A node entirely within l
// of several lanes is joined to the lowest such lane's point by the whole wave
// (64 links at a time), and that lane flags it; the others link to its first
// point.  Elsewhere each pair within l
// is linked by the point that comes first in tree order: a lane never enters a
// node that ends at or before its own position, so the search of a ball costs
// about half.  Leaves must hold at most 64 points.  The metric supplies the
// point distance and the node bounds (OpenMetric by default).
template <int D, class Metric = OpenMetric<D>>
__device__ __forceinline__ void packet_fof(const TreeView& t, const float p[D], int64_t pos,
                                           int32_t me, bool active, float l2, int32_t base,
                                           int32_t* __restrict__ parent,
                                           uint32_t* __restrict__ conn, float* lds,
                                           const Metric& metric = Metric()) {
  constexpr int S = rec_stride(D);
  const int lane = lane_id();
  const uint32_t first_leaf = (1u << t.levels) - 1u;
  const int32_t gme = base + me;
  int32_t myroot = gme;  // an ancestor of this lane's point (see uf_union_from)
  LeafReader<D> leaf(t.rec, lds);
  uint32_t stackv = 0;
  uint32_t stk_lo = 0xFFFFFFFFu, stk_hi = 0xFFFFFFFFu;
  int sp = 1;
  while (sp > 0) {
    --sp;
    const uint32_t node = (uint32_t)__builtin_amdgcn_readlane((int)stackv, sp);
    const uint64_t live = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)stk_hi, sp) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)stk_lo, sp);
    const int lev = node_level(node);
    const int64_t j = (int64_t)node - ((int64_t(1) << lev) - 1);
    const int64_t b = node_begin(t.n, lev, j), e = node_begin(t.n, lev, j + 1);
    // a lane links only towards later tree positions: a node that ends at or
    // before its own position is left to the points inside it
    const bool mine = active && ((live >> lane) & 1ull) && e > pos;
    float lo[D], hi[D];
    load_box_uniform<D>(t.box, node, lo, hi);
    bool touch = mine && metric.mindist(lo, hi, p) <= l2;
    if (!__any(touch)) continue;
    const int32_t gfirst = base + __float_as_int(t.rec[b * S + D]);
    const bool one = flag_ld(conn + node) != 0;
    if (one && touch) {
      const bool inside = pos >= b && pos < e;
      if (!inside) myroot = uf_find(parent, myroot);
      touch = !inside && myroot != uf_find(parent, gfirst);
    }
    if (!__any(touch)) continue;
    const bool full = touch && metric.maxdist(lo, hi, p) <= l2;
    if (one) {
      if (full) uf_union_from(parent, myroot, gfirst);
    } else {
      const uint64_t fm = __ballot(full);
      if (fm != 0) {
        // every point of the node is a friend of the leader's point: the
        // whole wave links them to it, 64 at a time
        const int leader = __ffsll((unsigned long long)fm) - 1;
        const int32_t lroot = __builtin_amdgcn_readlane(myroot, leader);
        for (int64_t i = b + lane; i < e; i += 64) {
          int32_t r = lroot;
          uf_union_from(parent, r, base + __float_as_int(t.rec[i * S + D]));
        }
        if (lane == leader) {
          flag_st(conn + node, 1u);
        } else if (full) {
          uf_union_from(parent, myroot, gfirst);
        }
      }
    }
    const bool part = touch && !full;
    const uint64_t pm = __ballot(part);
    if (pm == 0) continue;
    if (node >= first_leaf) {
      // Friends in the leaf: distances for every lane first, then each
      // lane links its own friends.
      const int cnt = (int)(e - b);
      leaf.open(b, cnt);
      uint64_t fr = 0;
#pragma unroll uniform_batch<D>()
      for (int i = 0; i < cnt; ++i) {
        float x[D];
        leaf.point(i, x);
        fr |= (uint64_t)(metric.dist(x, p) <= l2) << i;
      }
      if (!part) fr = 0;
      while (fr) {
        const int i = __ffsll((unsigned long long)fr) - 1;
        fr &= fr - 1;
        const int32_t id = __float_as_int(t.rec[(b + i) * S + D]);
        if (one) {
          uf_union_from(parent, myroot, base + id);
          break;
        }
        if (b + i > pos) uf_union_from(parent, myroot, base + id);
      }
    } else {
      const uint32_t mlo = (uint32_t)pm, mhi = (uint32_t)(pm >> 32);
#pragma unroll
      for (int c = 2; c >= 1; --c) {
        stackv = lane == sp ? 2 * node + c : stackv;
        stk_lo = lane == sp ? mlo : stk_lo;
        stk_hi = lane == sp ? mhi : stk_hi;
        ++sp;
      }
    }
  }
}

}  // namespace kdt
