// kdt_midpoint.hip -- the sliding-midpoint k-d tree of Sec. 2.1 (Algorithm 1)
// built level by level on gfx950.
//
// The rule, with the ties the paper leaves open fixed: a node of more than
// N_leaf points whose tight bounding box has positive extent is split along
// the longest side of that box (lowest axis on ties) at its midpoint
// lo + (hi - lo) / 2; points whose coordinate is below the split go left,
// keeping their order (a stable partition).  When one side would be empty the
// split slides to the nearest point: the point of smallest coordinate (lowest
// input index on ties) alone goes left, or the point of largest coordinate
// (lowest input index on ties) alone goes right.  Nodes of at most N_leaf
// points, or whose points all coincide, are leaves.  The depth depends on the
// data, so the nodes are stored: node v holds its left child (-1 for a leaf;
// the right child follows the left one), its first and end position in tree
// order, and its level.  Nodes are numbered level by level.
//
// Every node still to split is a segment [b, e) of the tree order.  Per level:
//   plan     (a thread per segment)  axis and midpoint from the node's box;
//   mark     (a thread per point)    1 if the point lies below its midpoint;
//   scan     exclusive sum of the marks: the left count of a segment and the
//            rank of a point among the left points of its segment, with no
//            atomics however large the segment;
//   resolve  (a thread per segment)  slides, the children's ranges and records;
//   slide    (a wave per sliding segment) the extreme point, by a wave
//            reduction over the segment (slides are rare and mostly small);
//   scatter  (a thread per point)    the stable partition into the other buffer;
//   boxes    (a thread per point, in the new order, where each child is one
//            run) the children's tight boxes: wave and workgroup reductions,
//            then one atomic min / max per child run and workgroup;
//   children (a thread per child)    box, leaf or not;
//   compact  the next level's segments, whose count the host reads back (the
//            one wait per level).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kdt_query.h"

namespace kdt {

constexpr int kMBlock = 256;
// Deepest sliding-midpoint tree accepted: the traversals keep a stack of one
// entry per level per lane in LDS.
constexpr int kMidMaxLevels = 96;

namespace {

// Calls f(key, group, leader, mine) once for each distinct key among the
// lanes with `active` set; `group` holds the lanes of that key.
template <typename F>
__device__ __forceinline__ void for_each_key(int key, bool active, F&& f) {
  uint64_t todo = __ballot(active);
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const int lk = __shfl(key, leader);
    const bool mine = active && key == lk;
    const uint64_t group = __ballot(mine);
    f(lk, group, leader, mine);
    todo &= ~group;
  }
}

__device__ __forceinline__ uint64_t wave_min64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t w = __shfl_xor(v, o);
    v = w < v ? w : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_max64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t w = __shfl_xor(v, o);
    v = w > v ? w : v;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_min32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
  return v;
}
__device__ __forceinline__ uint32_t wave_max32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
  return v;
}

// Box keys of a node: [2][D] order-preserving keys (min, then max).
template <int D>
__device__ __forceinline__ void keys_to_box(const uint32_t* k, float lo[D], float hi[D]) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lo[a] = fkey_inv(k[a]);
    hi[a] = fkey_inv(k[D + a]);
  }
}

template <int D>
__device__ __forceinline__ void store_box(float* box, int64_t v, const float lo[D],
                                          const float hi[D]) {
  constexpr int P = pad4(D);
  float* b = box + v * 2 * P;
#pragma unroll
  for (int a = 0; a < P; ++a) {
    b[a] = a < D ? lo[a] : 0.0f;
    b[P + a] = a < D ? hi[a] : 0.0f;
  }
}

// Longest side of a box (lowest axis on ties) and its extent, as the rule
// states it: ext = hi - lo per axis, compared with a strict >.
template <int D>
__device__ __forceinline__ int longest_axis(const float lo[D], const float hi[D], float& ext) {
  int ax = 0;
  ext = hi[0] - lo[0];
#pragma unroll
  for (int a = 1; a < D; ++a) {
    const float e = hi[a] - lo[a];
    if (e > ext) {
      ext = e;
      ax = a;
    }
  }
  return ax;
}

}  // namespace

// AoS -> SoA copy, identity order, finiteness flag and the root's box keys.
// Grid-stride: each workgroup folds its points' keys in registers, then in
// LDS, and adds one atomic per key and workgroup (one per wave and key made
// 2^24 points take 18 ms, the atomics on the 2d keys serialising).
template <int D>
__global__ __launch_bounds__(kMBlock) void k_mid_ingest(const float* __restrict__ pts, int64_t n,
                                                        float* __restrict__ x,
                                                        int32_t* __restrict__ perm,
                                                        uint32_t* __restrict__ rootkeys,
                                                        int32_t* __restrict__ bad) {
  constexpr int kW = kMBlock / 64;
  __shared__ uint32_t red[2 * D][kW];
  uint32_t mn[D], mx[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    mn[a] = 0xFFFFFFFFu;
    mx[a] = 0u;
  }
  bool fin = true;
  for (int64_t i = (int64_t)blockIdx.x * kMBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kMBlock) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const float v = pts[i * D + a];
      fin &= isfinite(v);
      x[(int64_t)a * n + i] = v;
      const uint32_t k = fkey(v);
      mn[a] = min(mn[a], k);
      mx[a] = max(mx[a], k);
    }
    perm[i] = (int32_t)i;
  }
  if (!fin) atomicOr(bad, 1);
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const uint32_t wmn = wave_min32(mn[a]);
    const uint32_t wmx = wave_max32(mx[a]);
    if (lane_id() == 0) {
      red[a][w] = wmn;
      red[D + a][w] = wmx;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * D) {
    const int j = threadIdx.x;
    uint32_t v = red[j][0];
    for (int q = 1; q < kW; ++q) v = j < D ? min(v, red[j][q]) : max(v, red[j][q]);
    if (j < D)
      atomicMin(rootkeys + j, v);
    else
      atomicMax(rootkeys + j, v);
  }
}

// The root's record and box; the first level's single segment if it splits.
template <int D>
__global__ void k_mid_root(int64_t n, int leaf, const uint32_t* __restrict__ rootkeys,
                           int4* __restrict__ node, float* __restrict__ box,
                           int32_t* __restrict__ axis, float* __restrict__ split,
                           int4* __restrict__ seg, int32_t* __restrict__ count) {
  float lo[D], hi[D];
  keys_to_box<D>(rootkeys, lo, hi);
  store_box<D>(box, 0, lo, hi);
  node[0] = make_int4(-1, 0, (int)n, 0);
  axis[0] = -1;
  split[0] = 0.0f;
  float ext = 0.0f;
  (void)longest_axis<D>(lo, hi, ext);
  const bool go = n > leaf && ext > 0.0f;
  if (go) seg[0] = make_int4(0, (int)n, 0, 0);
  *count = go ? 1 : 0;
}

__global__ void k_mid_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * kMBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

// Per segment: axis and midpoint from the node's box.
template <int D>
__global__ void k_mid_plan(int m, int4* __restrict__ seg, float* __restrict__ seg_split,
                           const float* __restrict__ box) {
  const int s = blockIdx.x * kMBlock + threadIdx.x;
  if (s >= m) return;
  int4 g = seg[s];
  float lo[D], hi[D];
  load_box<D>(box, (uint32_t)g.z, lo, hi);
  float ext = 0.0f;
  const int ax = longest_axis<D>(lo, hi, ext);
  g.w = ax;
  seg[s] = g;
  seg_split[s] = lo[ax] + (hi[ax] - lo[ax]) * 0.5f;  // box midpoint
}

// Per point: 1 if it lies below its segment's midpoint (0 outside segments
// and at position n, so the scan's entry n is the total).
__global__ __launch_bounds__(kMBlock) void k_mid_mark(int64_t n, const float* __restrict__ x,
                                                      const int32_t* __restrict__ sid,
                                                      const int4* __restrict__ seg,
                                                      const float* __restrict__ seg_split,
                                                      int32_t* __restrict__ mark) {
  const int64_t i = (int64_t)blockIdx.x * kMBlock + threadIdx.x;
  if (i > n) return;
  int f = 0;
  if (i < n) {
    const int s = sid[i];
    if (s >= 0) f = x[(int64_t)seg[s].w * n + i] < seg_split[s];
  }
  mark[i] = f;
}

// Per segment: the left count from the scan, the slide decision, the
// parent's link, axis and split, the children's records.  res[s] = (left
// count, mode, pick position): mode 0 splits at the midpoint, 1 sends the
// point of smallest coordinate alone left, 2 the point of largest coordinate
// alone right (the slide kernel finds it).
__global__ void k_mid_resolve(int m, const int4* __restrict__ seg,
                              const float* __restrict__ seg_split, const int32_t* __restrict__ rank,
                              int4* __restrict__ res, int64_t node_base, int level,
                              int4* __restrict__ node, int32_t* __restrict__ axis,
                              float* __restrict__ split) {
  const int s = blockIdx.x * kMBlock + threadIdx.x;
  if (s >= m) return;
  const int4 g = seg[s];
  const int size = g.y - g.x;
  int nl = rank[g.y] - rank[g.x], mode = 0;
  if (nl == 0) {
    mode = 1;
    nl = 1;
  } else if (nl == size) {
    mode = 2;
    nl = size - 1;
  }
  res[s] = make_int4(nl, mode, -1, 0);
  const int64_t lc = node_base + 2 * (int64_t)s;
  node[g.z].x = (int)lc;
  axis[g.z] = g.w;
  split[g.z] = seg_split[s];  // a slide overwrites it
  node[lc] = make_int4(-1, g.x, g.x + nl, level + 1);
  node[lc + 1] = make_int4(-1, g.x + nl, g.y, level + 1);
  axis[lc] = axis[lc + 1] = -1;
  split[lc] = split[lc + 1] = 0.0f;
}

// A wave per sliding segment (waves stride over all segments): the point to
// move -- smallest coordinate (mode 1) or largest (mode 2), lowest input
// index on ties -- by a wave reduction of (coordinate key, index) over the
// segment; its position goes to res[s].z and its coordinate becomes the
// split.
__global__ __launch_bounds__(kMBlock) void k_mid_slide(int m, const float* __restrict__ x,
                                                       const int32_t* __restrict__ perm,
                                                       int64_t n, const int4* __restrict__ seg,
                                                       float* __restrict__ seg_split,
                                                       int4* __restrict__ res,
                                                       float* __restrict__ split) {
  const int waves = gridDim.x * (kMBlock / 64);
  for (int s = blockIdx.x * (kMBlock / 64) + threadIdx.x / 64; s < m; s += waves) {
    const int4 r = res[s];
    if (r.y == 0) continue;
    const int4 g = seg[s];
    const float* xa = x + (int64_t)g.w * n;
    // mode 1 minimises (key, index); mode 2 maximises (key, ~index), i.e. the
    // largest coordinate with the lowest index
    uint64_t best = r.y == 1 ? ~0ull : 0ull;
    int64_t where = -1;
    for (int64_t i = g.x + lane_id(); i < g.y; i += 64) {
      const uint32_t id = (uint32_t)perm[i];
      const uint64_t k = ((uint64_t)fkey(xa[i]) << 32) | (r.y == 1 ? id : ~id);
      if (r.y == 1 ? k < best : k > best) {
        best = k;
        where = i;
      }
    }
    const uint64_t w = r.y == 1 ? wave_min64(best) : wave_max64(best);
    // the key is unique (it holds the index): one lane owns it
    const uint64_t own = __ballot(where >= 0 && best == w);
    const int owner = __ffsll((unsigned long long)own) - 1;
    const int64_t pos = __shfl(where, owner);
    if (lane_id() == 0) {
      const float v = fkey_inv((uint32_t)(w >> 32));
      seg_split[s] = v;
      split[g.z] = v;
      res[s] = make_int4(r.x, r.y, (int)pos, 0);
    }
  }
}

// Per point: the stable partition of every segment into the other buffer
// (left points first, each side in its old order) and the child slot of each
// moved point; points outside segments stay where they are.
template <int D>
__global__ __launch_bounds__(kMBlock) void k_mid_scatter(
    int64_t n, const float* __restrict__ x, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ sid, const int4* __restrict__ seg, const int4* __restrict__ res,
    const int32_t* __restrict__ mark, const int32_t* __restrict__ rank, float* __restrict__ xo,
    int32_t* __restrict__ po, int32_t* __restrict__ cid) {
  const int64_t i = (int64_t)blockIdx.x * kMBlock + threadIdx.x;
  if (i >= n) return;
  const int s = sid[i];
  int64_t dest = i;
  int child = -1;
  if (s >= 0) {
    const int4 g = seg[s];
    const int4 r = res[s];
    bool left;
    if (r.y == 0) {
      left = mark[i] != 0;
      const int64_t rl = (int64_t)rank[i] - rank[g.x];  // left points before i in the segment
      dest = left ? g.x + rl : g.x + r.x + (i - g.x - rl);
    } else {
      const int64_t before = i - g.x - (r.z < i ? 1 : 0);  // other points before i
      if (r.y == 1) {
        left = i == r.z;
        dest = left ? g.x : g.x + 1 + before;
      } else {
        left = i != r.z;
        dest = left ? g.x + before : g.y - 1;
      }
    }
    child = 2 * s + (left ? 0 : 1);
  }
#pragma unroll
  for (int a = 0; a < D; ++a) xo[(int64_t)a * n + dest] = x[(int64_t)a * n + i];
  po[dest] = perm[i];
  cid[dest] = child;
}

constexpr int kBoxBlock = 1024;
// Levels of at most kRunBoxChildren children take their boxes from the
// children's runs, with about kRunBoxBlocks workgroups in all.
constexpr int64_t kRunBoxChildren = 2048;
constexpr int64_t kRunBoxBlocks = 4096;

// Per point of the new order: the children's tight boxes.  A child is one run
// of positions, so a wave's points fall in one or two children; partial
// boxes are reduced per wave, then per workgroup in LDS, and each workgroup
// adds one atomic min and max per child run and axis.
template <int D>
__global__ __launch_bounds__(kBoxBlock) void k_mid_boxes(int64_t n, const float* __restrict__ x,
                                                         const int32_t* __restrict__ cid,
                                                         uint32_t* __restrict__ ckeys) {
  constexpr int W = kBoxBlock / 64;
  __shared__ int wkey[W][2];
  __shared__ uint32_t wbox[W][2][2 * D];
  const int64_t i = (int64_t)blockIdx.x * kBoxBlock + threadIdx.x;
  const int c = i < n ? cid[i] : -1;
  const int w = threadIdx.x / 64;
  if (lane_id() < 2) wkey[w][lane_id()] = -1;
  // a wave's children: its first and last keys (runs are contiguous)
  int slot = 0;
  for_each_key(c, c >= 0, [&](int key, uint64_t, int leader, bool mine) {
    uint32_t part[2 * D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const float v = mine ? x[(int64_t)a * n + i] : 0.0f;
      part[a] = wave_min32(mine ? fkey(v) : 0xFFFFFFFFu);
      part[D + a] = wave_max32(mine ? fkey(v) : 0u);
    }
    if (slot < 2) {
      if (lane_id() == leader) {
        wkey[w][slot] = key;
#pragma unroll
        for (int a = 0; a < 2 * D; ++a) wbox[w][slot][a] = part[a];
      }
    } else if (lane_id() == leader) {  // a third child in one wave: straight to global
      uint32_t* k = ckeys + (int64_t)key * 2 * D;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        atomicMin(k + a, part[a]);
        atomicMax(k + D + a, part[D + a]);
      }
    }
    ++slot;
  });
  __syncthreads();
  // one thread per (wave slot): merge equal keys of the workgroup, then flush
  if (threadIdx.x < 2 * W) {
    const int ws = threadIdx.x / 2, ss = threadIdx.x % 2;
    const int key = wkey[ws][ss];
    bool first = key >= 0;
    // only the first holder of a key in slot order flushes it
    for (int v = 0; v < 2 * W && first; ++v) {
      if (v == (int)threadIdx.x) break;
      if (wkey[v / 2][v % 2] == key) first = false;
    }
    if (first) {
      uint32_t acc[2 * D];
#pragma unroll
      for (int a = 0; a < 2 * D; ++a) acc[a] = wbox[ws][ss][a];
      for (int v = threadIdx.x + 1; v < 2 * W; ++v)
        if (wkey[v / 2][v % 2] == key) {
#pragma unroll
          for (int a = 0; a < D; ++a) {
            acc[a] = min(acc[a], wbox[v / 2][v % 2][a]);
            acc[D + a] = max(acc[D + a], wbox[v / 2][v % 2][D + a]);
          }
        }
      uint32_t* k = ckeys + (int64_t)key * 2 * D;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        atomicMin(k + a, acc[a]);
        atomicMax(k + D + a, acc[D + a]);
      }
    }
  }
}

// Resets the box keys of 2 m children (min keys to all ones, max keys to 0).
template <int D>
__global__ void k_mid_reset_keys(int64_t mc, uint32_t* __restrict__ ckeys) {
  const int64_t j = (int64_t)blockIdx.x * kMBlock + threadIdx.x;
  if (j >= mc * 2 * D) return;
  ckeys[j] = (j % (2 * D)) < D ? 0xFFFFFFFFu : 0u;
}

// The children's boxes at the top levels (few children, long runs): the
// runs are known from the children's node records, so G workgroups take a
// slice of each child's run, fold it in registers and LDS, and add one
// atomic per key; with one atomic per workgroup and child in k_mid_boxes,
// the 16 384 workgroups of a 2^24-point level queued on the same few keys.
template <int D>
__global__ __launch_bounds__(kBoxBlock) void k_mid_boxes_runs(int64_t n,
                                                              const float* __restrict__ x,
                                                              const int4* __restrict__ node,
                                                              int64_t node_base,
                                                              uint32_t* __restrict__ ckeys) {
  constexpr int W = kBoxBlock / 64;
  __shared__ uint32_t red[2 * D][W];
  const int c = blockIdx.y;
  const int4 r = node[node_base + c];
  const int64_t len = (int64_t)r.z - r.y;
  const int64_t s0 = r.y + len * blockIdx.x / gridDim.x;
  const int64_t s1 = r.y + len * (blockIdx.x + 1) / gridDim.x;
  uint32_t mn[D], mx[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    mn[a] = 0xFFFFFFFFu;
    mx[a] = 0u;
  }
  for (int64_t i = s0 + threadIdx.x; i < s1; i += kBoxBlock) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const uint32_t k = fkey(x[(int64_t)a * n + i]);
      mn[a] = min(mn[a], k);
      mx[a] = max(mx[a], k);
    }
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const uint32_t wmn = wave_min32(mn[a]);
    const uint32_t wmx = wave_max32(mx[a]);
    if (lane_id() == 0) {
      red[a][w] = wmn;
      red[D + a][w] = wmx;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * D && s1 > s0) {
    const int j = threadIdx.x;
    uint32_t v = red[j][0];
    for (int q = 1; q < W; ++q) v = j < D ? min(v, red[j][q]) : max(v, red[j][q]);
    uint32_t* k = ckeys + (int64_t)c * 2 * D;
    if (j < D)
      atomicMin(k + j, v);
    else
      atomicMax(k + j, v);
  }
}

// Per child slot: its box; 1 in act[] if it is split at the next level.
template <int D>
__global__ void k_mid_children(int mc, const uint32_t* __restrict__ ckeys, int64_t node_base,
                               int leaf, const int4* __restrict__ node, float* __restrict__ box,
                               int32_t* __restrict__ act) {
  const int c = blockIdx.x * kMBlock + threadIdx.x;
  if (c >= mc) return;
  float lo[D], hi[D];
  keys_to_box<D>(ckeys + (int64_t)c * 2 * D, lo, hi);
  const int64_t v = node_base + c;
  store_box<D>(box, v, lo, hi);
  const int4 r = node[v];
  float ext = 0.0f;
  (void)longest_axis<D>(lo, hi, ext);
  act[c] = (r.z - r.y > leaf && ext > 0.0f) ? 1 : 0;
}

// The next level's segments in child order; the count into *count.
__global__ void k_mid_compact(int mc, const int32_t* __restrict__ act,
                              const int32_t* __restrict__ pos, int64_t node_base,
                              const int4* __restrict__ node, int4* __restrict__ nseg,
                              int32_t* __restrict__ count) {
  const int c = blockIdx.x * kMBlock + threadIdx.x;
  if (c >= mc) return;
  if (act[c]) {
    const int4 r = node[node_base + c];
    nseg[pos[c]] = make_int4(r.y, r.z, (int)(node_base + c), 0);
  }
  if (c == mc - 1) *count = pos[c] + act[c];
}

// Per point: its segment at the next level, or -1 once its node is a leaf.
__global__ __launch_bounds__(kMBlock) void k_mid_sid(int64_t n, const int32_t* __restrict__ cid,
                                                     const int32_t* __restrict__ act,
                                                     const int32_t* __restrict__ pos,
                                                     int32_t* __restrict__ sid) {
  const int64_t i = (int64_t)blockIdx.x * kMBlock + threadIdx.x;
  if (i >= n) return;
  const int c = cid[i];
  sid[i] = (c >= 0 && act[c]) ? pos[c] : -1;
}

// The tree-ordered records and the order.
template <int D>
__global__ __launch_bounds__(kMBlock) void k_mid_records(int64_t n, const float* __restrict__ x,
                                                         const int32_t* __restrict__ perm,
                                                         float* __restrict__ rec,
                                                         int32_t* __restrict__ perm_out) {
  constexpr int S = rec_stride(D);
  const int64_t t = (int64_t)blockIdx.x * kMBlock + threadIdx.x;
  if (t >= n) return;
  float r[S];
#pragma unroll
  for (int a = 0; a < S; ++a) r[a] = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) r[a] = x[(int64_t)a * n + t];
  const int32_t id = perm[t];
  r[D] = __int_as_float(id);
  float4* dst = reinterpret_cast<float4*>(rec + t * S);
#pragma unroll
  for (int q = 0; q < S / 4; ++q) dst[q] = make_float4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
  perm_out[t] = id;
}

namespace {

#define KDT_M(call)                                                   \
  do {                                                                \
    hipError_t e_ = (call);                                           \
    if (e_ != hipSuccess) {                                           \
      kdt_set_error("kdt_build (sliding midpoint): %s: %s", #call,   \
                    hipGetErrorString(e_));                           \
      return KDT_EDEVICE;                                             \
    }                                                                 \
  } while (0)

// Node arrays that grow with the levels (stream-ordered).
struct NodeArrays {
  int64_t cap = 0;
  int4* node = nullptr;
  float* box = nullptr;
  int32_t* axis = nullptr;
  float* split = nullptr;
};

template <int D>
bool grow_nodes(NodeArrays& a, int64_t need, int64_t used, hipStream_t stream) {
  if (need <= a.cap) return true;
  constexpr int P = pad4(D);
  NodeArrays b;
  b.cap = std::max<int64_t>(need, 2 * a.cap);
  if (dev_alloc((void**)&b.node, sizeof(int4) * b.cap, stream) != hipSuccess) return false;
  if (dev_alloc((void**)&b.box, sizeof(float) * 2 * P * b.cap, stream) != hipSuccess ||
      dev_alloc((void**)&b.axis, sizeof(int32_t) * b.cap, stream) != hipSuccess ||
      dev_alloc((void**)&b.split, sizeof(float) * b.cap, stream) != hipSuccess) {
    (void)hipFreeAsync(b.node, stream);
    if (b.box) (void)hipFreeAsync(b.box, stream);
    if (b.axis) (void)hipFreeAsync(b.axis, stream);
    return false;
  }
  if (used > 0) {
    (void)hipMemcpyAsync(b.node, a.node, sizeof(int4) * used, hipMemcpyDeviceToDevice, stream);
    (void)hipMemcpyAsync(b.box, a.box, sizeof(float) * 2 * P * used, hipMemcpyDeviceToDevice,
                         stream);
    (void)hipMemcpyAsync(b.axis, a.axis, sizeof(int32_t) * used, hipMemcpyDeviceToDevice, stream);
    (void)hipMemcpyAsync(b.split, a.split, sizeof(float) * used, hipMemcpyDeviceToDevice, stream);
  }
  for (void* p : {(void*)a.node, (void*)a.box, (void*)a.axis, (void*)a.split})
    if (p) (void)hipFreeAsync(p, stream);
  a = b;
  return true;
}

void free_nodes(NodeArrays& a, hipStream_t stream) {
  for (void* p : {(void*)a.node, (void*)a.box, (void*)a.axis, (void*)a.split})
    if (p) (void)hipFreeAsync(p, stream);
  a = NodeArrays();
}

template <int D>
kdt_status build_midpoint_d(const float* d_pts, int64_t n, int leaf, bool check,
                            hipStream_t stream, kdt_tree* t) {
  constexpr int P = pad4(D);
  PoolBuffers buf(stream);
  float* X[2] = {nullptr, nullptr};
  int32_t* Pm[2] = {nullptr, nullptr};
  int32_t *sid = nullptr, *mark = nullptr, *rank = nullptr, *cid = nullptr, *flags = nullptr;
  uint32_t* rootkeys = nullptr;
  void* scan_tmp = nullptr;
  // the marks and their scan have n + 1 entries: rank[n] is the total
  const size_t scan_bytes = scan_scratch_bytes(n + 1);
  if (!buf.get(&X[0], (size_t)D * n) || !buf.get(&X[1], (size_t)D * n) ||
      !buf.get(&Pm[0], (size_t)n) || !buf.get(&Pm[1], (size_t)n) || !buf.get(&sid, (size_t)n) ||
      !buf.get(&mark, (size_t)n + 1) || !buf.get(&rank, (size_t)n + 1) ||
      !buf.get(&cid, (size_t)n) ||
      !buf.get(&flags, 64) || !buf.get(&rootkeys, 2 * D) ||
      !buf.get((char**)&scan_tmp, scan_bytes)) {
    kdt_set_error("kdt_build (sliding midpoint): device allocation failed (%lld points)",
                  (long long)n);
    return KDT_ENOMEM;
  }
  int32_t* bad = flags;
  int32_t* d_count = flags + 16;
  const unsigned gn = (unsigned)((n + kMBlock - 1) / kMBlock);
  k_mid_fill_i32<<<1, kMBlock, 0, stream>>>(flags, 64, 0);
  k_mid_fill_i32<<<1, kMBlock, 0, stream>>>(reinterpret_cast<int32_t*>(rootkeys), D, -1);
  k_mid_fill_i32<<<1, kMBlock, 0, stream>>>(reinterpret_cast<int32_t*>(rootkeys) + D, D, 0);
  k_mid_ingest<D><<<std::min(gn, 2048u), kMBlock, 0, stream>>>(d_pts, n, X[0], Pm[0], rootkeys,
                                                               bad);

  NodeArrays na;
  struct Guard {
    NodeArrays& na;
    hipStream_t s;
    ~Guard() { free_nodes(na, s); }
  } guard{na, stream};
  if (!grow_nodes<D>(na, std::max<int64_t>(1024, 4 * (n / std::max(leaf, 1)) + 16), 0, stream)) {
    kdt_set_error("kdt_build (sliding midpoint): cannot allocate the nodes");
    return KDT_ENOMEM;
  }
  // per-segment and per-child buffers, grown with the widest level
  int64_t mcap = 0;
  PoolBuffers lvl(stream);
  int4 *seg = nullptr, *nseg = nullptr, *res = nullptr;
  float* seg_split = nullptr;
  uint32_t* ckeys = nullptr;
  int32_t *act = nullptr, *pos = nullptr;
  void* cscan_tmp = nullptr;
  // capacity for c segments (and 2 c children); the buffers' contents are lost
  auto ensure = [&](int64_t m) -> bool {
    if (m <= mcap) return true;
    const int64_t c = std::max<int64_t>(m, 2 * mcap);
    lvl.release();
    if (!lvl.get(&seg, (size_t)c) || !lvl.get(&nseg, (size_t)c) || !lvl.get(&res, (size_t)c) ||
        !lvl.get(&seg_split, (size_t)c) || !lvl.get(&ckeys, (size_t)c * 4 * D) ||
        !lvl.get(&act, (size_t)2 * c) ||
        !lvl.get(&pos, (size_t)2 * c) ||
        !lvl.get((char**)&cscan_tmp, scan_scratch_bytes(2 * c)))
      return false;
    mcap = c;
    return true;
  };
  if (!ensure(1024)) {
    kdt_set_error("kdt_build (sliding midpoint): device allocation failed");
    return KDT_ENOMEM;
  }
  k_mid_root<D><<<1, 1, 0, stream>>>(n, leaf, rootkeys, na.node, na.box, na.axis, na.split, seg,
                                     d_count);
  int32_t hc[2] = {0, 0};
  KDT_M(hipMemcpyAsync(hc, flags, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  KDT_M(hipMemcpyAsync(hc + 1, d_count, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  KDT_M(hipStreamSynchronize(stream));
  if (check && hc[0]) {
    kdt_set_error("kdt_build: the points contain NaN or infinite coordinates");
    return KDT_EINVAL;
  }
  int64_t m = hc[1];
  k_mid_fill_i32<<<gn, kMBlock, 0, stream>>>(sid, n, m > 0 ? 0 : -1);
  int64_t node_base = 1;  // nodes written so far
  int level = 0, cur = 0;
  while (m > 0) {
    if (level >= kMidMaxLevels) {
      kdt_set_error("kdt_build (sliding midpoint): the tree is deeper than %d levels",
                    kdt::kMidMaxLevels);
      return KDT_EUNSUPPORTED;
    }
    if (2 * m > mcap) {
      // the next level can hold 2 m segments: grow, keeping this level's
      int4* tmp = nullptr;
      if (dev_alloc((void**)&tmp, sizeof(int4) * (size_t)m, stream) != hipSuccess) {
        kdt_set_error("kdt_build (sliding midpoint): device allocation failed");
        return KDT_ENOMEM;
      }
      KDT_M(hipMemcpyAsync(tmp, seg, sizeof(int4) * (size_t)m, hipMemcpyDeviceToDevice, stream));
      if (!ensure(2 * m)) {
        (void)hipFreeAsync(tmp, stream);
        kdt_set_error("kdt_build (sliding midpoint): device allocation failed");
        return KDT_ENOMEM;
      }
      KDT_M(hipMemcpyAsync(seg, tmp, sizeof(int4) * (size_t)m, hipMemcpyDeviceToDevice, stream));
      (void)hipFreeAsync(tmp, stream);
    }
    if (!grow_nodes<D>(na, node_base + 2 * m, node_base, stream)) {
      kdt_set_error("kdt_build (sliding midpoint): cannot grow the nodes");
      return KDT_ENOMEM;
    }
    const unsigned gm = (unsigned)((m + kMBlock - 1) / kMBlock);
    const unsigned gc = (unsigned)((2 * m + kMBlock - 1) / kMBlock);
    const unsigned gk = (unsigned)((2 * m * 2 * D + kMBlock - 1) / kMBlock);
    const unsigned gn1 = (unsigned)((n + 1 + kMBlock - 1) / kMBlock);
    const unsigned gs = (unsigned)std::min<int64_t>((m + 3) / 4, 16384);  // slide: 4 waves each
    const unsigned gb = (unsigned)((n + kBoxBlock - 1) / kBoxBlock);
    k_mid_plan<D><<<gm, kMBlock, 0, stream>>>((int)m, seg, seg_split, na.box);
    k_mid_mark<<<gn1, kMBlock, 0, stream>>>(n, X[cur], sid, seg, seg_split, mark);
    if (exclusive_scan<int32_t>(mark, rank, n + 1, nullptr, scan_tmp, stream) != KDT_OK) {
      kdt_set_error("kdt_build (sliding midpoint): the scan of the marks failed");
      return KDT_EDEVICE;
    }
    k_mid_resolve<<<gm, kMBlock, 0, stream>>>((int)m, seg, seg_split, rank, res, node_base, level,
                                              na.node, na.axis, na.split);
    k_mid_slide<<<gs, kMBlock, 0, stream>>>((int)m, X[cur], Pm[cur], n, seg, seg_split, res,
                                            na.split);
    k_mid_scatter<D><<<gn, kMBlock, 0, stream>>>(n, X[cur], Pm[cur], sid, seg, res, mark, rank,
                                                 X[1 - cur], Pm[1 - cur], cid);
    cur = 1 - cur;
    k_mid_reset_keys<D><<<gk, kMBlock, 0, stream>>>(2 * m, ckeys);
    if (2 * m <= kRunBoxChildren) {
      const unsigned G = (unsigned)std::max<int64_t>(1, kRunBoxBlocks / (2 * m));
      k_mid_boxes_runs<D><<<dim3(G, (unsigned)(2 * m)), kBoxBlock, 0, stream>>>(
          n, X[cur], na.node, node_base, ckeys);
    } else {
      k_mid_boxes<D><<<gb, kBoxBlock, 0, stream>>>(n, X[cur], cid, ckeys);
    }
    k_mid_children<D><<<gc, kMBlock, 0, stream>>>((int)(2 * m), ckeys, node_base, leaf, na.node,
                                                  na.box, act);
    if (exclusive_scan<int32_t>(act, pos, 2 * m, nullptr, cscan_tmp, stream) != KDT_OK) {
      kdt_set_error("kdt_build (sliding midpoint): the scan of the children failed");
      return KDT_EDEVICE;
    }
    k_mid_compact<<<gc, kMBlock, 0, stream>>>((int)(2 * m), act, pos, node_base, na.node, nseg,
                                              d_count);
    k_mid_sid<<<gn, kMBlock, 0, stream>>>(n, cid, act, pos, sid);
    KDT_M(hipGetLastError());
    int32_t next = 0;
    KDT_M(hipMemcpyAsync(&next, d_count, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    KDT_M(hipStreamSynchronize(stream));
    node_base += 2 * m;
    ++level;
    std::swap(seg, nseg);
    m = next;
  }
  // the tree: records, order, node boxes, axes, splits, node records
  const int64_t nn = node_base;
  t->levels = level;
  t->n_nodes = nn;
  const size_t b_rec = sizeof(float) * (size_t)n * t->stride;
  const size_t b_box = sizeof(float) * (size_t)nn * 2 * P;
  const size_t b_perm = sizeof(int32_t) * (size_t)n;
  const size_t b_axis = sizeof(int32_t) * (size_t)nn;
  const size_t b_split = sizeof(float) * (size_t)nn;
  const size_t b_node = sizeof(int4) * (size_t)nn;
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  void* block = nullptr;
  if (dev_alloc(&block, up(b_rec) + up(b_box) + up(b_perm) + up(b_axis) + up(b_split) + up(b_node),
                stream) != hipSuccess) {
    kdt_set_error("kdt_build: cannot allocate the tree (%lld points)", (long long)n);
    return KDT_ENOMEM;
  }
  unsigned char* bp = static_cast<unsigned char*>(block);
  t->rec = reinterpret_cast<float*>(bp);
  t->box = reinterpret_cast<float*>(bp + up(b_rec));
  t->perm = reinterpret_cast<int32_t*>(bp + up(b_rec) + up(b_box));
  t->axis = reinterpret_cast<int32_t*>(bp + up(b_rec) + up(b_box) + up(b_perm));
  t->split = reinterpret_cast<float*>(bp + up(b_rec) + up(b_box) + up(b_perm) + up(b_axis));
  t->nodes = reinterpret_cast<int4*>(bp + up(b_rec) + up(b_box) + up(b_perm) + up(b_axis) +
                                     up(b_split));
  k_mid_records<D><<<gn, kMBlock, 0, stream>>>(n, X[cur], Pm[cur], t->rec, t->perm);
  hipError_t e = hipMemcpyAsync(t->box, na.box, b_box, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(t->axis, na.axis, b_axis, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(t->split, na.split, b_split, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(t->nodes, na.node, b_node, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    (void)hipFreeAsync(block, stream);
    t->rec = nullptr;
    kdt_set_error("kdt_build (sliding midpoint): %s", hipGetErrorString(e));
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

}  // namespace

kdt_status build_midpoint(const float* d_pts, int64_t n, int d, int leaf, bool check,
                          hipStream_t stream, kdt_tree* t) {
  switch (d) {
    case 2: return build_midpoint_d<2>(d_pts, n, leaf, check, stream, t);
    case 3: return build_midpoint_d<3>(d_pts, n, leaf, check, stream, t);
    case 4: return build_midpoint_d<4>(d_pts, n, leaf, check, stream, t);
    case 8: return build_midpoint_d<8>(d_pts, n, leaf, check, stream, t);
    case 16: return build_midpoint_d<16>(d_pts, n, leaf, check, stream, t);
  }
  kdt_set_error("kdt_build: unsupported dimension %d", d);
  return KDT_EUNSUPPORTED;
}

}  // namespace kdt
