// kdt_build.hip -- level-synchronous median k-d tree construction on gfx950.
//
// The tree of Sec. 2.1 / Algorithm 1 is built top-down, but with balanced
// splits: node (l, j) of a set of n points owns rows [floor(j n / 2^l),
// floor((j+1) n / 2^l)) of the tree order, is split along the longest side of
// its tight bounding box (lowest axis on ties) and sends its
// floor((2j+1) n / 2^(l+1)) - floor(j n / 2^l) smallest coordinates to the
// left child.  Because every node's size is known from n, the whole launch
// schedule is fixed on the host.
//
// Two phases:
//  * global levels -- nodes too large for one workgroup's LDS are split by
//    multi-workgroup kernels.  Workgroups never talk to each other inside a
//    launch (no device-scope fences or counters, which are expensive across
//    the chip's XCDs): every cross-workgroup sum goes through a kernel
//    boundary.  Per level: an init pass (one wave per node reduces the partial
//    boxes its points left behind, picks the axis), four 8-bit radix-select
//    passes over order-preserving uint32 keys of the split coordinate (each a
//    per-chunk histogram kernel plus a per-node select kernel), a per-chunk
//    count of keys below / equal to the pivot, and a stable scatter that
//    partitions each chunk in LDS and writes whole runs of the other
//    ping-pong buffer, leaving partial child boxes per chunk;
//  * LDS subtrees -- each node small enough to fit is loaded once into one
//    workgroup's LDS, which finishes all remaining levels there (one wave per
//    node; radix select or, for <= 64 points, rank counting) and writes the
//    final tree-ordered point records.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "kdt_internal.h"

namespace kdt {

constexpr int kChunk = 16384;  // rows per workgroup in the global-level passes
constexpr int kBuildBlock = 256;

int levels_for(int64_t n, int leaf) {
  int L = 0;
  while (((n + (int64_t(1) << L) - 1) >> L) > leaf) ++L;
  return L;
}

// Largest node handled inside one workgroup: coordinates and two uint16
// ping-pong index arrays fit in 32 KiB of LDS, so four workgroups share a CU
// (the subtree finish is bound by LDS latency, not by its instruction count).
int lds_capacity(int d) { return 32768 / (4 * d + 4); }

// LDS of a subtree workgroup whose largest node holds `cap` points.
static size_t lds_bytes(int d, int cap) {
  return (size_t)cap * 4 * d + 4 * 256 * 4 + (size_t)cap * 2 * 2;
}

bool make_plan(const int64_t* offsets, int n_sets, int d, const int* leaves, Plan& p,
               std::string& err) {
  p = Plan();
  p.d = d;
  p.leaf = 0;
  p.lds_cap = lds_capacity(d);
  p.total = offsets[n_sets] - offsets[0];
  int64_t nb = 0;
  for (int s = 0; s < n_sets; ++s) {
    SetDesc sd;
    sd.off = offsets[s];
    sd.n = offsets[s + 1] - offsets[s];
    if (sd.n < 1 || sd.n > INT32_MAX) {
      err = "every set must hold between 1 and 2^31-1 points";
      return false;
    }
    sd.levels = levels_for(sd.n, leaves[s]);
    p.leaf = std::max(p.leaf, leaves[s]);
    int g = 0;
    while (g < sd.levels && ((sd.n + (int64_t(1) << g) - 1) >> g) > p.lds_cap) ++g;
    sd.glevels = g;
    sd.node_base = nb;
    nb += (int64_t(2) << sd.levels) - 1;
    p.n_glevels = std::max(p.n_glevels, g);
    p.sets.push_back(sd);
  }
  p.n_nodes = nb;
  p.segs.resize(p.n_glevels);
  p.multi_chunk.assign(p.n_glevels, 0);
  p.chunks.resize(p.n_glevels);
  auto add_chunks = [](std::vector<ChunkEntry>& out, int64_t b, int64_t e, int32_t seg) {
    int64_t nch = std::max<int64_t>(1, (e - b + kChunk - 1) / kChunk);
    for (int64_t c = 0; c < nch; ++c) {
      ChunkEntry ce;
      ce.b = b + (e - b) * c / nch;
      ce.e = b + (e - b) * (c + 1) / nch;
      ce.seg = seg;
      ce.sole = nch == 1;
      out.push_back(ce);
    }
    return (int32_t)nch;
  };
  std::vector<int32_t> root_first(n_sets), root_count(n_sets);
  for (int s = 0; s < n_sets; ++s) {
    root_first[s] = (int32_t)p.root_chunks.size();
    root_count[s] = add_chunks(p.root_chunks, p.sets[s].off, p.sets[s].off + p.sets[s].n, s);
  }
  // index of each set's first segment in the previous level (for box sources)
  std::vector<int64_t> prev_first(n_sets, -1), cur_first(n_sets, -1);
  for (int l = 0; l < p.n_glevels; ++l) {
    for (int s = 0; s < n_sets; ++s) {
      const SetDesc& sd = p.sets[s];
      if (sd.glevels <= l) continue;
      cur_first[s] = (int64_t)p.segs[l].size();
      for (int64_t j = 0; j < (int64_t(1) << l); ++j) {
        SegEntry se;
        se.b = sd.off + node_begin(sd.n, l, j);
        se.e = sd.off + node_begin(sd.n, l, j + 1);
        se.m = sd.off + node_begin(sd.n, l + 1, 2 * j + 1);
        se.node = sd.node_base + (int64_t(1) << l) - 1 + j;
        se.child = (l + 1 < sd.glevels) ? sd.node_base + (int64_t(2) << l) - 1 + 2 * j : -1;
        se.first_chunk = (int32_t)p.chunks[l].size();
        se.n_chunks = add_chunks(p.chunks[l], se.b, se.e, (int32_t)p.segs[l].size());
        if (se.n_chunks > 1) p.multi_chunk[l] = 1;
        if (l == 0) {
          se.src_first = root_first[s];
          se.src_count = root_count[s];
          se.src_side = -1;
        } else {
          const SegEntry& par = p.segs[l - 1][prev_first[s] + (j >> 1)];
          se.src_first = par.first_chunk;
          se.src_count = par.n_chunks;
          se.src_side = (int32_t)(j & 1);
        }
        se.pad = 0;
        p.segs[l].push_back(se);
      }
    }
    prev_first = cur_first;
  }
  for (int s = 0; s < n_sets; ++s) {
    const SetDesc& sd = p.sets[s];
    for (int64_t j = 0; j < (int64_t(1) << sd.glevels); ++j) {
      SubEntry e;
      e.j = j;
      e.set = s;
      e.level = sd.glevels;
      p.subs.push_back(e);
      p.sub_max = std::max<int>(p.sub_max, (int)(node_begin(sd.n, sd.glevels, j + 1) -
                                                 node_begin(sd.n, sd.glevels, j)));
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// Wave / block helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ uint32_t wave_umin(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
  return v;
}
__device__ __forceinline__ uint32_t wave_umax(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
  return v;
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = (uint32_t)__shfl_up((int)v, o);
    if (lane >= o) v += t;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o);
  return v;
}

// Inclusive scan over the 256 threads of a block.  `tmp` holds 4 words.
__device__ __forceinline__ uint32_t block_incl_scan(uint32_t v, uint32_t* tmp) {
  const int wave = threadIdx.x >> 6, lane = lane_id();
  uint32_t inc = wave_incl_scan(v);
  if (lane == 63) tmp[wave] = inc;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wave; ++w) before += tmp[w];
  __syncthreads();
  return inc + before;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

constexpr int kBins = 256;       // 8-bit digits
constexpr int kRadixPasses = 4;  // 4 x 8 bits resolve a 32-bit key
constexpr int kPassUnroll = 8;   // rows per thread whose loads are in flight together

// Rows of one scatter tile: coordinates and index of the tile fit in 32 KiB.
template <int D>
__host__ __device__ constexpr int scatter_tile() {
  return (8192 / (D + 1)) / kBuildBlock * kBuildBlock > 0 ? (8192 / (D + 1)) / kBuildBlock * kBuildBlock
                                                          : kBuildBlock;
}

// Block-wide min/max of per-thread key boxes; the result lands in out[0..2D).
template <int D>
__device__ __forceinline__ void block_box(const uint32_t lo[D], const uint32_t hi[D],
                                          uint32_t* red /*[4][2D]*/, uint32_t* out) {
  const int wave = threadIdx.x >> 6, lane = lane_id();
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const uint32_t l = wave_umin(lo[a]), h = wave_umax(hi[a]);
    if (lane == 0) {
      red[wave * 2 * D + a] = l;
      red[wave * 2 * D + D + a] = h;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * D) {
    const int a = threadIdx.x;
    uint32_t v = red[a];
    for (int w = 1; w < 4; ++w) {
      const uint32_t u = red[w * 2 * D + a];
      v = a < D ? min(v, u) : max(v, u);
    }
    out[a] = v;
  }
  __syncthreads();
}

template <int D>
__global__ __launch_bounds__(kBuildBlock) void k_ingest(const ChunkEntry* __restrict__ chunks,
                                                        const SetDesc* __restrict__ sets,
                                                        const float* __restrict__ in,
                                                        float* __restrict__ x,
                                                        int32_t* __restrict__ perm, int64_t tot,
                                                        uint32_t* __restrict__ pbox,
                                                        int32_t* __restrict__ bad) {
  __shared__ uint32_t red[4 * 2 * D];
  const ChunkEntry ch = chunks[blockIdx.x];
  const SetDesc sd = sets[ch.seg];
  uint32_t lo[D], hi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lo[a] = 0xFFFFFFFFu;
    hi[a] = 0u;
  }
  bool nonfinite = false;
  for (int64_t i = ch.b + threadIdx.x; i < ch.e; i += kBuildBlock) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      // a non-finite coordinate is flagged and enters the build's copy as 0,
      // so that the later passes only ever see finite keys (a deferred or
      // skipped check builds a well-formed tree of meaningless points)
      const float raw = in[i * D + a];
      const bool fin = isfinite(raw);
      nonfinite |= !fin;
      const float v = fin ? raw : 0.0f;
      x[a * tot + i] = v;
      const uint32_t k = fkey(v);
      lo[a] = min(lo[a], k);
      hi[a] = max(hi[a], k);
    }
    perm[i] = (int32_t)(i - sd.off);
  }
  if (__any(nonfinite) && lane_id() == 0) atomicOr(bad, 1);
  block_box<D>(lo, hi, red, pbox + (int64_t)blockIdx.x * 2 * D);
}

// One wave per node: reduce the partial boxes of the node's points, write the
// node's box and split axis, and start its pivot selection.
template <int D>
__global__ __launch_bounds__(kBuildBlock) void k_level_init(const SegEntry* __restrict__ segs,
                                                            int nseg, SegState* __restrict__ st,
                                                            const uint32_t* __restrict__ pbox,
                                                            const uint32_t* __restrict__ cbox,
                                                            float* __restrict__ box,
                                                            int32_t* __restrict__ axis_out) {
  constexpr int P = pad4(D);
  const int wave = threadIdx.x >> 6, lane = lane_id();
  const int s = blockIdx.x * 4 + wave;
  if (s >= nseg) return;
  const SegEntry se = segs[s];
  uint32_t ulo[D], uhi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    ulo[a] = 0xFFFFFFFFu;
    uhi[a] = 0u;
  }
  for (int c = lane; c < se.src_count; c += kWave) {
    const uint32_t* src = se.src_side < 0 ? pbox + (int64_t)(se.src_first + c) * 2 * D
                                          : cbox + ((int64_t)(se.src_first + c) * 2 + se.src_side) * 2 * D;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      ulo[a] = min(ulo[a], src[a]);
      uhi[a] = max(uhi[a], src[D + a]);
    }
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    ulo[a] = wave_umin(ulo[a]);
    uhi[a] = wave_umax(uhi[a]);
  }
  int ax = 0;
  float ext = -1.0f;
  uint32_t klo = 0, khi = 0;
  float wv = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float lo = fkey_inv(ulo[a]), hi = fkey_inv(uhi[a]);
    const float e = hi - lo;
    if (e > ext) {
      ext = e;
      ax = a;
      klo = ulo[a];
      khi = uhi[a];
    }
    if (lane == a) wv = lo;
    if (lane == P + a) wv = hi;
  }
  if (lane < 2 * P) box[se.node * 2 * P + lane] = wv;
  if (lane == 0) {
    axis_out[se.node] = ax;
    const uint32_t xr = klo ^ khi;
    SegState ss;
    ss.hb = xr ? 31 - __clz(xr) : -1;
    ss.prefix = ss.hb >= 0 ? (klo & ~((2u << ss.hb) - 1u)) : klo;
    ss.rank = (int32_t)(se.m - se.b) - 1;
    ss.axis = ax;
    ss.n_eq_left = 0;
    ss.pad[0] = ss.pad[1] = ss.pad[2] = 0;
    st[s] = ss;
  }
}

// Histogram of the next 8-bit digit over one chunk (keys that match the
// resolved prefix only), written densely per chunk.  Lanes of a wave whose bin
// equals that of the wave's first valid lane add their count with one LDS
// atomic (clustered data puts most keys of a node in few bins).
template <int D>
__global__ __launch_bounds__(kBuildBlock) void k_hist(const ChunkEntry* __restrict__ chunks,
                                                      SegState* __restrict__ st,
                                                      const float* __restrict__ x, int64_t tot,
                                                      uint32_t* __restrict__ chist) {
  __shared__ uint32_t h[kBins];
  __shared__ uint32_t tmp[4];
  const ChunkEntry ch = chunks[blockIdx.x];
  const SegState s = st[ch.seg];
  if (s.hb < 0) return;
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int sh = s.hb >= 7 ? s.hb - 7 : 0;
  const uint32_t dmask = (1u << (s.hb - sh + 1)) - 1u;
  const uint64_t want = (uint64_t)s.prefix >> (s.hb + 1);
  const float* kx = x + (int64_t)s.axis * tot + ch.b;
  const int nr = (int)(ch.e - ch.b);
  for (int base = 0; base < nr; base += kBuildBlock * kPassUnroll) {
    // every load of the round is issued before the first is used (indexes
    // clamped into the chunk; rows past its end are masked afterwards)
    float v[kPassUnroll];
#pragma unroll
    for (int u = 0; u < kPassUnroll; ++u) v[u] = kx[min(base + u * kBuildBlock + tid, nr - 1)];
#pragma unroll
    for (int u = 0; u < kPassUnroll; ++u) {
      const uint32_t k = fkey(v[u]);
      const bool ok = base + u * kBuildBlock + tid < nr && ((uint64_t)k >> (s.hb + 1)) == want;
      const uint32_t bin = (k >> sh) & dmask;
      const uint64_t m_ok = __ballot(ok);
      if (m_ok == 0) continue;
      const uint32_t lead =
          (uint32_t)__builtin_amdgcn_readlane((int)bin, __ffsll((unsigned long long)m_ok) - 1);
      const bool same = ok && bin == lead;
      const uint64_t m = __ballot(same);
      if (same) {
        if (lanes_below(m) == 0) atomicAdd(&h[lead], (uint32_t)__popcll(m));
      } else if (ok) {
        atomicAdd(&h[bin], 1u);
      }
    }
  }
  __syncthreads();
  if (ch.sole) {
    // the node's only chunk: narrow its selection state here
    const uint32_t c = h[tid];
    const uint32_t inc = block_incl_scan(c, tmp);
    const uint32_t exc = inc - c;
    const uint32_t r = (uint32_t)s.rank;
    if (exc <= r && r < inc) {
      SegState* o = st + ch.seg;
      o->prefix = s.prefix | ((uint32_t)tid << sh);
      o->rank = (int32_t)(r - exc);
      o->hb = sh - 1;
    }
    return;
  }
  chist[(int64_t)blockIdx.x * kBins + tid] = h[tid];
}

// One workgroup per node of more than one chunk: sum the chunk histograms,
// find the digit bin that holds the pivot's rank and narrow the selection
// state.  Top-level nodes own hundreds of chunks: each wave reads whole chunk
// histograms as 16-byte quads of bins, kSelUnroll chunks in flight.
constexpr int kSelBlock = 1024;
constexpr int kSelQuads = kBins / 4;
constexpr int kSelGroups = kSelBlock / kSelQuads;
constexpr int kSelUnroll = 8;
__global__ __launch_bounds__(kSelBlock) void k_select(const SegEntry* __restrict__ segs,
                                                      SegState* __restrict__ st,
                                                      const uint32_t* __restrict__ chist) {
  __shared__ uint4 part[kSelGroups][kSelQuads];
  __shared__ uint32_t tmp[kBins / kWave];
  const int tid = threadIdx.x;
  const SegEntry se = segs[blockIdx.x];
  if (se.n_chunks == 1) return;  // resolved by its histogram pass
  const SegState s = st[blockIdx.x];
  if (s.hb < 0) return;
  const int quad = tid % kSelQuads, grp = tid / kSelQuads;
  const uint4* hp = reinterpret_cast<const uint4*>(chist + (int64_t)se.first_chunk * kBins) + quad;
  uint4 c = make_uint4(0, 0, 0, 0);
  int q = grp;
  for (; q + kSelGroups * (kSelUnroll - 1) < se.n_chunks; q += kSelGroups * kSelUnroll) {
    uint4 v[kSelUnroll];
#pragma unroll
    for (int u = 0; u < kSelUnroll; ++u) v[u] = hp[(int64_t)(q + u * kSelGroups) * kSelQuads];
#pragma unroll
    for (int u = 0; u < kSelUnroll; ++u) {
      c.x += v[u].x;
      c.y += v[u].y;
      c.z += v[u].z;
      c.w += v[u].w;
    }
  }
  for (; q < se.n_chunks; q += kSelGroups) {
    const uint4 v = hp[(int64_t)q * kSelQuads];
    c.x += v.x;
    c.y += v.y;
    c.z += v.z;
    c.w += v.w;
  }
  part[grp][quad] = c;
  __syncthreads();
  const int wave = tid >> 6, lane = lane_id();
  uint32_t sum = 0, inc = 0;
  if (tid < kBins) {
#pragma unroll
    for (int g = 0; g < kSelGroups; ++g) sum += reinterpret_cast<const uint32_t*>(part[g])[tid];
    inc = wave_incl_scan(sum);
    if (lane == kWave - 1) tmp[wave] = inc;
  }
  __syncthreads();
  if (tid < kBins) {
    for (int w = 0; w < wave; ++w) inc += tmp[w];
    const uint32_t exc = inc - sum;
    const uint32_t r = (uint32_t)s.rank;
    if (exc <= r && r < inc) {
      const int sh = s.hb >= 7 ? s.hb - 7 : 0;
      SegState* o = st + blockIdx.x;
      o->prefix = s.prefix | ((uint32_t)tid << sh);
      o->rank = (int32_t)(r - exc);
      o->hb = sh - 1;
    }
  }
}

// Keys below / equal to the pivot in each chunk.
template <int D>
__global__ __launch_bounds__(kBuildBlock) void k_count(const ChunkEntry* __restrict__ chunks,
                                                       const SegEntry* __restrict__ segs,
                                                       const SegState* __restrict__ st,
                                                       const float* __restrict__ x, int64_t tot,
                                                       int32_t* __restrict__ cnt,
                                                       float* __restrict__ split_out) {
  __shared__ uint32_t red[2][4];
  const int tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
  const ChunkEntry ch = chunks[blockIdx.x];
  const SegState s = st[ch.seg];
  const uint32_t pivot = s.prefix;
  const float* kx = x + (int64_t)s.axis * tot + ch.b;
  const int nr = (int)(ch.e - ch.b);
  uint32_t nl = 0, ne = 0;
  for (int base = 0; base < nr; base += kBuildBlock * kPassUnroll) {
    float v[kPassUnroll];
#pragma unroll
    for (int u = 0; u < kPassUnroll; ++u) v[u] = kx[min(base + u * kBuildBlock + tid, nr - 1)];
#pragma unroll
    for (int u = 0; u < kPassUnroll; ++u) {
      const uint32_t k = fkey(v[u]);
      const bool valid = base + u * kBuildBlock + tid < nr;
      nl += valid && k < pivot;
      ne += valid && k == pivot;
    }
  }
  nl = wave_sum(nl);
  ne = wave_sum(ne);
  if (lane == 0) {
    red[0][wave] = nl;
    red[1][wave] = ne;
  }
  __syncthreads();
  if (tid == 0) {
    cnt[2 * blockIdx.x] = (int32_t)(red[0][0] + red[0][1] + red[0][2] + red[0][3]);
    cnt[2 * blockIdx.x + 1] = (int32_t)(red[1][0] + red[1][1] + red[1][2] + red[1][3]);
    const SegEntry se = segs[ch.seg];
    if (blockIdx.x == (unsigned)se.first_chunk) split_out[se.node] = fkey_inv(pivot);
  }
}

// Stable partition of each chunk around its node's pivot.  A tile of rows is
// partitioned inside LDS (left rows first, both in input order) and then
// written as two contiguous runs per coordinate array, so every global store
// is coalesced.  The chunk's left and right boxes are left in cbox.
template <int D>
__global__ __launch_bounds__(kBuildBlock) void k_scatter(const ChunkEntry* __restrict__ chunks,
                                                         const SegEntry* __restrict__ segs,
                                                         const SegState* __restrict__ st,
                                                         const int32_t* __restrict__ cnt,
                                                         const float* __restrict__ xin,
                                                         const int32_t* __restrict__ pin,
                                                         float* __restrict__ xout,
                                                         int32_t* __restrict__ pout, int64_t tot,
                                                         uint32_t* __restrict__ cbox,
                                                         int32_t* __restrict__ bad) {
  constexpr int T = scatter_tile<D>();
  constexpr int R = T / kBuildBlock;  // rows per thread in a tile
  __shared__ float sx[D][T];
  __shared__ int32_t sp[T];
  __shared__ uint32_t tmp[4];
  __shared__ uint32_t red[4 * 2 * D];
  __shared__ uint4 wcnt[2][R];  // per round of rows: counts of the four waves (equal, left)
  __shared__ int64_t pre[2];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const ChunkEntry ch = chunks[blockIdx.x];
  const SegEntry se = segs[ch.seg];
  const SegState s = st[ch.seg];
  const uint32_t pivot = s.prefix;
  const int64_t n_eq_left = (int64_t)s.rank + 1;
  // keys below / equal to the pivot in the earlier chunks of this node
  {
    uint32_t nl = 0, ne = 0;
    for (int c = se.first_chunk + tid; c < (int)blockIdx.x; c += kBuildBlock) {
      nl += (uint32_t)cnt[2 * c];
      ne += (uint32_t)cnt[2 * c + 1];
    }
    const uint32_t il = block_incl_scan(nl, tmp);
    const uint32_t ie = block_incl_scan(ne, tmp);
    if (tid == kBuildBlock - 1) {
      pre[0] = il;
      pre[1] = ie;
    }
    __syncthreads();
  }
  const int64_t less_before = pre[0], eq_before = pre[1];
  const int64_t left_before = less_before + min(eq_before, n_eq_left);
  const int64_t right_before = (ch.b - se.b) - left_before;
  uint32_t lmin[D], lmax[D], rmin[D], rmax[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lmin[a] = rmin[a] = 0xFFFFFFFFu;
    lmax[a] = rmax[a] = 0u;
  }
  // Rows of a tile are dealt out round by round (row r * 256 + tid), so every
  // load is coalesced; ballots give each row its rank in input order.
  int64_t run_left = 0, run_right = 0, run_eq = 0;
  for (int64_t base = ch.b; base < ch.e; base += T) {
    const int nt = (int)min((int64_t)T, ch.e - base);
    float v[R][D];
    int32_t p[R];
    uint32_t key[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = r * kBuildBlock + tid;
      const int64_t row = base + (i < nt ? i : 0);
#pragma unroll
      for (int a = 0; a < D; ++a) v[r][a] = xin[a * tot + row];
      p[r] = pin[row];
    }
    uint32_t below_eq[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float kv = v[r][0];
#pragma unroll
      for (int a = 1; a < D; ++a) kv = a == s.axis ? v[r][a] : kv;
      key[r] = fkey(kv);
      const bool eq = r * kBuildBlock + tid < nt && key[r] == pivot;
      const uint64_t b = __ballot(eq);
      below_eq[r] = (uint32_t)lanes_below(b);
      if (lane == 0) (&wcnt[0][r].x)[wave] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    uint32_t acc = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint4 c = wcnt[0][r];
      below_eq[r] += acc + (wave > 0 ? c.x : 0) + (wave > 1 ? c.y : 0) + (wave > 2 ? c.z : 0);
      acc += c.x + c.y + c.z + c.w;
    }
    const uint32_t tile_eq = acc;
    uint32_t below_left[R];
    uint32_t left_bits = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool valid = r * kBuildBlock + tid < nt;
      const bool eq = valid && key[r] == pivot;
      const bool left =
          valid && (key[r] < pivot || (eq && eq_before + run_eq + (int64_t)below_eq[r] < n_eq_left));
      left_bits |= (uint32_t)left << r;
      const uint64_t b = __ballot(left);
      below_left[r] = (uint32_t)lanes_below(b);
      if (lane == 0) (&wcnt[1][r].x)[wave] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    acc = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint4 c = wcnt[1][r];
      below_left[r] += acc + (wave > 0 ? c.x : 0) + (wave > 1 ? c.y : 0) + (wave > 2 ? c.z : 0);
      acc += c.x + c.y + c.z + c.w;
    }
    const int tl = (int)acc;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = r * kBuildBlock + tid;
      if (i >= nt) break;
      const bool left = (left_bits >> r) & 1u;
      const int dst = left ? (int)below_left[r] : tl + (i - (int)below_left[r]);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        sx[a][dst] = v[r][a];
        const uint32_t kv = fkey(v[r][a]);
        if (left) {
          lmin[a] = min(lmin[a], kv);
          lmax[a] = max(lmax[a], kv);
        } else {
          rmin[a] = min(rmin[a], kv);
          rmax[a] = max(rmax[a], kv);
        }
      }
      sp[dst] = p[r];
    }
    __syncthreads();
    for (int i = tid; i < nt; i += kBuildBlock) {
      int64_t g = i < tl ? se.b + left_before + run_left + i : se.m + right_before + run_right + (i - tl);
      if (g < se.b || g >= se.e) {  // cannot happen; keeps a logic slip in bounds
        atomicOr(bad, 2);
        g = se.b;
      }
#pragma unroll
      for (int a = 0; a < D; ++a) xout[a * tot + g] = sx[a][i];
      pout[g] = sp[i];
    }
    run_eq += tile_eq;
    run_left += tl;
    run_right += nt - tl;
    __syncthreads();
  }
  if (se.child >= 0) {
    uint32_t* c = cbox + (int64_t)blockIdx.x * 4 * D;
    block_box<D>(lmin, lmax, red, c);
    block_box<D>(rmin, rmax, red, c + 2 * D);
  }
}

// Finishes every level below a node inside one workgroup's LDS and writes the
// final tree-ordered records.
template <int D>
__global__ __launch_bounds__(kBuildBlock) void k_lds_subtree(
    const SubEntry* __restrict__ subs, const SetDesc* __restrict__ sets,
    const float* __restrict__ x0, const int32_t* __restrict__ p0, const float* __restrict__ x1,
    const int32_t* __restrict__ p1, int64_t tot, int cap, float* __restrict__ box,
    int32_t* __restrict__ axis_out, float* __restrict__ split_out, float* __restrict__ rec,
    int32_t* __restrict__ perm_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int P = pad4(D);
  constexpr int S = rec_stride(D);
  float* lx = reinterpret_cast<float*>(smem);
  uint32_t* hist = reinterpret_cast<uint32_t*>(lx + (size_t)D * cap);
  uint16_t* lpa = reinterpret_cast<uint16_t*>(hist + 4 * 256);
  uint16_t* lpb = lpa + cap;

  const SubEntry se = subs[blockIdx.x];
  const SetDesc sd = sets[se.set];
  const float* xin = (sd.glevels & 1) ? x1 : x0;
  const int32_t* pin = (sd.glevels & 1) ? p1 : p0;
  const int64_t g0 = sd.off + node_begin(sd.n, se.level, se.j);
  const int m = (int)(sd.off + node_begin(sd.n, se.level, se.j + 1) - g0);
  for (int i = threadIdx.x; i < m; i += kBuildBlock) {
#pragma unroll
    for (int a = 0; a < D; ++a) lx[a * cap + i] = xin[a * tot + g0 + i];
    lpa[i] = (uint16_t)i;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = lane_id();
  uint32_t* h = hist + wave * 256;
  uint16_t* cur = lpa;
  uint16_t* nxt = lpb;
  for (int lev = se.level; lev <= sd.levels; ++lev) {
    const int depth = lev - se.level;
    const int64_t nn = int64_t(1) << depth;
    for (int64_t kk = wave; kk < nn; kk += 4) {
      const int64_t j = (se.j << depth) + kk;
      const int lb = (int)(sd.off + node_begin(sd.n, lev, j) - g0);
      const int le = (int)(sd.off + node_begin(sd.n, lev, j + 1) - g0);
      const int64_t node = sd.node_base + (int64_t(1) << lev) - 1 + j;
      float lo[D], hi[D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        lo[a] = INFINITY;
        hi[a] = -INFINITY;
      }
      for (int i = lb + lane; i < le; i += kWave) {
        const int s = cur[i];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          float v = lx[a * cap + s];
          lo[a] = fminf(lo[a], v);
          hi[a] = fmaxf(hi[a], v);
        }
      }
      int ax = 0;
      float ext = -1.0f, alo = 0.0f, ahi = 0.0f;
      float wv = 0.0f;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        lo[a] = wave_min(lo[a]);
        hi[a] = wave_max(hi[a]);
        float e = hi[a] - lo[a];
        if (e > ext) {
          ext = e;
          ax = a;
          alo = lo[a];
          ahi = hi[a];
        }
        if (lane == a) wv = lo[a];
        if (lane == P + a) wv = hi[a];
      }
      if (lane < 2 * P) box[node * 2 * P + lane] = wv;
      if (lev == sd.levels) {
        if (lane == 0) {
          axis_out[node] = -1;
          split_out[node] = 0.0f;
        }
        continue;
      }
      const int nl = (int)(sd.off + node_begin(sd.n, lev + 1, 2 * j + 1) - g0) - lb;
      const float* kx = lx + ax * cap;
      const int msz = le - lb;
      uint32_t pivot;
      if (msz <= kWave) {
        // rank counting: the node comes out sorted along the axis
        const uint32_t key = lane < msz ? fkey(kx[cur[lb + lane]]) : 0xFFFFFFFFu;
        int rank = 0;
        for (int t = 0; t < msz; ++t) {
          uint32_t kt = (uint32_t)__builtin_amdgcn_readlane((int)key, t);
          rank += (kt < key) || (kt == key && t < lane);
        }
        if (lane < msz && rank < msz) nxt[lb + rank] = cur[lb + lane];
        const uint64_t bal = __ballot(lane < msz && rank == nl - 1);
        const int src = __ffsll((unsigned long long)bal) - 1;
        pivot = (uint32_t)__builtin_amdgcn_readlane((int)key, src);
      } else {
        const uint32_t klo = fkey(alo), khi = fkey(ahi);
        const uint32_t xr = klo ^ khi;
        int hb = xr ? 31 - __clz(xr) : -1;
        uint32_t prefix = hb >= 0 ? (klo & ~((2u << hb) - 1u)) : klo;
        int rank = nl - 1;
        while (hb >= 0) {
          const int sh = hb >= 7 ? hb - 7 : 0;
          const uint32_t dmask = (1u << (hb - sh + 1)) - 1u;
          const uint64_t want = (uint64_t)prefix >> (hb + 1);
          for (int b = lane; b < 256; b += kWave) h[b] = 0;
          wave_sync();
          // four rounds of loads before their atomics
          int i = lb + lane;
          for (; i + 3 * kWave < le; i += 4 * kWave) {
            uint32_t k[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) k[u] = fkey(kx[cur[i + u * kWave]]);
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (((uint64_t)k[u] >> (hb + 1)) == want) atomicAdd(&h[(k[u] >> sh) & dmask], 1u);
          }
          for (; i < le; i += kWave) {
            uint32_t k = fkey(kx[cur[i]]);
            if (((uint64_t)k >> (hb + 1)) == want) atomicAdd(&h[(k >> sh) & dmask], 1u);
          }
          wave_sync();
          const uint32_t c0 = h[4 * lane], c1 = h[4 * lane + 1], c2 = h[4 * lane + 2],
                         c3 = h[4 * lane + 3];
          const uint32_t sum = c0 + c1 + c2 + c3;
          const uint32_t inc = wave_incl_scan(sum);
          const uint32_t exc = inc - sum;
          const bool hit = exc <= (uint32_t)rank && (uint32_t)rank < inc;
          uint32_t r = (uint32_t)rank - exc;
          int b = 0;
          if (r >= c0) {
            r -= c0;
            b = 1;
            if (r >= c1) {
              r -= c1;
              b = 2;
              if (r >= c2) {
                r -= c2;
                b = 3;
              }
            }
          }
          const uint64_t bal = __ballot(hit);
          const int src = __ffsll((unsigned long long)bal) - 1;
          const int bin = __builtin_amdgcn_readlane(4 * lane + b, src);
          rank = __builtin_amdgcn_readlane((int)r, src);
          prefix |= (uint32_t)bin << sh;
          hb = sh - 1;
          wave_sync();
        }
        pivot = prefix;
        const int n_eq_left = rank + 1;
        int run_left = 0, run_right = 0, run_eq = 0;
        for (int base = lb; base < le; base += kWave) {
          const int i = base + lane;
          const bool valid = i < le;
          const uint16_t s = valid ? cur[i] : (uint16_t)0;
          const uint32_t k = valid ? fkey(kx[s]) : 0xFFFFFFFFu;
          const bool less = valid && k < pivot;
          const bool eq = valid && k == pivot;
          const uint64_t be = __ballot(eq);
          const int eq_rank = run_eq + lanes_below(be);
          const bool left = less || (eq && eq_rank < n_eq_left);
          const uint64_t bl = __ballot(left);
          const int lpos = lanes_below(bl);
          if (valid) {
            const int dst = left ? lb + run_left + lpos : lb + nl + run_right + (lane - lpos);
            if (dst >= lb && dst < le) nxt[dst] = s;
          }
          const int nvalid = min(kWave, le - base);
          run_eq += __popcll(be);
          run_left += __popcll(bl);
          run_right += nvalid - __popcll(bl);
        }
      }
      if (lane == 0) {
        axis_out[node] = ax;
        split_out[node] = fkey_inv(pivot);
      }
    }
    __syncthreads();
    if (lev < sd.levels) {
      uint16_t* t = cur;
      cur = nxt;
      nxt = t;
    }
  }
  for (int i = threadIdx.x; i < m; i += kBuildBlock) {
    const int s = cur[i];
    const int64_t row = g0 + i;
    float r[S];
#pragma unroll
    for (int a = 0; a < S; ++a) r[a] = 0.0f;
#pragma unroll
    for (int a = 0; a < D; ++a) r[a] = lx[a * cap + s];
    const int32_t id = pin[g0 + s];
    r[D] = __int_as_float(id);
    float4* dst = reinterpret_cast<float4*>(rec + row * S);
#pragma unroll
    for (int q = 0; q < S / 4; ++q) dst[q] = make_float4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
    perm_out[row] = id;
  }
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------

#define KDT_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      kdt_set_error("%s failed: %s", #call, hipGetErrorString(e_));          \
      return KDT_EDEVICE;                                                    \
    }                                                                        \
  } while (0)

kdt_status plan_upload(const Plan& p, PlanDev& pd, hipStream_t stream) {
  size_t bytes = 0;
  auto take = [&](size_t b) {
    size_t o = bytes;
    bytes += (b + 255) & ~size_t(255);
    return o;
  };
  size_t o_sets = take(sizeof(SetDesc) * p.sets.size());
  size_t o_root = take(sizeof(ChunkEntry) * p.root_chunks.size());
  std::vector<size_t> o_segs, o_chunks;
  pd.max_segs = pd.max_chunks = 1;
  for (int l = 0; l < p.n_glevels; ++l) {
    o_segs.push_back(take(sizeof(SegEntry) * p.segs[l].size()));
    o_chunks.push_back(take(sizeof(ChunkEntry) * p.chunks[l].size()));
    pd.max_segs = std::max(pd.max_segs, p.segs[l].size());
    pd.max_chunks = std::max(pd.max_chunks, p.chunks[l].size());
  }
  size_t o_subs = take(sizeof(SubEntry) * p.subs.size());
  std::vector<unsigned char> host(bytes);
  memcpy(host.data() + o_sets, p.sets.data(), sizeof(SetDesc) * p.sets.size());
  memcpy(host.data() + o_root, p.root_chunks.data(), sizeof(ChunkEntry) * p.root_chunks.size());
  for (int l = 0; l < p.n_glevels; ++l) {
    memcpy(host.data() + o_segs[l], p.segs[l].data(), sizeof(SegEntry) * p.segs[l].size());
    memcpy(host.data() + o_chunks[l], p.chunks[l].data(), sizeof(ChunkEntry) * p.chunks[l].size());
  }
  memcpy(host.data() + o_subs, p.subs.data(), sizeof(SubEntry) * p.subs.size());
  if (hipMalloc(&pd.block, bytes) != hipSuccess) {
    kdt_set_error("cannot allocate %zu bytes for the build schedule", bytes);
    return KDT_ENOMEM;
  }
  KDT_HIP(hipMemcpy(pd.block, host.data(), bytes, hipMemcpyHostToDevice));
  unsigned char* base = static_cast<unsigned char*>(pd.block);
  pd.sets = reinterpret_cast<SetDesc*>(base + o_sets);
  pd.root_chunks = reinterpret_cast<ChunkEntry*>(base + o_root);
  pd.segs.resize(p.n_glevels);
  pd.chunks.resize(p.n_glevels);
  for (int l = 0; l < p.n_glevels; ++l) {
    pd.segs[l] = reinterpret_cast<SegEntry*>(base + o_segs[l]);
    pd.chunks[l] = reinterpret_cast<ChunkEntry*>(base + o_chunks[l]);
  }
  pd.subs = reinterpret_cast<SubEntry*>(base + o_subs);
  (void)stream;
  return KDT_OK;
}

void plan_release(PlanDev& pd) {
  if (pd.block) (void)hipFree(pd.block);
  pd = PlanDev();
}

template <int D>
static kdt_status run_build(const Plan& p, const PlanDev& pd, const float* d_pts,
                            const BuildScratch& w, const BuildOut& o, int phase,
                            hipStream_t stream) {
  const int64_t tot = p.total;
  if (phase == 0) {
    k_ingest<D><<<(unsigned)p.root_chunks.size(), kBuildBlock, 0, stream>>>(
        pd.root_chunks, pd.sets, d_pts, w.x[0], w.p[0], tot, w.pbox, w.bad);
    KDT_HIP(hipGetLastError());
    return KDT_OK;
  }
  for (int l = 0; l < p.n_glevels; ++l) {
    const int nseg = (int)p.segs[l].size();
    const unsigned nch = (unsigned)p.chunks[l].size();
    const int src = l & 1, dst = src ^ 1;
    k_level_init<D><<<(nseg + 3) / 4, kBuildBlock, 0, stream>>>(pd.segs[l], nseg, w.st, w.pbox,
                                                                w.cbox, o.box, o.axis);
    for (int pass = 0; pass < kRadixPasses; ++pass) {
      k_hist<D><<<nch, kBuildBlock, 0, stream>>>(pd.chunks[l], w.st, w.x[src], tot, w.chist);
      if (p.multi_chunk[l])
        k_select<<<nseg, kSelBlock, 0, stream>>>(pd.segs[l], w.st, w.chist);
    }
    k_count<D><<<nch, kBuildBlock, 0, stream>>>(pd.chunks[l], pd.segs[l], w.st, w.x[src], tot,
                                                w.cnt, o.split);
    k_scatter<D><<<nch, kBuildBlock, 0, stream>>>(pd.chunks[l], pd.segs[l], w.st, w.cnt,
                                                  w.x[src], w.p[src], w.x[dst], w.p[dst], tot,
                                                  w.cbox, w.bad);
  }
  const size_t smem = lds_bytes(D, p.sub_max);
  k_lds_subtree<D><<<(unsigned)p.subs.size(), kBuildBlock, smem, stream>>>(
      pd.subs, pd.sets, w.x[0], w.p[0], w.x[1], w.p[1], tot, p.sub_max, o.box, o.axis, o.split,
      o.rec, o.perm);
  KDT_HIP(hipGetLastError());
  return KDT_OK;
}

template <int D>
static void set_smem_attr(int cap) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lds_subtree<D>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes(D, cap));
}

hipError_t dev_alloc(void** ptr, size_t bytes, hipStream_t stream) {
  if (alloc_should_fail()) return hipErrorOutOfMemory;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t keep = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
  });
  return hipMallocAsync(ptr, std::max<size_t>(bytes, 256), stream);
}

kdt_status build_scratch_alloc(const Plan& p, const PlanDev& pd, BuildScratch& w,
                               hipStream_t stream) {
  const int64_t tot = p.total;
  const int d = p.d;
  auto A = [&](void** ptr, size_t bytes) -> bool {
    if (stream == kPlainAlloc) return hipMalloc(ptr, std::max<size_t>(bytes, 256)) == hipSuccess;
    return dev_alloc(ptr, bytes, stream) == hipSuccess;
  };
  const int64_t nroot = (int64_t)p.root_chunks.size();
  bool ok = A((void**)&w.x[0], sizeof(float) * d * tot) && A((void**)&w.x[1], sizeof(float) * d * tot) &&
            A((void**)&w.p[0], sizeof(int32_t) * tot) && A((void**)&w.p[1], sizeof(int32_t) * tot) &&
            A((void**)&w.pbox, sizeof(uint32_t) * 2 * d * nroot) &&
            A((void**)&w.cbox, sizeof(uint32_t) * 4 * d * pd.max_chunks) &&
            A((void**)&w.st, sizeof(SegState) * pd.max_segs) &&
            A((void**)&w.chist, sizeof(uint32_t) * kBins * pd.max_chunks) &&
            A((void**)&w.cnt, sizeof(int32_t) * 2 * pd.max_chunks) && A((void**)&w.bad, 256);
  if (!ok) {
    build_scratch_free(w, stream);
    kdt_set_error("device allocation failed for the build scratch (%lld points)", (long long)tot);
    return KDT_ENOMEM;
  }
  return KDT_OK;
}

void build_scratch_free(BuildScratch& w, hipStream_t stream) {
  void* ptrs[] = {w.x[0], w.x[1], w.p[0], w.p[1], w.pbox, w.cbox, w.st, w.chist, w.cnt, w.bad};
  for (void* q : ptrs)
    if (q) (void)(stream == kPlainAlloc ? hipFree(q) : hipFreeAsync(q, stream));
  w = BuildScratch();
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

static void zero_u32(uint32_t* p, int64_t n, hipStream_t stream) {
  if (n <= 0) return;
  k_zero_u32<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(p, n);
}

void build_init_once() {
  static std::once_flag attr_once;
  std::call_once(attr_once, [] {
    set_smem_attr<2>(lds_capacity(2));
    set_smem_attr<3>(lds_capacity(3));
    set_smem_attr<4>(lds_capacity(4));
    set_smem_attr<8>(lds_capacity(8));
    set_smem_attr<16>(lds_capacity(16));
  });
}

kdt_status build_launch(const Plan& p, const PlanDev& pd, const float* d_pts,
                        const BuildScratch& w, const BuildOut& o, int phase, hipStream_t stream) {
  if (phase == 0) zero_u32(reinterpret_cast<uint32_t*>(w.bad), 1, stream);
  build_init_once();
  switch (p.d) {
    case 2: return run_build<2>(p, pd, d_pts, w, o, phase, stream);
    case 3: return run_build<3>(p, pd, d_pts, w, o, phase, stream);
    case 4: return run_build<4>(p, pd, d_pts, w, o, phase, stream);
    case 8: return run_build<8>(p, pd, d_pts, w, o, phase, stream);
    case 16: return run_build<16>(p, pd, d_pts, w, o, phase, stream);
    default:
      kdt_set_error("unsupported dimension %d", p.d);
      return KDT_EUNSUPPORTED;
  }
}

}  // namespace kdt
