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
//    multi-workgroup kernels: per level an init pass (box, axis), up to four
//    8-bit radix-select passes over order-preserving uint32 keys of the split
//    coordinate (histograms merged by the last workgroup of each node), a
//    count pass and a stable scatter of the SoA coordinates and indices into
//    the other ping-pong buffer, which also accumulates the children's tight
//    boxes;
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

constexpr int kChunk = 4096;  // rows per workgroup in the global-level passes
constexpr int kBuildBlock = 256;

int levels_for(int64_t n, int leaf) {
  int L = 0;
  while (((n + (int64_t(1) << L) - 1) >> L) > leaf) ++L;
  return L;
}

// Largest node handled inside one workgroup: coordinates, index and two
// uint16 ping-pong index arrays must fit in ~60 KiB of LDS.
int lds_capacity(int d) { return (61440) / (4 * d + 8); }

static size_t lds_bytes(int d, int cap) {
  return (size_t)cap * (4 * d + 4) + 4 * 256 * 4 + (size_t)cap * 2 * 2;
}

bool make_plan(const int64_t* offsets, int n_sets, int d, int leaf, Plan& p, std::string& err) {
  p = Plan();
  p.d = d;
  p.leaf = leaf;
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
    sd.levels = levels_for(sd.n, leaf);
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
  p.chunks.resize(p.n_glevels);
  auto add_chunks = [](std::vector<ChunkEntry>& out, int64_t b, int64_t e, int32_t seg) {
    int64_t nch = std::max<int64_t>(1, (e - b + kChunk - 1) / kChunk);
    for (int64_t c = 0; c < nch; ++c) {
      ChunkEntry ce;
      ce.b = b + (e - b) * c / nch;
      ce.e = b + (e - b) * (c + 1) / nch;
      ce.seg = seg;
      ce.pad = 0;
      out.push_back(ce);
    }
    return (int32_t)nch;
  };
  for (int s = 0; s < n_sets; ++s) add_chunks(p.root_chunks, p.sets[s].off, p.sets[s].off + p.sets[s].n, s);
  for (int l = 0; l < p.n_glevels; ++l) {
    for (int s = 0; s < n_sets; ++s) {
      const SetDesc& sd = p.sets[s];
      if (sd.glevels <= l) continue;
      for (int64_t j = 0; j < (int64_t(1) << l); ++j) {
        SegEntry se;
        se.b = sd.off + node_begin(sd.n, l, j);
        se.e = sd.off + node_begin(sd.n, l, j + 1);
        se.m = sd.off + node_begin(sd.n, l + 1, 2 * j + 1);
        se.node = sd.node_base + (int64_t(1) << l) - 1 + j;
        se.child = (l + 1 < sd.glevels) ? sd.node_base + (int64_t(2) << l) - 1 + 2 * j : -1;
        se.first_chunk = (int32_t)p.chunks[l].size();
        se.n_chunks = add_chunks(p.chunks[l], se.b, se.e, (int32_t)p.segs[l].size());
        p.segs[l].push_back(se);
      }
    }
  }
  for (int s = 0; s < n_sets; ++s) {
    const SetDesc& sd = p.sets[s];
    for (int64_t j = 0; j < (int64_t(1) << sd.glevels); ++j) {
      SubEntry e;
      e.j = j;
      e.set = s;
      e.level = sd.glevels;
      p.subs.push_back(e);
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

template <int D>
__global__ void k_init_roots(const SetDesc* __restrict__ sets, int n_sets, uint32_t* __restrict__ ubox) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sets) return;
  uint32_t* u = ubox + sets[s].node_base * 2 * D;
  for (int a = 0; a < D; ++a) {
    u[a] = 0xFFFFFFFFu;
    u[D + a] = 0u;
  }
}

template <int D>
__global__ __launch_bounds__(kBuildBlock) void k_ingest(const ChunkEntry* __restrict__ chunks,
                                                        const SetDesc* __restrict__ sets,
                                                        const float* __restrict__ in,
                                                        float* __restrict__ x,
                                                        int32_t* __restrict__ perm, int64_t tot,
                                                        uint32_t* __restrict__ ubox,
                                                        int32_t* __restrict__ bad) {
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
      float v = in[i * D + a];
      nonfinite |= !isfinite(v);
      x[a * tot + i] = v;
      uint32_t k = fkey(v);
      lo[a] = min(lo[a], k);
      hi[a] = max(hi[a], k);
    }
    perm[i] = (int32_t)(i - sd.off);
  }
  if (__any(nonfinite) && lane_id() == 0) atomicOr(bad, 1);
  uint32_t* u = ubox + sd.node_base * 2 * D;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    uint32_t l = wave_umin(lo[a]), h = wave_umax(hi[a]);
    if (lane_id() == 0) {
      atomicMin(u + a, l);
      atomicMax(u + D + a, h);
    }
  }
}

template <int D>
__global__ void k_level_init(const SegEntry* __restrict__ segs, int nseg, SegState* __restrict__ st,
                             uint32_t* __restrict__ ubox, float* __restrict__ box,
                             int32_t* __restrict__ axis_out) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  constexpr int P = pad4(D);
  const SegEntry se = segs[s];
  const uint32_t* u = ubox + se.node * 2 * D;
  float lo[D], hi[D];
  uint32_t klo = 0, khi = 0;
  int ax = 0;
  float ext = -1.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lo[a] = fkey_inv(u[a]);
    hi[a] = fkey_inv(u[D + a]);
    float e = hi[a] - lo[a];
    if (e > ext) {
      ext = e;
      ax = a;
      klo = u[a];
      khi = u[D + a];
    }
  }
  float* bx = box + se.node * 2 * P;
#pragma unroll
  for (int a = 0; a < P; ++a) {
    bx[a] = a < D ? lo[a] : 0.0f;
    bx[P + a] = a < D ? hi[a] : 0.0f;
  }
  axis_out[se.node] = ax;
  uint32_t xr = klo ^ khi;
  SegState ss;
  ss.hb = xr ? 31 - __clz(xr) : -1;
  ss.prefix = ss.hb >= 0 ? (klo & ~((2u << ss.hb) - 1u)) : klo;
  ss.rank = (int32_t)(se.m - se.b) - 1;
  ss.axis = ax;
  ss.n_eq_left = 0;
  ss.pad[0] = ss.pad[1] = ss.pad[2] = 0;
  st[s] = ss;
  if (se.child >= 0) {
    uint32_t* c = ubox + se.child * 2 * D;
    for (int a = 0; a < 2 * D; ++a) {
      c[a] = 0xFFFFFFFFu;             // left child lo
      c[2 * D + a] = 0xFFFFFFFFu;     // right child lo
    }
    for (int a = 0; a < D; ++a) {
      c[D + a] = 0u;                  // left child hi
      c[3 * D + a] = 0u;              // right child hi
    }
  }
}

// One radix-select pass over 11-bit digits (three passes resolve a 32-bit
// key).  Lanes of a wave that fall in the same bin as the wave's first lane
// add their count with one LDS atomic (clustered data puts most keys of a
// node in few bins).  The last workgroup of each segment scans the merged
// histogram and narrows the pivot.
constexpr int kDigitBits = 11;
constexpr int kBins = 1 << kDigitBits;
constexpr int kRadixPasses = (32 + kDigitBits - 1) / kDigitBits;

template <int D>
__global__ __launch_bounds__(kBuildBlock) void k_radix_pass(const ChunkEntry* __restrict__ chunks,
                                                            const SegEntry* __restrict__ segs,
                                                            SegState* __restrict__ st,
                                                            uint32_t* __restrict__ hist,
                                                            uint32_t* __restrict__ ctr,
                                                            const float* __restrict__ x, int64_t tot) {
  __shared__ uint32_t h[kBins];
  __shared__ uint32_t tmp[4];
  __shared__ int is_last;
  const ChunkEntry ch = chunks[blockIdx.x];
  const SegState s = st[ch.seg];
  if (s.hb < 0) return;
  const int tid = threadIdx.x, lane = lane_id();
  for (int b = tid; b < kBins; b += kBuildBlock) h[b] = 0;
  __syncthreads();
  const int sh = s.hb >= kDigitBits - 1 ? s.hb - (kDigitBits - 1) : 0;
  const uint32_t dmask = (1u << (s.hb - sh + 1)) - 1u;
  const uint64_t want = (uint64_t)s.prefix >> (s.hb + 1);
  const float* kx = x + (int64_t)s.axis * tot;
  for (int64_t base = ch.b; base < ch.e; base += kBuildBlock) {
    const int64_t i = base + tid;
    bool ok = false;
    uint32_t bin = 0;
    if (i < ch.e) {
      const uint32_t k = fkey(kx[i]);
      ok = ((uint64_t)k >> (s.hb + 1)) == want;
      bin = (k >> sh) & dmask;
    }
    const uint64_t m_ok = __ballot(ok);
    if (m_ok == 0) continue;
    const uint32_t lead = (uint32_t)__builtin_amdgcn_readlane((int)bin, __ffsll((unsigned long long)m_ok) - 1);
    const bool same = ok && bin == lead;
    const uint64_t m = __ballot(same);
    if (same) {
      if (lanes_below(m) == 0) atomicAdd(&h[lead], (uint32_t)__popcll(m));
    } else if (ok) {
      atomicAdd(&h[bin], 1u);
    }
  }
  __syncthreads();
  uint32_t* gh = hist + (int64_t)ch.seg * kBins;
  for (int b = tid; b < kBins; b += kBuildBlock)
    if (h[b]) atomicAdd(gh + b, h[b]);
  __threadfence();
  __syncthreads();
  if (tid == 0) is_last = atomicAdd(ctr + ch.seg, 1u) == (uint32_t)(segs[ch.seg].n_chunks - 1);
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  constexpr int per = kBins / kBuildBlock;
  uint32_t c[per];
  uint32_t sum = 0;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    c[q] = ld_acquire_u32(gh + tid * per + q);
    sum += c[q];
  }
  const uint32_t inc = block_incl_scan(sum, tmp);
  const uint32_t exc = inc - sum;
  const uint32_t r = (uint32_t)s.rank;
  if (exc <= r && r < inc) {
    uint32_t rr = r - exc;
    int b = 0;
#pragma unroll
    for (int q = 0; q < per; ++q) {
      if (b == q && rr >= c[q]) {
        rr -= c[q];
        b = q + 1;
      }
    }
    SegState ns = s;
    ns.prefix = s.prefix | ((uint32_t)(tid * per + b) << sh);
    ns.rank = (int32_t)rr;
    ns.hb = sh - 1;
    st[ch.seg] = ns;
  }
#pragma unroll
  for (int q = 0; q < per; ++q) gh[tid * per + q] = 0;
  if (tid == 0) ctr[ch.seg] = 0;
}

// Counts keys below / equal to the pivot per chunk; the last workgroup of the
// segment turns the counts into exclusive prefixes.
template <int D>
__global__ __launch_bounds__(kBuildBlock) void k_count(const ChunkEntry* __restrict__ chunks,
                                                       const SegEntry* __restrict__ segs,
                                                       const SegState* __restrict__ st,
                                                       const float* __restrict__ x, int64_t tot,
                                                       int32_t* __restrict__ cnt,
                                                       int32_t* __restrict__ pref,
                                                       uint32_t* __restrict__ ctr,
                                                       float* __restrict__ split_out) {
  __shared__ uint32_t tmp[4];
  __shared__ uint32_t red[2][4];
  __shared__ int is_last;
  const int tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
  const ChunkEntry ch = chunks[blockIdx.x];
  const SegState s = st[ch.seg];
  const uint32_t pivot = s.prefix;
  const float* kx = x + (int64_t)s.axis * tot;
  uint32_t nl = 0, ne = 0;
  for (int64_t i = ch.b + tid; i < ch.e; i += kBuildBlock) {
    uint32_t k = fkey(kx[i]);
    nl += k < pivot;
    ne += k == pivot;
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
  }
  __threadfence();
  __syncthreads();
  const SegEntry se = segs[ch.seg];
  if (tid == 0) is_last = atomicAdd(ctr + ch.seg, 1u) == (uint32_t)(se.n_chunks - 1);
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  uint32_t run_l = 0, run_e = 0;
  for (int base = 0; base < se.n_chunks; base += kBuildBlock) {
    int c = base + tid;
    uint32_t vl = 0, ve = 0;
    if (c < se.n_chunks) {
      vl = (uint32_t)ld_agent_i32(cnt + 2 * (se.first_chunk + c));
      ve = (uint32_t)ld_agent_i32(cnt + 2 * (se.first_chunk + c) + 1);
    }
    uint32_t il = block_incl_scan(vl, tmp);
    uint32_t ie = block_incl_scan(ve, tmp);
    if (c < se.n_chunks) {
      pref[2 * (se.first_chunk + c)] = (int32_t)(run_l + il - vl);
      pref[2 * (se.first_chunk + c) + 1] = (int32_t)(run_e + ie - ve);
    }
    __shared__ uint32_t last_l, last_e;
    if (tid == kBuildBlock - 1) {
      last_l = il;
      last_e = ie;
    }
    __syncthreads();
    run_l += last_l;
    run_e += last_e;
    __syncthreads();
  }
  if (tid == 0) {
    split_out[se.node] = fkey_inv(pivot);
    ctr[ch.seg] = 0;
  }
}

// Stable partition of each segment around its pivot into the other buffer,
// accumulating the children's tight boxes.  Each wave owns a contiguous
// quarter of the chunk: it first counts its keys below / equal to the pivot,
// one barrier publishes the per-wave counts, then every wave scatters its rows
// in order with wave ballots only.
template <int D>
__global__ __launch_bounds__(kBuildBlock) void k_scatter(const ChunkEntry* __restrict__ chunks,
                                                         const SegEntry* __restrict__ segs,
                                                         const SegState* __restrict__ st,
                                                         const int32_t* __restrict__ pref,
                                                         const float* __restrict__ xin,
                                                         const int32_t* __restrict__ pin,
                                                         float* __restrict__ xout,
                                                         int32_t* __restrict__ pout, int64_t tot,
                                                         uint32_t* __restrict__ ubox,
                                                         int32_t* __restrict__ bad) {
  __shared__ uint32_t wcnt[2][4];
  const int tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
  const ChunkEntry ch = chunks[blockIdx.x];
  const SegEntry se = segs[ch.seg];
  const SegState s = st[ch.seg];
  const uint32_t pivot = s.prefix;
  const int64_t n_eq_left = (int64_t)s.rank + 1;
  const float* kx = xin + (int64_t)s.axis * tot;
  const int64_t len = ch.e - ch.b;
  const int64_t wb = ch.b + len * wave / 4, we = ch.b + len * (wave + 1) / 4;
  uint32_t nl = 0, ne = 0;
  for (int64_t i = wb + lane; i < we; i += kWave) {
    const uint32_t k = fkey(kx[i]);
    nl += k < pivot;
    ne += k == pivot;
  }
  nl = wave_sum(nl);
  ne = wave_sum(ne);
  if (lane == 0) {
    wcnt[0][wave] = nl;
    wcnt[1][wave] = ne;
  }
  __syncthreads();
  int64_t less_before = pref[2 * blockIdx.x], eq_before = pref[2 * blockIdx.x + 1];
  for (int w = 0; w < wave; ++w) {
    less_before += wcnt[0][w];
    eq_before += wcnt[1][w];
  }
  const int64_t left_before = less_before + min(eq_before, n_eq_left);
  const int64_t right_before = (wb - se.b) - left_before;
  uint32_t lmin[D], lmax[D], rmin[D], rmax[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    lmin[a] = rmin[a] = 0xFFFFFFFFu;
    lmax[a] = rmax[a] = 0u;
  }
  int64_t run_left = 0, run_right = 0, run_eq = 0;
  for (int64_t base = wb; base < we; base += kWave) {
    const int64_t i = base + lane;
    const bool valid = i < we;
    const uint32_t k = valid ? fkey(kx[i]) : 0xFFFFFFFFu;
    const bool less = valid && k < pivot;
    const bool eq = valid && k == pivot;
    const uint64_t be = __ballot(eq);
    const int64_t eq_rank = eq_before + run_eq + lanes_below(be);
    const bool left = less || (eq && eq_rank < n_eq_left);
    const uint64_t bl = __ballot(left);
    const int lpos = lanes_below(bl);
    if (valid) {
      int64_t dst = left ? se.b + left_before + run_left + lpos
                         : se.m + right_before + run_right + (lane - lpos);
      if (dst < se.b || dst >= se.e) {  // cannot happen; keeps a logic slip in bounds
        atomicOr(bad, 2);
        dst = se.b;
      }
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const float v = xin[a * tot + i];
        xout[a * tot + dst] = v;
        const uint32_t kv = fkey(v);
        if (left) {
          lmin[a] = min(lmin[a], kv);
          lmax[a] = max(lmax[a], kv);
        } else {
          rmin[a] = min(rmin[a], kv);
          rmax[a] = max(rmax[a], kv);
        }
      }
      pout[dst] = pin[i];
    }
    const int64_t nvalid = min((int64_t)kWave, we - base);
    run_eq += __popcll(be);
    run_left += __popcll(bl);
    run_right += nvalid - __popcll(bl);
  }
  if (se.child >= 0) {
    uint32_t* c = ubox + se.child * 2 * D;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const uint32_t v0 = wave_umin(lmin[a]), v1 = wave_umax(lmax[a]);
      const uint32_t v2 = wave_umin(rmin[a]), v3 = wave_umax(rmax[a]);
      if (lane == 0) {
        if (v0 != 0xFFFFFFFFu) atomicMin(c + a, v0);
        if (v1 != 0u) atomicMax(c + D + a, v1);
        if (v2 != 0xFFFFFFFFu) atomicMin(c + 2 * D + a, v2);
        if (v3 != 0u) atomicMax(c + 3 * D + a, v3);
      }
    }
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
  int32_t* lperm = reinterpret_cast<int32_t*>(lx + (size_t)D * cap);
  uint32_t* hist = reinterpret_cast<uint32_t*>(lperm + cap);
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
    lperm[i] = pin[g0 + i];
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
          for (int i = lb + lane; i < le; i += kWave) {
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
    r[D] = __int_as_float(lperm[s]);
    float4* dst = reinterpret_cast<float4*>(rec + row * S);
#pragma unroll
    for (int q = 0; q < S / 4; ++q) dst[q] = make_float4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
    perm_out[row] = lperm[s];
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
  const int ns = (int)p.sets.size();
  if (phase == 0) {
    k_init_roots<D><<<(ns + 127) / 128, 128, 0, stream>>>(pd.sets, ns, w.ubox);
    k_ingest<D><<<(unsigned)p.root_chunks.size(), kBuildBlock, 0, stream>>>(
        pd.root_chunks, pd.sets, d_pts, w.x[0], w.p[0], tot, w.ubox, w.bad);
    KDT_HIP(hipGetLastError());
    return KDT_OK;
  }
  for (int l = 0; l < p.n_glevels; ++l) {
    const int nseg = (int)p.segs[l].size();
    const unsigned nch = (unsigned)p.chunks[l].size();
    const int src = l & 1, dst = src ^ 1;
    k_level_init<D><<<(nseg + 127) / 128, 128, 0, stream>>>(pd.segs[l], nseg, w.st, w.ubox, o.box,
                                                            o.axis);
    for (int pass = 0; pass < kRadixPasses; ++pass)
      k_radix_pass<D><<<nch, kBuildBlock, 0, stream>>>(pd.chunks[l], pd.segs[l], w.st, w.hist,
                                                       w.ctr, w.x[src], tot);
    k_count<D><<<nch, kBuildBlock, 0, stream>>>(pd.chunks[l], pd.segs[l], w.st, w.x[src], tot,
                                                w.cnt, w.pref, w.ctr, o.split);
    k_scatter<D><<<nch, kBuildBlock, 0, stream>>>(pd.chunks[l], pd.segs[l], w.st, w.pref,
                                                  w.x[src], w.p[src], w.x[dst], w.p[dst], tot,
                                                  w.ubox, w.bad);
  }
  const size_t smem = lds_bytes(D, p.lds_cap);
  k_lds_subtree<D><<<(unsigned)p.subs.size(), kBuildBlock, smem, stream>>>(
      pd.subs, pd.sets, w.x[0], w.p[0], w.x[1], w.p[1], tot, p.lds_cap, o.box, o.axis, o.split,
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
  bool ok = A((void**)&w.x[0], sizeof(float) * d * tot) && A((void**)&w.x[1], sizeof(float) * d * tot) &&
            A((void**)&w.p[0], sizeof(int32_t) * tot) && A((void**)&w.p[1], sizeof(int32_t) * tot) &&
            A((void**)&w.ubox, sizeof(uint32_t) * 2 * d * p.n_nodes) &&
            A((void**)&w.st, sizeof(SegState) * pd.max_segs) &&
            A((void**)&w.hist, sizeof(uint32_t) * kBins * pd.max_segs) &&
            A((void**)&w.ctr, sizeof(uint32_t) * pd.max_segs) &&
            A((void**)&w.cnt, sizeof(int32_t) * 2 * pd.max_chunks) &&
            A((void**)&w.pref, sizeof(int32_t) * 2 * pd.max_chunks) && A((void**)&w.bad, 256);
  if (!ok) {
    build_scratch_free(w, stream);
    kdt_set_error("device allocation failed for the build scratch (%lld points)", (long long)tot);
    return KDT_ENOMEM;
  }
  return KDT_OK;
}

void build_scratch_free(BuildScratch& w, hipStream_t stream) {
  void* ptrs[] = {w.x[0], w.x[1], w.p[0], w.p[1], w.ubox, w.st, w.hist, w.ctr, w.cnt, w.pref, w.bad};
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
  if (phase == 0) {
    zero_u32(w.hist, kBins * (int64_t)pd.max_segs, stream);
    zero_u32(w.ctr, (int64_t)pd.max_segs, stream);
    zero_u32(reinterpret_cast<uint32_t*>(w.bad), 1, stream);
  }
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
