// kdt_bigk.hip -- k nearest neighbours for k above the 64 entries a register
// list holds (Sec. 3.3 measures k up to 10^4) on gfx950.  Exact, in three
// steps:
//   1. a squared radius per query whose closed ball holds at least k points:
//      the 64th neighbour's d2 (the register path) scaled by (k/64)^(2/d),
//      grown from the density a count shows where it falls short;
//   2. the (d2, index) keys of every point in that ball, one wave per query;
//   3. a segmented sort of the keys: the first k of each row are the answer,
//      since every point outside the ball is farther than the k-th key.
// Keys are (d2 bits << b | index), b the bits of the largest index, with the
// same float32 distances as the register path, so results are identical to
// it wherever both apply; the radix sort passes over 32 + b bits only.  The
// kernels take the metric as a parameter: open space, or the D-torus of
// periodic boundaries (the node bound and the point distance change).
// Queries are processed in chunks whose keys fit a bounded buffer.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <vector>

#include "kdt_bitonic.h"
#include "kdt_packet.h"
#include "kdt_torus.h"

namespace kdt {

constexpr int kLBlock = 128;
// Keys per chunk (8 GiB): each chunk's fill and sort launches wait for their
// widest rows, so fewer, larger chunks keep more rows in flight (at k = 10^4
// the balls average about 28 000 keys: 4800 rows per chunk of 2^27 keys)
constexpr int64_t kBigKeysPerChunk = int64_t(1) << 30;
constexpr int kBigGrowRounds = 24;  // then the radius becomes infinite
// Largest k sorted in LDS (16384 keys, 136 KiB with the padding slots, per workgroup; gfx950 gives a
// workgroup up to 160 KiB); larger k takes the segmented radix sort.
constexpr int kTopkMax = 16384;
// Margin on estimated squared radii (x 1.1^(d/2) expected points), the least
// growth of a radius that fell short, and the cap of that least growth for
// stuck rows.
constexpr float kBigMargin = 1.1f;
constexpr float kBigGrowMin = 1.1f;
constexpr float kBigGrowCap = 64.0f;
// A ball holding more than kBigShrinkAt k points and more than the 16384
// keys a row sort holds in LDS (a query in a void whose scaled radius
// reached a halo) shrinks, at most kBigShrinks times, towards kBigShrinkTo k
// points.
constexpr int kBigShrinkAt = 2;
constexpr float kBigShrinkTo = 1.3f;
constexpr int kBigShrinks = 1;  // a second shrink cost more than it saved (k = 10^4: 239 -> 254 ms)
constexpr int kShrinkShift = 29;  // stuck[]: shrinks done above this bit, stuck rounds below
constexpr int kBigShrinkMinK = 2048;

// Queries in a spatially coherent order, pos -> row: the tree's own points
// in tree order (self queries; rowof NULL: the rows stay in tree order) or
// the given queries gathered through `order`.
template <int D>
__global__ void k_gather_self(const float* __restrict__ rec, int64_t n, float* __restrict__ qs,
                              int32_t* __restrict__ rowof) {
  constexpr int S = rec_stride(D);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int a = 0; a < D; ++a) qs[i * D + a] = rec[i * S + a];
  if (rowof) rowof[i] = __float_as_int(rec[i * S + D]);
}

template <int D>
__global__ void k_gather_queries(const float* __restrict__ q, const int32_t* __restrict__ order,
                                 int64_t nq, float* __restrict__ qs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const int64_t r = order[i];
#pragma unroll
  for (int a = 0; a < D; ++a) qs[i * D + a] = q[r * D + a];
}

// r2 <- 64th neighbour's d2 x scale (+inf when the tree holds at most k
// points); also clears the growth state and the first offset.
__global__ void k_start_radius(float* __restrict__ r2, int64_t nq, float scale, int all,
                               int32_t* __restrict__ prev, int32_t* __restrict__ stuck,
                               int32_t* __restrict__ again, int rounds,
                               int64_t* __restrict__ off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nq) {
    r2[i] = all ? INFINITY : r2[i] * scale;
    prev[i] = 0;
    stuck[i] = 0;
  }
  if (i < rounds) again[i] = 0;
  if (i == 0) off[0] = 0;
}

// Per query, one lane each: the number of points of the closed ball of
// squared radius r2[s] around it.  A node inside the ball counts whole, a
// leaf that straddles it tests its points.  With `only_marked`, rows whose
// count is not negative (not grown since they were counted) are skipped.
template <int D, class M>
__global__ __launch_bounds__(kLBlock) void k_ball_count(TreeView t, const float* __restrict__ q,
                                                        int64_t nq, const float* __restrict__ r2v,
                                                        int32_t* __restrict__ count,
                                                        int only_marked, M metric) {
  extern __shared__ uint32_t var_stk[];
  uint32_t* col = var_stk + threadIdx.x;
  const int64_t s = (int64_t)blockIdx.x * kLBlock + threadIdx.x;
  if (s >= nq || (only_marked && count[s] >= 0)) return;
  float p[D];
#pragma unroll
  for (int a = 0; a < D; ++a) p[a] = q[s * D + a];
  const float r2 = r2v[s];
  const uint32_t first_leaf = (1u << t.levels) - 1u;
  int64_t c = 0;
  int sp = 0;
  col[kLBlock * sp++] = 0;
  while (sp > 0) {
    const uint32_t node = col[kLBlock * --sp];
    float lo[D], hi[D];
    load_box<D>(t.box, node, lo, hi);
    if (metric.mindist(lo, hi, p) > r2) continue;
    const int lev = node_level(node);
    const int64_t j = (int64_t)node - ((int64_t(1) << lev) - 1);
    const int64_t b = node_begin(t.n, lev, j), e = node_begin(t.n, lev, j + 1);
    if (metric.maxdist(lo, hi, p) <= r2) {
      c += e - b;
      continue;
    }
    if (node >= first_leaf) {
      for (int64_t i = b; i < e; ++i) {
        float x[D];
        int32_t id = 0;
        load_rec<D>(t.rec, i, x, id);
        c += metric.dist(x, p) <= r2;
      }
      continue;
    }
    col[kLBlock * sp++] = 2 * node + 2;
    col[kLBlock * sp++] = 2 * node + 1;
  }
  count[s] = (int32_t)c;
}

// Per query, one wave each: the keys of the points k_ball_count counted,
// written from offsets[s] - base on.  The wave walks the tree together and
// scans a node's points 64 at a time with coalesced loads; lanes holding a
// point append its key at their rank in the wave's ballot.  The node tests
// are those of k_ball_count, so exactly count[s] keys are written.
constexpr int kFillWaves = 4;
template <int D, class M>
__global__ __launch_bounds__(64 * kFillWaves) void k_ball_fill(
    TreeView t, const float* __restrict__ q, int64_t s0, int64_t s1,
    const float* __restrict__ r2v, const int64_t* __restrict__ offsets, int64_t base,
    uint64_t* __restrict__ keys, int stack_len, int ib, M metric) {
  extern __shared__ uint32_t fill_stk[];
  const int lane = threadIdx.x & 63;
  uint32_t* stk = fill_stk + (threadIdx.x >> 6) * stack_len;
  const int64_t s = s0 + (int64_t)blockIdx.x * kFillWaves + (threadIdx.x >> 6);
  if (s >= s1) return;  // uniform over the wave
  float p[D];
#pragma unroll
  for (int a = 0; a < D; ++a) p[a] = q[s * D + a];
  const float r2 = r2v[s];
  const uint32_t first_leaf = (1u << t.levels) - 1u;
  const uint64_t below = (1ull << lane) - 1ull;
  int64_t pos = offsets[s] - base;
  // every lane writes the same entries, so each reads back its own writes
  int sp = 0;
  stk[sp++] = 0;
  while (sp > 0) {
    const uint32_t node = stk[--sp];
    float lo[D], hi[D];
    load_box<D>(t.box, node, lo, hi);
    if (metric.mindist(lo, hi, p) > r2) continue;
    const int lev = node_level(node);
    const int64_t j = (int64_t)node - ((int64_t(1) << lev) - 1);
    const int64_t b = node_begin(t.n, lev, j), e = node_begin(t.n, lev, j + 1);
    const bool whole = metric.maxdist(lo, hi, p) <= r2;
    if (whole || node >= first_leaf) {
      for (int64_t c = b; c < e; c += 64) {
        const int64_t i = c + lane;
        bool in = false;
        uint64_t key = 0;
        if (i < e) {
          float x[D];
          int32_t id = 0;
          load_rec<D>(t.rec, i, x, id);
          const float d2 = metric.dist(x, p);
          in = whole || d2 <= r2;
          key = ((uint64_t)__float_as_uint(d2) << ib) | (uint32_t)id;
        }
        const uint64_t m = __ballot(in);
        if (in) keys[pos + __popcll(m & below)] = key;
        pos += __popcll(m);
      }
      continue;
    }
    stk[sp++] = 2 * node + 2;
    stk[sp++] = 2 * node + 1;
  }
}

// Rows whose ball holds fewer than k points get a larger radius, from the
// density the count shows: r2 x kBigMargin (k / count)^(2/d), at least
// x kBigGrowMin (a zero radius restarts from `floor`); the row is marked for
// recounting (its index appended to `list`, their number in again[0]).  A
// row whose count grew by less than an eighth since its last
// round is stuck (its ball is crossing empty space, e.g. around a small
// isolated clump): each time, its least growth is multiplied by four, up to
// kBigGrowCap.  In the last round the radius becomes infinite.  A row whose
// ball holds more than kBigShrinkAt k points and more than `lds_keys` (the
// row sort's LDS capacity) shrinks, up to kBigShrinks times (not in the last
// two rounds), by
// (kBigShrinkTo k / count)^(2/d): its keys are written and selected
// afterwards, so an oversized ball costs in proportion, and a row beyond
// the LDS sort needs the radix select; should the smaller ball hold fewer
// than k points, it grows again as above.  Only for k of at least
// kBigShrinkMinK: below, few rows pass the LDS capacity and the recount
// round costs more than it saves (10^5 queries at k = 1000: 44 -> 50 ms,
// while k = 10^4 drops from 295 to 240 ms).
__global__ void k_grow_radius(float* __restrict__ r2, int32_t* __restrict__ count,
                              int32_t* __restrict__ prev, int32_t* __restrict__ stuck, int64_t nq,
                              int k, float two_over_d, float floor, int last, int lds_keys,
                              int32_t* __restrict__ again, int32_t* __restrict__ list) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq || isinf(r2[i])) return;
  if (count[i] >= k) {
    const int c = count[i];
    if (last || k < kBigShrinkMinK || c / kBigShrinkAt <= k || c <= lds_keys ||
        (stuck[i] >> kShrinkShift) >= kBigShrinks || !(r2[i] > 0.0f))
      return;
    stuck[i] += 1 << kShrinkShift;
    prev[i] = 0;
    r2[i] *= powf(kBigShrinkTo * (float)k / (float)c, two_over_d);
    count[i] = -1;
    list[atomicAdd(again, 1)] = (int32_t)i;
    return;
  }
  const int c = count[i], p = prev[i];
  const int32_t shrinks = stuck[i] & ~((1 << kShrinkShift) - 1);
  const int l = (stuck[i] & ((1 << kShrinkShift) - 1)) + (p > 0 && c - p < (p >> 3) ? 1 : 0);
  stuck[i] = shrinks | l;
  prev[i] = c;
  const float least = fminf(kBigGrowCap, kBigGrowMin * exp2f(2.0f * (float)l));
  const float f = c > 0 ? fmaxf(least, kBigMargin * powf((float)k / (float)c, two_over_d)) : least;
  r2[i] = last ? INFINITY : (r2[i] > 0.0f ? r2[i] * f : floor);
  count[i] = -1;
  list[atomicAdd(again, 1)] = (int32_t)i;
}

__global__ void k_chunk_offsets(const int64_t* __restrict__ off, int64_t s0, int64_t m,
                                int32_t* __restrict__ rel, uint32_t* __restrict__ ctr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= m) rel[i] = (int32_t)(off[s0 + i] - off[s0]);
  if (i < 3) ctr[i] = 0u;
}

// The LDS sort a row of `have` keys takes: the smallest of the 1024, 4096
// and 16384-key workgroup sorts holding max(k, min(have, 16384)) keys (rows
// wider than 16384 select their k smallest first).  Classes 0, 1, 2; the
// host and the device classify alike.
__host__ __device__ __forceinline__ int topk_class(int64_t have, int k) {
  const int64_t want = have < 16384 ? (have > k ? have : k) : (k > 16384 ? k : 16384);
  return want <= 1024 ? 0 : want <= 4096 ? 1 : 2;
}

// Chunk rows listed by class: row i of class c goes to
// rows[base[c] + slot], slots taken in any order (each row is sorted on its
// own, so the order of a class list does not change any result), one atomic
// per wave and class.  ctr holds three zeroed counters.
__global__ void k_topk_classes(const int32_t* __restrict__ rel, int64_t m, int k, int64_t base1,
                               int64_t base2, uint32_t* __restrict__ ctr,
                               int32_t* __restrict__ rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int c = i < m ? topk_class(rel[i + 1] - rel[i], k) : -1;
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    const uint64_t mk = __ballot(c == cc);
    if (!mk) continue;
    const int lead = __ffsll((unsigned long long)mk) - 1;
    uint32_t at = 0u;
    if (lane == lead) at = atomicAdd(ctr + cc, (uint32_t)__popcll(mk));
    at = __shfl(at, lead);
    const int64_t base = cc == 0 ? 0 : cc == 1 ? base1 : base2;
    if (c == cc) rows[base + at + __popcll(mk & ((1ull << lane) - 1ull))] = (int32_t)i;
  }
}

// The first k sorted keys of each query of the chunk: (index, d2) pairs, or
// the k-th d2 / distance.  Rows with fewer than k keys are padded (-1, +inf).
__global__ void k_take_first(const uint64_t* __restrict__ keys, const int32_t* __restrict__ rel,
                             const int32_t* __restrict__ rowof, int64_t s0, int64_t m, int k,
                             int mode, int ib, int32_t* __restrict__ oidx,
                             float* __restrict__ od2) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = mode == 0 ? k : 1;
  if (t >= m * per) return;
  const int64_t i = t / per;
  const int j = mode == 0 ? (int)(t % per) : k - 1;
  const int have = rel[i + 1] - rel[i];
  const int64_t row = rowof ? (int64_t)rowof[s0 + i] : s0 + i;
  const bool empty = j >= have;
  const uint64_t key = empty ? 0ull : keys[rel[i] + j];
  const float d2 = empty ? INFINITY : __uint_as_float((uint32_t)(key >> ib));
  if (mode == 0) {
    if (oidx) oidx[row * k + j] = empty ? -1 : (int32_t)(key & ((1ull << ib) - 1ull));
    od2[row * k + j] = d2;
  } else {
    od2[row] = mode == 2 ? sqrtf(d2) : d2;
  }
}

// One wave picks the digit of a radix-select pass: given the 256-bin
// histogram of the keys that match the digits chosen so far and the rank
// (from 1) of the wanted key among them, the bin that holds it and the
// number of matching keys in lower bins.  Each lane sums four bins, a
// prefix sum over the lanes finds the first lane that reaches the rank, and
// that lane's bins are walked.  Every lane of the wave gets the result.
__device__ __forceinline__ void wave_pick_digit(const uint32_t* hist, int lane, uint32_t rank,
                                                uint32_t& bin, uint32_t& below) {
  const uint32_t c0 = hist[4 * lane], c1 = hist[4 * lane + 1];
  const uint32_t c2 = hist[4 * lane + 2], c3 = hist[4 * lane + 3];
  const uint32_t mine = c0 + c1 + c2 + c3;
  uint32_t incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t up = __shfl_up(incl, o);
    if (lane >= o) incl += up;
  }
  const int at = __ffsll((unsigned long long)__ballot(incl >= rank)) - 1;
  uint32_t acc = __shfl(incl - mine, at);
  const uint32_t e0 = __shfl(c0, at), e1 = __shfl(c1, at), e2 = __shfl(c2, at);
  uint32_t b = 4u * (uint32_t)at;
  if (acc + e0 < rank) {
    acc += e0;
    ++b;
    if (acc + e1 < rank) {
      acc += e1;
      ++b;
      if (acc + e2 < rank) {
        acc += e2;
        ++b;
      }
    }
  }
  bin = b;
  below = acc;
}

// The k smallest keys of each row of the chunk, sorted and written as
// (index, d2) pairs (mode 0), one workgroup per row: row rows[b] of the
// chunk for workgroup b, or row b when rows is null.  A row of at most kp
// keys (kp: the power of two at or above k, at least 32) goes to LDS whole.
// A longer row first bounds its k smallest by a radix select over the key
// bits, 8 bits per pass from the top, each pass a histogram of the keys that
// match the digits chosen so far; the passes stop once the keys at or below
// the chosen range number at most kp (after the last pass that range is the
// k-th key alone: keys are distinct, they end in the point index).  Rows of
// up to R T keys hold them in registers for this; longer rows read them from
// global memory each pass.  The kept keys go to LDS, and are sorted there by
// a bitonic network over the next power of two, padded with all-ones keys.
// Needs k <= P.
template <int P>
constexpr int topk_threads() {
  return P <= 1024 ? 128 : P <= 4096 ? 256 : 1024;
}

template <int P>
__global__ __launch_bounds__(topk_threads<P>()) void k_row_topk(
    const uint64_t* __restrict__ keys, const int32_t* __restrict__ rel,
    const int32_t* __restrict__ rowof, const int32_t* __restrict__ rows, int64_t s0, int k,
    int ib, int32_t* __restrict__ oidx, float* __restrict__ od2) {
  constexpr int T = topk_threads<P>();
  static_assert(T * 16 >= P, "a thread owns one run of 16 keys of the row");
  __shared__ uint64_t s[P + P / 16];  // key i at s[pad16(i)]
  __shared__ uint32_t hist[256];
  __shared__ uint32_t sh_digit, sh_rank, sh_fill;
  const int tid = threadIdx.x;
  const int64_t i = rows ? (int64_t)rows[blockIdx.x] : (int64_t)blockIdx.x;
  const int64_t row = rowof ? (int64_t)rowof[s0 + i] : s0 + i;
  const int32_t have = rel[i + 1] - rel[i];
  const uint64_t* __restrict__ src = keys + rel[i];
  const int lane = tid & 63;
  const int bits = 32 + ib;
  int kp = 32;  // the sort size k keys need
  while (kp < k) kp <<= 1;
  // keys per thread in registers: the 16384-key sort (1024 threads, one
  // workgroup per CU) holds rows of up to 32768
  constexpr int R = P >= 16384 ? 32 : P / T;
  int n = have;
  uint64_t bound = 0ull;  // the kept keys are those at or below it
  if (have > kp) {
    const bool in_regs = have <= R * T;
    uint64_t v[R];
    if (in_regs) {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int e = tid + j * T;
        v[j] = e < have ? src[e] : ~0ull;  // ~0 is no key: its d2 bits would be a NaN
      }
    }
    uint64_t prefix = 0ull, mask = 0ull;
    uint32_t rank = (uint32_t)k, base = 0u;  // base: keys below the chosen range
    for (int shift = (bits - 1) / 8 * 8; shift >= 0; shift -= 8) {
      for (int j = tid; j < 256; j += T) hist[j] = 0u;
      __syncthreads();
      if (in_regs) {
#pragma unroll
        for (int j = 0; j < R; ++j)
          if (v[j] != ~0ull && (v[j] & mask) == prefix)
            atomicAdd(&hist[(uint32_t)(v[j] >> shift) & 255u], 1u);
      } else {
        for (int32_t e = tid; e < have; e += T) {
          const uint64_t key = src[e];
          if ((key & mask) == prefix) atomicAdd(&hist[(uint32_t)(key >> shift) & 255u], 1u);
        }
      }
      __syncthreads();
      if (tid < 64) {
        uint32_t bin, below;
        wave_pick_digit(hist, tid, rank, bin, below);
        if (tid == 0) {
          sh_digit = bin;
          sh_rank = rank - below;
          sh_fill = below + hist[bin];
        }
      }
      __syncthreads();
      const uint32_t kept = base + sh_fill;  // keys at or below the range's top
      base += rank - sh_rank;
      rank = sh_rank;
      prefix |= (uint64_t)sh_digit << shift;
      mask |= 255ull << shift;
      __syncthreads();  // every thread has read sh_* and hist before they change
      if (kept <= (uint32_t)kp || shift == 0) {  // uniform over the workgroup
        bound = prefix | ((1ull << shift) - 1ull);
        n = (int)kept;
        break;
      }
    }
    if (tid == 0) sh_fill = 0u;
    __syncthreads();
    // the kept keys to s[0, n), one LDS atomic per wave and step
    const auto put = [&](uint64_t key) {
      const bool keep = key != ~0ull && key <= bound;
      const uint64_t m = __ballot(keep);
      if (m) {
        const int lead = __ffsll((unsigned long long)m) - 1;
        uint32_t at = 0u;
        if (lane == lead) at = atomicAdd(&sh_fill, (uint32_t)__popcll(m));
        at = __shfl(at, lead);
        if (keep) s[pad16((int)(at + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))))] = key;
      }
    };
    if (in_regs) {
#pragma unroll
      for (int j = 0; j < R; ++j) put(v[j]);
    } else {
      for (int32_t j = 0; j < (have + T - 1) / T; ++j) {  // the same trip count on every lane
        const int32_t e = tid + j * T;
        put(e < have ? src[e] : ~0ull);
      }
    }
  } else {
    for (int32_t e = tid; e < have; e += T) s[pad16(e)] = src[e];
  }
  int pn = 1;
  while (pn < n) pn <<= 1;
  if (pn >= 32) {
    for (int e = n + tid; e < pn; e += T) s[pad16(e)] = ~0ull;
    bitonic_runs16(s, pn, tid, T);
  } else {
    for (int e = n + tid; e < pn; e += T) s[pad16(e)] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= pn; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int t = tid; t < pn / 2; t += T) {
          const int lo = 2 * t - (t & (stride - 1));
          const int hi = lo + stride;
          const uint64_t a = s[pad16(lo)], c = s[pad16(hi)];
          if ((a > c) == ((lo & size) == 0)) {
            s[pad16(lo)] = c;
            s[pad16(hi)] = a;
          }
        }
        __syncthreads();
      }
    }
  }
  for (int j = tid; j < k; j += T) {
    const bool empty = j >= n;
    const uint64_t key = empty ? 0ull : s[pad16(j)];
    if (oidx) oidx[row * k + j] = empty ? -1 : (int32_t)(key & ((1ull << ib) - 1ull));
    od2[row * k + j] = empty ? INFINITY : __uint_as_float((uint32_t)(key >> ib));
  }
}

// The k-th smallest squared distance of each row of the chunk (modes 1 and
// 2), without sorting: one wave per row selects it digit by digit, 8 bits of
// the distance per pass from highest to lowest, each pass a histogram (in
// LDS) of the row's keys that match the digits chosen so far.  Only the
// value is wanted, so the order of equal distances does not matter.  Rows
// with fewer than k keys give +inf.
__global__ __launch_bounds__(64) void k_row_kth(const uint64_t* __restrict__ keys,
                                               const int32_t* __restrict__ rel,
                                               const int32_t* __restrict__ rowof, int64_t s0,
                                               int k, int mode, int ib,
                                               float* __restrict__ od2) {
  __shared__ uint32_t hist[256];
  const int lane = threadIdx.x;
  const int64_t i = blockIdx.x;
  const int64_t row = rowof ? (int64_t)rowof[s0 + i] : s0 + i;
  const int32_t b = rel[i], have = rel[i + 1] - rel[i];
  if (have < k) {  // uniform over the block
    if (lane == 0) od2[row] = INFINITY;
    return;
  }
  uint32_t prefix = 0, mask = 0, rank = (uint32_t)k;  // rank among keys matching prefix
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int j = lane; j < 256; j += 64) hist[j] = 0u;
    __syncthreads();
    for (int32_t e = lane; e < have; e += 64) {
      const uint32_t v = (uint32_t)(keys[b + e] >> ib);
      if ((v & mask) == prefix) atomicAdd(&hist[(v >> shift) & 255u], 1u);
    }
    __syncthreads();
    uint32_t bin, acc;
    wave_pick_digit(hist, lane, rank, bin, acc);
    rank -= acc;
    prefix |= bin << shift;
    mask |= 255u << shift;
    __syncthreads();  // every lane has read the histogram before it is cleared
  }
  if (lane == 0) {
    const float d2 = __uint_as_float(prefix);
    od2[row] = mode == 2 ? sqrtf(d2) : d2;
  }
}

template <int D, class M>
static kdt_status knn_large_impl(const kdt_tree* tr, const float* d_q, int64_t nq, int k,
                                 int32_t* d_idx, float* d_d2, int mode, bool sort_q,
                                 const int32_t* given, const M& metric, const float* period,
                                 hipStream_t stream) {
  TreeView v;
  v.rec = tr->rec;
  v.box = tr->box;
  v.n = tr->n;
  v.levels = tr->levels;
  PoolBuffers buf(stream);
  const unsigned gq = (unsigned)((nq + 255) / 256);
  // 0. queries in a coherent order (pos), rowof[pos] their output row
  const float* q = d_q;
  const int32_t* rowof = nullptr;
  if (!d_q || given || (sort_q && nq > 1)) {
    float* qs = nullptr;
    int32_t* rows = nullptr;
    if (!buf.get(&qs, (size_t)nq * D) || (!given && !buf.get(&rows, (size_t)nq))) {
      kdt_set_error("kdt_knn: device allocation failed for the large-k query order");
      return KDT_ENOMEM;
    }
    if (!d_q) {
      // `given` set: the tree-order row marker -- row = position
      k_gather_self<D><<<gq, 256, 0, stream>>>(tr->rec, nq, qs, given ? nullptr : rows);
      rowof = given ? nullptr : rows;
    } else {
      if (!given) {
        const kdt_status st = kdt_query_order(tr, d_q, nq, 0, rows, stream);
        if (st != KDT_OK) return st;
      }
      rowof = given ? given : rows;
      k_gather_queries<D><<<gq, 256, 0, stream>>>(d_q, rowof, nq, qs);
    }
    q = qs;
  }
  float* r2 = nullptr;
  int32_t* count = nullptr;
  int64_t* off = nullptr;
  int32_t* again = nullptr;
  int32_t* prev = nullptr;
  int32_t* stuck = nullptr;
  if (!buf.get(&r2, (size_t)nq) || !buf.get(&count, (size_t)nq) || !buf.get(&prev, (size_t)nq) ||
      !buf.get(&stuck, (size_t)nq) ||
      !buf.get(&off, (size_t)nq + 1) || !buf.get(&again, (size_t)kBigGrowRounds)) {
    kdt_set_error("kdt_knn: device allocation failed for the large-k radii");
    return KDT_ENOMEM;
  }
  // 1. start from the 64th neighbour (the register path), scaled to hold k
  kdt_query_opts in_order{};
  in_order.sort_queries = 0;
  in_order.period = period;  // the torus kNN also checks the period
  kdt_status st = kdt_knn(tr, q, nq, KDT_MAX_K, nullptr, r2, 1, &in_order, stream);
  if (st != KDT_OK) return st;
  const float scale = kBigMargin * std::pow((float)k / (float)KDT_MAX_K, 2.0f / (float)D);
  k_start_radius<<<gq, 256, 0, stream>>>(r2, nq, scale, tr->n <= k ? 1 : 0, prev, stuck, again,
                                         kBigGrowRounds, off);
  float root_lo[D], root_hi[D];
  if (hipMemcpyAsync(root_lo, tr->box, sizeof(float) * D, hipMemcpyDeviceToHost, stream) !=
          hipSuccess ||
      hipMemcpyAsync(root_hi, tr->box + pad4(D), sizeof(float) * D, hipMemcpyDeviceToHost,
                     stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    kdt_set_error("kdt_knn: reading the root box failed");
    return KDT_EDEVICE;
  }
  float diag2 = 0.0f;
  for (int a = 0; a < D; ++a) diag2 += (root_hi[a] - root_lo[a]) * (root_hi[a] - root_lo[a]);
  const float floor = diag2 > 0.0f ? std::ldexp(diag2, -24) : 1e-30f;
  const int stack_len = tr->levels + 2;
  const size_t smem = sizeof(uint32_t) * (size_t)stack_len * kLBlock;
  const unsigned gl = (unsigned)((nq + kLBlock - 1) / kLBlock);
  // Counts: the wave-shared count traversal (leaves of at most 64 points)
  // over every query first, then over the list of grown rows; else one
  // traversal per lane, skipping rows that did not grow.
  int32_t* list = nullptr;
  if (!buf.get(&list, (size_t)nq)) {
    kdt_set_error("kdt_knn: device allocation failed for the large-k row list");
    return KDT_ENOMEM;
  }
  int32_t h_again = (int32_t)nq;
  for (int round = 0; round < kBigGrowRounds; ++round) {
    if (tr->leaf <= 64) {
      st = var_ball_count_launch<D>(v, tr->leaf, q, r2, round == 0 ? nq : (int64_t)h_again,
                                    round == 0 ? nullptr : list, metric, count, stream);
      if (st != KDT_OK) return st;
    } else {
      k_ball_count<D><<<gl, kLBlock, smem, stream>>>(v, q, nq, r2, count, round > 0 ? 1 : 0,
                                                     metric);
    }
    k_grow_radius<<<gq, 256, 0, stream>>>(r2, count, prev, stuck, nq, k, 2.0f / (float)D, floor,
                                          round + 2 >= kBigGrowRounds ? 1 : 0, kTopkMax,
                                          again + round, list);
    h_again = 0;
    if (hipMemcpyAsync(&h_again, again + round, sizeof(int32_t), hipMemcpyDeviceToHost,
                       stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
      kdt_set_error("kdt_knn: reading the growth flag failed");
      return KDT_EDEVICE;
    }
    if (!h_again) break;
  }
  // 2. offsets of each query's keys; chunks of at most kBigKeysPerChunk keys
  {
    void* tmp = nullptr;
    if (!buf.get((char**)&tmp, scan_scratch_bytes(nq))) {
      kdt_set_error("kdt_knn: device allocation failed for the large-k offsets");
      return KDT_ENOMEM;
    }
    if (exclusive_scan<int64_t>(count, off, nq, off + nq, tmp, stream) != KDT_OK) {
      kdt_set_error("kdt_knn: large-k offsets failed");
      return KDT_EDEVICE;
    }
  }
  std::vector<int64_t> h_off((size_t)nq + 1);
  if (hipMemcpyAsync(h_off.data(), off, sizeof(int64_t) * (nq + 1), hipMemcpyDeviceToHost,
                     stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    kdt_set_error("kdt_knn: reading the large-k offsets failed");
    return KDT_EDEVICE;
  }
  int64_t max_row = 0;
  for (int64_t i = 0; i < nq; ++i) max_row = std::max(max_row, h_off[i + 1] - h_off[i]);
  const int64_t cap = std::max(kBigKeysPerChunk, max_row);
  if (cap > INT32_MAX) {
    kdt_set_error("kdt_knn: a query's candidate ball holds more than 2^31-1 points");
    return KDT_EUNSUPPORTED;
  }
  uint64_t* keys = nullptr;
  uint64_t* sorted = nullptr;
  int32_t* rel = nullptr;
  uint32_t* cls_ctr = nullptr;
  const int64_t biggest = std::min(cap, h_off[nq]);
  const bool radix_rows = mode == 0 && k > kTopkMax;  // the segmented radix sort's output
  if (!buf.get(&keys, (size_t)std::max<int64_t>(biggest, 1)) ||
      (radix_rows && !buf.get(&sorted, (size_t)std::max<int64_t>(biggest, 1))) ||
      !buf.get(&rel, (size_t)nq + 1) || !buf.get(&cls_ctr, 4)) {
    kdt_set_error("kdt_knn: device allocation failed for the large-k keys");
    return KDT_ENOMEM;
  }
  // 3. per chunk: keys, then a segmented sort and the first k (or, for the
  // k-th distance alone, a selection).  A key is (d2 bits << ib | index) with
  // ib = the bits of the largest index, so the radix sort passes over
  // 32 + ib bits only.
  int ib = 1;
  while (ib < 31 && (int64_t(1) << ib) < tr->n) ++ib;
  // the fill reads the tree at its nodes of at most 64 points: a wave scans
  // such a node in one step, and a ball of 10^4 points takes a quarter of
  // the steps of 16-point leaves (whole-node and per-point tests decide the
  // same points at any level, so the keys are the ones counted)
  int fill_cap = 0;
  const TreeView vfill = coarse_view(v, tr->leaf, 64, &fill_cap);
  void* stmp = nullptr;
  size_t stmp_bytes = 0;
  for (int64_t s0 = 0; s0 < nq;) {
    int64_t s1 = s0 + 1;
    while (s1 < nq && h_off[s1 + 1] - h_off[s0] <= cap) ++s1;
    const int64_t m = s1 - s0, total = h_off[s1] - h_off[s0];
    k_chunk_offsets<<<(unsigned)((m + 256) / 256), 256, 0, stream>>>(off, s0, m, rel, cls_ctr);
    if (total > 0) {
      k_ball_fill<D><<<(unsigned)((m + kFillWaves - 1) / kFillWaves), 64 * kFillWaves,
                       sizeof(uint32_t) * (size_t)stack_len * kFillWaves, stream>>>(
          vfill, q, s0, s1, r2, off, h_off[s0], keys, stack_len, ib, metric);
    }
    if (mode != 0) {  // only the k-th distance: selected, not sorted
      k_row_kth<<<(unsigned)m, 64, 0, stream>>>(keys, rel, rowof, s0, k, mode, ib, d_d2);
      s0 = s1;
      continue;
    }
    if (k <= kTopkMax) {  // rows sorted in LDS, the k smallest written directly
      // Each row takes the smallest workgroup sort that holds it: a few wide
      // rows no longer move every row of the chunk to the 1024-thread sort,
      // whose 128 KiB of LDS leave one workgroup per CU.
      int64_t cnt[3] = {0, 0, 0};
      for (int64_t r = s0; r < s1; ++r) ++cnt[topk_class(h_off[r + 1] - h_off[r], k)];
      const int used = (cnt[0] > 0) + (cnt[1] > 0) + (cnt[2] > 0);
      int32_t* cls_rows = list;  // the grown-row list is no longer needed
      if (used > 1)
        k_topk_classes<<<(unsigned)((m + 255) / 256), 256, 0, stream>>>(
            rel, m, k, cnt[0], cnt[0] + cnt[1], cls_ctr, cls_rows);
      const int32_t* r0 = used > 1 ? cls_rows : nullptr;
      const int32_t* r1 = used > 1 ? cls_rows + cnt[0] : nullptr;
      const int32_t* r2l = used > 1 ? cls_rows + cnt[0] + cnt[1] : nullptr;
      if (cnt[0] > 0)
        k_row_topk<1024><<<(unsigned)cnt[0], topk_threads<1024>(), 0, stream>>>(
            keys, rel, rowof, r0, s0, k, ib, d_idx, d_d2);
      if (cnt[1] > 0)
        k_row_topk<4096><<<(unsigned)cnt[1], topk_threads<4096>(), 0, stream>>>(
            keys, rel, rowof, r1, s0, k, ib, d_idx, d_d2);
      if (cnt[2] > 0)
        k_row_topk<kTopkMax><<<(unsigned)cnt[2], topk_threads<kTopkMax>(), 0, stream>>>(
            keys, rel, rowof, r2l, s0, k, ib, d_idx, d_d2);
      s0 = s1;
      continue;
    }
    if (total > 0) {
      size_t sb = 0;
      if (hipcub::DeviceSegmentedRadixSort::SortKeys(nullptr, sb, keys, sorted, (int)total, (int)m,
                                                     rel, rel + 1, 0, 32 + ib, stream) !=
          hipSuccess) {
        kdt_set_error("kdt_knn: large-k sort setup failed");
        return KDT_EDEVICE;
      }
      if (sb > stmp_bytes) {
        if (!buf.get((char**)&stmp, sb)) {
          kdt_set_error("kdt_knn: device allocation failed for the large-k sort");
          return KDT_ENOMEM;
        }
        stmp_bytes = sb;
      }
      if (hipcub::DeviceSegmentedRadixSort::SortKeys(stmp, sb, keys, sorted, (int)total, (int)m,
                                                     rel, rel + 1, 0, 32 + ib, stream) !=
          hipSuccess) {
        kdt_set_error("kdt_knn: large-k sort failed");
        return KDT_EDEVICE;
      }
    }
    const int64_t outs = m * (mode == 0 ? k : 1);
    k_take_first<<<(unsigned)((outs + 255) / 256), 256, 0, stream>>>(sorted, rel, rowof, s0, m,
                                                                   k, mode, ib, d_idx, d_d2);
    s0 = s1;
  }
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_knn: a large-k kernel launch failed");
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

template <int D>
static kdt_status knn_large_metric(const kdt_tree* tr, const float* d_q, int64_t nq, int k,
                                   int32_t* d_idx, float* d_d2, int mode, bool sort_q,
                                   const int32_t* given, const float* period,
                                   hipStream_t stream) {
  if (!period)
    return knn_large_impl<D>(tr, d_q, nq, k, d_idx, d_d2, mode, sort_q, given, OpenMetric<D>{},
                             nullptr, stream);
  TorusMetric<D> m;
  for (int a = 0; a < D; ++a) m.T.L[a] = period[a];
  return knn_large_impl<D>(tr, d_q, nq, k, d_idx, d_d2, mode, sort_q, given, m, period, stream);
}

kdt_status knn_large(const kdt_tree* tr, const float* d_q, int64_t nq, int k, int32_t* d_idx,
                     float* d_d2, int mode, bool sort_q, const int32_t* given,
                     const float* period, hipStream_t stream) {
  if (nq > INT32_MAX) {
    kdt_set_error("kdt_knn: k above %d supports at most 2^31-1 queries", KDT_MAX_K);
    return KDT_EUNSUPPORTED;
  }
  switch (tr->d) {
    case 2: return knn_large_metric<2>(tr, d_q, nq, k, d_idx, d_d2, mode, sort_q, given, period, stream);
    case 3: return knn_large_metric<3>(tr, d_q, nq, k, d_idx, d_d2, mode, sort_q, given, period, stream);
    case 4: return knn_large_metric<4>(tr, d_q, nq, k, d_idx, d_d2, mode, sort_q, given, period, stream);
    case 8: return knn_large_metric<8>(tr, d_q, nq, k, d_idx, d_d2, mode, sort_q, given, period, stream);
    case 16: return knn_large_metric<16>(tr, d_q, nq, k, d_idx, d_d2, mode, sort_q, given, period, stream);
  }
  kdt_set_error("kdt_knn: unsupported dimension %d", tr->d);
  return KDT_EUNSUPPORTED;
}

}  // namespace kdt
