// Stable LSD radix sort of (uint32 key, int32 value) pairs: the query orders
// (Hilbert or leaf keys) and the deposit's particle order.
//
// 8 key bits per pass over [begin_bit, end_bit).  A pass is three kernels:
//   hist     one workgroup per tile of kTile keys: the tile's digit counts,
//            stored digit-major (count[digit][tile]);
//   scan     one workgroup per digit: the exclusive running sum of the
//            digit's counts over the tiles (a contiguous row), and the
//            digit's total; the scatter adds the running sum of the totals
//            over the lower digits, so (digit, tile) gives the first output
//            slot of the tile's keys of that digit (keys of lower digits, then
//            of the same digit in earlier tiles: the sort is stable);
//   scatter  per tile: each key's rank among the tile's keys of its digit,
//            in input order -- items are dealt out round by round (item
//            r * kThreads + thread), and within a round a wave finds the
//            lanes that share a digit with eight ballots -- then the tile is
//            staged in LDS in digit order and written out as one coalesced
//            run per digit.
// Results are bit-identical to a stable sort on the selected bits.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kdt.h"
#include "kdt_internal.h"

namespace kdt {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // 4096 keys per tile
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ uint32_t digit_of(uint32_t key, int shift, uint32_t mask) {
  return (key >> shift) & mask;
}

__global__ __launch_bounds__(kThreads) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                      int shift, uint32_t mask, int64_t tiles,
                                                      uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + r * kThreads + tid;
    if (i < n) atomicAdd(&h[digit_of(keys[i], shift, mask)], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * tiles + blockIdx.x] = h[tid];
}

// Exclusive running sum of a block of kThreads values, one per thread; the
// block total in *total (every thread).
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = (uint32_t)__shfl_up((int)incl, off);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t carry = 0u, all = 0u;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    if (w < wave) carry += wsum[w];
    all += wsum[w];
  }
  __syncthreads();  // wsum may be reused
  *total = all;
  return carry + incl - v;
}

// One workgroup per digit: the exclusive running sum of its row of tile
// counts (coalesced, kThreads tiles per step) and the row total.
__global__ __launch_bounds__(kThreads) void k_rs_scan(uint32_t* __restrict__ hist, int64_t tiles,
                                                      uint32_t* __restrict__ totals) {
  __shared__ uint32_t wsum[kWaves];
  uint32_t* row = hist + (int64_t)blockIdx.x * tiles;
  uint32_t run = 0u;
  for (int64_t b = 0; b < tiles; b += kThreads) {
    const int64_t i = b + threadIdx.x;
    const uint32_t v = i < tiles ? row[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive(v, wsum, &tot);
    if (i < tiles) row[i] = run + ex;
    run += tot;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = run;
}

__global__ __launch_bounds__(kThreads) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                         const int32_t* __restrict__ vin,
                                                         int64_t n, int shift, uint32_t mask,
                                                         int64_t tiles,
                                                         const uint32_t* __restrict__ hist,
                                                         const uint32_t* __restrict__ totals,
                                                         uint32_t* __restrict__ kout,
                                                         int32_t* __restrict__ vout) {
  __shared__ uint32_t sk[kTile];
  __shared__ uint32_t dbase[256];  // keys of lower digits, over all tiles
  __shared__ int32_t sv[kTile];
  __shared__ uint32_t wcnt[kWaves][256];
  __shared__ uint32_t cnt[256];
  __shared__ uint32_t start[256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  cnt[tid] = 0u;
  {
    __shared__ uint32_t ws[kWaves];
    uint32_t tot;
    dbase[tid] = block_exclusive(totals[tid], ws, &tot);
  }
  uint32_t key[kItems];
  int32_t val[kItems];
  uint32_t rank[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + r * kThreads + tid;
    const bool valid = i < n;
    key[r] = valid ? kin[i] : 0u;
    val[r] = valid ? vin[i] : 0;
    const uint32_t dg = digit_of(key[r], shift, mask);
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0u;
    __syncthreads();
    // the lanes of this wave holding the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool b = (dg >> bit) & 1u;
      const uint64_t m = __ballot(valid && b);
      peers &= b ? m : ~m;
    }
    const uint32_t rw = (uint32_t)__popcll(peers & below);
    if (valid && rw == 0u) wcnt[wave][dg] = (uint32_t)__popcll(peers);
    __syncthreads();
    uint32_t before = cnt[dg];
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
      if (w < wave) before += wcnt[w][dg];
    rank[r] = before + rw;
    __syncthreads();
    uint32_t add = 0u;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) add += wcnt[w][tid];
    cnt[tid] += add;
    __syncthreads();
  }
  // first position of each digit in the tile (exclusive scan of cnt)
  {
    __shared__ uint32_t ws[kWaves];
    uint32_t tot;
    start[tid] = block_exclusive(cnt[tid], ws, &tot);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + r * kThreads + tid;
    if (i < n) {
      const uint32_t p = start[digit_of(key[r], shift, mask)] + rank[r];
      sk[p] = key[r];
      sv[p] = val[r];
    }
  }
  __syncthreads();
  const int64_t have = n - base < kTile ? n - base : kTile;
  for (int j = tid; j < have; j += kThreads) {
    const uint32_t k = sk[j];
    const uint32_t dg = digit_of(k, shift, mask);
    const int64_t at =
        (int64_t)dbase[dg] + hist[(int64_t)dg * tiles + blockIdx.x] + (j - start[dg]);
    kout[at] = k;
    vout[at] = sv[j];
  }
}

// --- exclusive scan of int32 values (CSR offsets, the midpoint build's ranks)
//
// Three kernels: the sum of each tile of kTile values; one workgroup turning
// the tile sums into tile offsets (and the total); per tile, the running sum
// of its values from its offset.  Loads and stores go through LDS so that
// both are coalesced; sums are 64-bit.

// Per tile of kTile values: their sum (ROOTS: the number of i with in[i] == i).
template <bool ROOTS>
__global__ __launch_bounds__(kThreads) void k_scan_tiles(const int32_t* __restrict__ in, int64_t n,
                                                         int64_t* __restrict__ tsum) {
  __shared__ int64_t part[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  int64_t s = 0;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + r * kThreads + threadIdx.x;
    if (i < n) s += ROOTS ? (int64_t)(in[i] == (int32_t)i) : (int64_t)in[i];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kWaves; ++w) t += part[w];
    tsum[blockIdx.x] = t;
  }
}

// Exclusive running sum of a block of values (64-bit), the block total in *total.
__device__ __forceinline__ int64_t block_exclusive64(int64_t v, int64_t* wsum, int64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int64_t carry = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    if (w < wave) carry += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return carry + incl - v;
}

// One workgroup: tile sums -> tile offsets, in steps of kThreads; tsum[tiles]
// gets the total.
__global__ __launch_bounds__(kThreads) void k_scan_top(int64_t* __restrict__ tsum, int64_t tiles) {
  __shared__ int64_t wsum[kWaves];
  int64_t run = 0;
  for (int64_t b = 0; b < tiles; b += kThreads) {
    const int64_t i = b + threadIdx.x;
    const int64_t v = i < tiles ? tsum[i] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive64(v, wsum, &tot);
    if (i < tiles) tsum[i] = run + ex;
    run += tot;
  }
  if (threadIdx.x == 0) tsum[tiles] = run;
}

// Per tile: out[i] = offset of the tile + the sum of the tile's values before i.
template <typename Out>
__global__ __launch_bounds__(kThreads) void k_scan_apply(const int32_t* __restrict__ in, int64_t n,
                                                         const int64_t* __restrict__ tsum,
                                                         Out* __restrict__ out) {
  __shared__ int64_t buf[kTile];
  __shared__ int64_t wsum[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const int tid = threadIdx.x;
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + r * kThreads + tid;
    buf[r * kThreads + tid] = i < n ? (int64_t)in[i] : 0;
  }
  __syncthreads();
  // thread t owns values [t * kItems, (t + 1) * kItems) of the tile
  int64_t mine = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) mine += buf[tid * kItems + j];
  int64_t tot;
  int64_t run = tsum[blockIdx.x] + block_exclusive64(mine, wsum, &tot);
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int64_t v = buf[tid * kItems + j];
    buf[tid * kItems + j] = run;
    run += v;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + r * kThreads + tid;
    if (i < n) out[i] = (Out)buf[r * kThreads + tid];
  }
}

__global__ void k_scan_total(const int64_t* __restrict__ tsum, int64_t tiles, int64_t* out_n) {
  *out_n = tsum[tiles];
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
  const int64_t tiles = (n + kTile - 1) / kTile;
  return sizeof(int64_t) * (size_t)(tiles + 1);
}

template <typename Out>
kdt_status exclusive_scan(const int32_t* in, Out* out, int64_t n, int64_t* total_at,
                          void* scratch, hipStream_t stream) {
  if (n <= 0) {
    if (total_at) {
      int64_t* z = static_cast<int64_t*>(scratch);
      k_scan_top<<<1, kThreads, 0, stream>>>(z, 0);
      k_scan_total<<<1, 1, 0, stream>>>(z, 0, total_at);
    }
    return hipGetLastError() == hipSuccess ? KDT_OK : KDT_EDEVICE;
  }
  const int64_t tiles = (n + kTile - 1) / kTile;
  int64_t* tsum = static_cast<int64_t*>(scratch);
  k_scan_tiles<false><<<(unsigned)tiles, kThreads, 0, stream>>>(in, n, tsum);
  k_scan_top<<<1, kThreads, 0, stream>>>(tsum, tiles);
  k_scan_apply<Out><<<(unsigned)tiles, kThreads, 0, stream>>>(in, n, tsum, out);
  if (total_at) k_scan_total<<<1, 1, 0, stream>>>(tsum, tiles, total_at);
  return hipGetLastError() == hipSuccess ? KDT_OK : KDT_EDEVICE;
}

kdt_status count_roots(const int32_t* labels, int64_t n, int64_t* out, void* scratch,
                       hipStream_t stream) {
  const int64_t tiles = (n + kTile - 1) / kTile;
  int64_t* tsum = static_cast<int64_t*>(scratch);
  if (tiles > 0) k_scan_tiles<true><<<(unsigned)tiles, kThreads, 0, stream>>>(labels, n, tsum);
  k_scan_top<<<1, kThreads, 0, stream>>>(tsum, tiles);
  k_scan_total<<<1, 1, 0, stream>>>(tsum, tiles, out);
  return hipGetLastError() == hipSuccess ? KDT_OK : KDT_EDEVICE;
}

template kdt_status exclusive_scan<int32_t>(const int32_t*, int32_t*, int64_t, int64_t*, void*,
                                            hipStream_t);
template kdt_status exclusive_scan<int64_t>(const int32_t*, int64_t*, int64_t, int64_t*, void*,
                                            hipStream_t);

size_t radix_sort_scratch_bytes(int64_t n) {
  const int64_t tiles = (n + kTile - 1) / kTile;
  return sizeof(uint32_t) * 256 * ((size_t)(tiles > 0 ? tiles : 1) + 1);
}

int radix_sort_pairs(uint32_t* keys[2], int32_t* vals[2], int64_t n, int begin_bit, int end_bit,
                     void* scratch, hipStream_t stream) {
  int cur = 0;
  if (n <= 1 || end_bit <= begin_bit) return cur;
  const int64_t tiles = (n + kTile - 1) / kTile;
  uint32_t* hist = static_cast<uint32_t*>(scratch);
  uint32_t* totals = hist + 256 * tiles;
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    const int bits = end_bit - shift < 8 ? end_bit - shift : 8;
    const uint32_t mask = (1u << bits) - 1u;
    k_rs_hist<<<(unsigned)tiles, kThreads, 0, stream>>>(keys[cur], n, shift, mask, tiles, hist);
    k_rs_scan<<<256, kThreads, 0, stream>>>(hist, tiles, totals);
    k_rs_scatter<<<(unsigned)tiles, kThreads, 0, stream>>>(keys[cur], vals[cur], n, shift, mask,
                                                          tiles, hist, totals, keys[cur ^ 1],
                                                          vals[cur ^ 1]);
    cur ^= 1;
  }
  return cur;
}

}  // namespace kdt

extern "C" kdt_status kdt_debug_radix_sort(uint32_t* d_keys, int32_t* d_vals, int64_t n,
                                           int32_t begin_bit, int32_t end_bit,
                                           hipStream_t stream) {
  kdt_clear_error();
  if (n < 0 || n > INT32_MAX || (n > 0 && (!d_keys || !d_vals)) || begin_bit < 0 ||
      end_bit > 32 || begin_bit > end_bit) {
    kdt_set_error("kdt_debug_radix_sort: NULL arrays, n outside [0, 2^31-1] or bits outside "
                  "0 <= begin <= end <= 32");
    return KDT_EINVAL;
  }
  if (n <= 1 || begin_bit == end_bit) return KDT_OK;
  kdt::PoolBuffers buf(stream);
  uint32_t* k1 = nullptr;
  int32_t* v1 = nullptr;
  void* scratch = nullptr;
  if (!buf.get(&k1, (size_t)n) || !buf.get(&v1, (size_t)n) ||
      !buf.get((char**)&scratch, kdt::radix_sort_scratch_bytes(n))) {
    kdt_set_error("kdt_debug_radix_sort: device allocation failed");
    return KDT_ENOMEM;
  }
  uint32_t* keys[2] = {d_keys, k1};
  int32_t* vals[2] = {d_vals, v1};
  const int cur = kdt::radix_sort_pairs(keys, vals, n, begin_bit, end_bit, scratch, stream);
  if (cur == 1) {
    if (hipMemcpyAsync(d_keys, k1, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice,
                       stream) != hipSuccess ||
        hipMemcpyAsync(d_vals, v1, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice,
                       stream) != hipSuccess) {
      kdt_set_error("kdt_debug_radix_sort: copy failed");
      return KDT_EDEVICE;
    }
  }
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_debug_radix_sort: launch failed");
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

extern "C" kdt_status kdt_debug_exclusive_scan(const int32_t* d_in, void* d_out, int64_t n,
                                               int32_t out_bits, hipStream_t stream) {
  kdt_clear_error();
  if (n < 0 || n > INT32_MAX || (n > 0 && !d_in) || ((n > 0 || out_bits == 64) && !d_out) ||
      (out_bits != 32 && out_bits != 64)) {
    kdt_set_error("kdt_debug_exclusive_scan: NULL arrays, n outside [0, 2^31-1] or out_bits "
                  "not 32 or 64");
    return KDT_EINVAL;
  }
  kdt::PoolBuffers buf(stream);
  void* scratch = nullptr;
  if (!buf.get((char**)&scratch, kdt::scan_scratch_bytes(n))) {
    kdt_set_error("kdt_debug_exclusive_scan: device allocation failed");
    return KDT_ENOMEM;
  }
  kdt_status st;
  if (out_bits == 64) {
    int64_t* out = static_cast<int64_t*>(d_out);
    st = kdt::exclusive_scan<int64_t>(d_in, out, n, out + n, scratch, stream);
  } else {
    st = n > 0 ? kdt::exclusive_scan<int32_t>(d_in, static_cast<int32_t*>(d_out), n, nullptr,
                                              scratch, stream)
               : KDT_OK;
  }
  if (st != KDT_OK) kdt_set_error("kdt_debug_exclusive_scan: launch failed");
  return st;
}
