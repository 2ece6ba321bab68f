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

}  // namespace

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
