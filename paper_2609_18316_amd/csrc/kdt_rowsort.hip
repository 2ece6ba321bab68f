// Per-row sort of CSR lists: every row of a ball or box list (the input
// indices of the points inside one query's region) ascending.
//
// Rows come in four sizes, each sorted where it fits:
//   <= 64 entries     in registers: one wave per row, one entry per lane,
//                     a bitonic network over the lanes (shuffles), sized to
//                     the next power of two of the row;
//   <= kSmallMax      in LDS by the same 64-lane workgroup (bitonic);
//   <= kMidMax        by a 1024-lane workgroup: bitonic over LDS (68 KiB),
//                     the steps inside each lane's run of 16 in registers;
//   longer            the library's LSD radix sort over the concatenation of
//                     those rows, ordered by (row, entry): with one composite
//                     key (row rank above the entry's bits) when both fit in
//                     32 bits, else by the entry, then stably by the row.
// A 64-lane workgroup walks chunks of 64 consecutive rows: one coalesced load
// gives the chunk's offsets, and the next row's entries are loaded while the
// current one is sorted.  Rows of the two larger classes are collected (by
// row id, through counters) for the later passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "kdt.h"
#include "kdt_bitonic.h"
#include "kdt_debug.h"
#include "kdt_internal.h"

namespace kdt {
namespace {

constexpr int kSmallMax = 1024;   // rows sorted by one 64-lane workgroup
constexpr int kMidMax = 16384;    // rows sorted by one 1024-lane workgroup
constexpr int kMidThreads = 1024;

__device__ __forceinline__ int pow2_at_least(int64_t L) {
  int P = 1;
  while (P < L) P <<= 1;
  return P;
}

// Ascending bitonic sort of s[0, P) (P a power of two) by T threads.
__device__ __forceinline__ void lds_bitonic(int32_t* s, int P, int tid, int T) {
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < (P >> 1); i += T) {
        const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
        const int hi = lo + j;
        const int32_t a = s[lo], c = s[hi];
        if ((a > c) == ((lo & k) == 0)) {
          s[lo] = c;
          s[hi] = a;
        }
      }
      __syncthreads();
    }
}

__global__ void k_zero_ctr(uint32_t* c) {
  if (threadIdx.x < 2) c[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(64) void k_rows_small(const int32_t* __restrict__ in,
                                                   int32_t* __restrict__ out,
                                                   const int64_t* __restrict__ off, int64_t nq,
                                                   uint32_t* __restrict__ ctr,
                                                   int32_t* __restrict__ mid_rows,
                                                   int32_t* __restrict__ big_rows) {
  __shared__ int32_t s[kSmallMax];
  const int lane = threadIdx.x;
  for (int64_t r0 = (int64_t)blockIdx.x * 64; r0 < nq; r0 += (int64_t)gridDim.x * 64) {
    const int nr = (int)std::min<int64_t>(64, nq - r0);
    // lane j: the bounds of row r0 + j
    const int64_t mb = lane < nr ? off[r0 + lane] : 0;
    const int64_t me = lane < nr ? off[r0 + lane + 1] : 0;
    int64_t nb = __shfl(mb, 0), ne = __shfl(me, 0);
    int32_t nxt = (ne - nb <= 64 && lane < ne - nb) ? in[nb + lane] : INT_MAX;
    for (int j = 0; j < nr; ++j) {
      const int64_t b = nb, L = ne - nb;
      int32_t v = nxt;
      if (j + 1 < nr) {  // the next row's entries load while this one sorts
        nb = __shfl(mb, j + 1);
        ne = __shfl(me, j + 1);
        nxt = (ne - nb <= 64 && lane < ne - nb) ? in[nb + lane] : INT_MAX;
      }
      if (L <= 1) {
        if (L == 1 && lane == 0) out[b] = v;
      } else if (L <= 64) {
        const int P = pow2_at_least(L);
        for (int k = 2; k <= P; k <<= 1)
          for (int m = k >> 1; m > 0; m >>= 1) {
            const int32_t o = __shfl_xor(v, m);
            v = (((lane & m) == 0) == ((lane & k) == 0)) ? min(v, o) : max(v, o);
          }
        if (lane < L) out[b + lane] = v;
      } else if (L <= kSmallMax) {
        const int P = pow2_at_least(L);
        for (int i = lane; i < P; i += 64) s[i] = i < L ? in[b + i] : INT_MAX;
        __syncthreads();
        lds_bitonic(s, P, lane, 64);
        for (int i = lane; i < L; i += 64) out[b + i] = s[i];
        __syncthreads();  // s is reused by the next row
      } else if (lane == 0) {
        if (L <= kMidMax)
          mid_rows[atomicAdd(ctr, 1u)] = (int32_t)(r0 + j);
        else
          big_rows[atomicAdd(ctr + 1, 1u)] = (int32_t)(r0 + j);
      }
    }
  }
}

// A mid row per workgroup: the entries go to LDS (padded, one slot after
// every 16), then the workgroup bitonic sort whose steps inside a thread's
// run of 16 run in registers.
__global__ __launch_bounds__(kMidThreads) void k_rows_mid(const int32_t* __restrict__ in,
                                                          int32_t* __restrict__ out,
                                                          const int64_t* __restrict__ off,
                                                          const uint32_t* __restrict__ ctr,
                                                          const int32_t* __restrict__ rows) {
  static_assert(kMidMax <= 16 * kMidThreads, "a thread owns one run of 16 entries of a row");
  __shared__ int32_t s[kMidMax + kMidMax / 16];  // entry i at s[pad16(i)]
  const uint32_t m = ctr[0];
  const int t = threadIdx.x;
  for (uint32_t i = blockIdx.x; i < m; i += gridDim.x) {
    const int64_t r = rows[i];
    const int64_t b = off[r], L = off[r + 1] - b;
    const int P = max(pow2_at_least(L), 32);  // mid rows hold more than kSmallMax entries
    for (int e = t; e < P; e += kMidThreads) s[pad16(e)] = e < L ? in[b + e] : INT_MAX;
    bitonic_runs16(s, P, t, kMidThreads);
    for (int e = t; e < L; e += kMidThreads) out[b + e] = s[pad16(e)];
    __syncthreads();
  }
}

__global__ void k_big_len(const int32_t* __restrict__ rows, uint32_t nbig,
                          const int64_t* __restrict__ off, int32_t* __restrict__ len) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nbig) len[i] = (int32_t)(off[rows[i] + 1] - off[rows[i]]);
}

// The long rows' entries are handled in chunks of kBigChunk of their
// concatenation (row rank i owns [boff[i], boff[i+1])): every row is longer
// than a chunk, so a chunk meets at most two rows -- the one holding its
// first entry (a binary search over boff) and the next.
constexpr int kBigChunk = 4096;

__device__ __forceinline__ uint32_t chunk_row(const int64_t* __restrict__ boff, uint32_t nbig,
                                              int64_t e0) {
  __shared__ uint32_t row0;
  if (threadIdx.x == 0) {
    uint32_t lo = 0, hi = nbig - 1;  // the last i with boff[i] <= e0
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (boff[mid] <= e0)
        lo = mid;
      else
        hi = mid - 1;
    }
    row0 = lo;
  }
  __syncthreads();
  return row0;
}

// Entries into the sort's arrays; composite: key = i << shift | entry,
// value = entry; else key = entry, value = i.
__global__ __launch_bounds__(256) void k_big_gather(const int32_t* __restrict__ rows,
                                                    uint32_t nbig,
                                                    const int64_t* __restrict__ off,
                                                    const int64_t* __restrict__ boff, int64_t tb,
                                                    const int32_t* __restrict__ in, int shift,
                                                    int composite, uint32_t* __restrict__ keys,
                                                    int32_t* __restrict__ vals) {
  const int64_t e0 = (int64_t)blockIdx.x * kBigChunk;
  const uint32_t i0 = chunk_row(boff, nbig, e0);
  const int64_t split = i0 + 1 < nbig ? boff[i0 + 1] : tb;
  for (int64_t e = e0 + threadIdx.x; e < e0 + kBigChunk && e < tb; e += 256) {
    const uint32_t i = e < split ? i0 : i0 + 1;
    const int32_t v = in[off[rows[i]] + (e - boff[i])];
    keys[e] = composite ? (i << shift) | (uint32_t)v : (uint32_t)v;
    vals[e] = composite ? v : (int32_t)i;
  }
}

// The sorted concatenation back into each long row's range of out.
__global__ __launch_bounds__(256) void k_big_place(const int32_t* __restrict__ rows,
                                                   uint32_t nbig,
                                                   const int64_t* __restrict__ off,
                                                   const int64_t* __restrict__ boff, int64_t tb,
                                                   const int32_t* __restrict__ sorted,
                                                   int32_t* __restrict__ out) {
  const int64_t e0 = (int64_t)blockIdx.x * kBigChunk;
  const uint32_t i0 = chunk_row(boff, nbig, e0);
  const int64_t split = i0 + 1 < nbig ? boff[i0 + 1] : tb;
  for (int64_t e = e0 + threadIdx.x; e < e0 + kBigChunk && e < tb; e += 256) {
    const uint32_t i = e < split ? i0 : i0 + 1;
    out[off[rows[i]] + (e - boff[i])] = sorted[e];
  }
}

int bits_below(int64_t limit) {  // bits of limit - 1 (at least 1)
  int b = 1;
  while (b < 32 && (int64_t(1) << b) < limit) ++b;
  return b;
}

}  // namespace

kdt_status sort_list_rows(const int32_t* in, int32_t* out, const int64_t* off, int64_t nq,
                          int64_t total, int64_t key_limit, hipStream_t stream) {
  if (nq <= 0 || total <= 0) return KDT_OK;
  if (total > INT32_MAX || nq > INT32_MAX) {
    kdt_set_error("lists above 2^31-1 entries or rows are not supported");
    return KDT_EUNSUPPORTED;
  }
  PoolBuffers buf(stream);
  uint32_t* ctr = nullptr;
  int32_t *mid = nullptr, *big = nullptr;
  if (!buf.get(&ctr, 64) || !buf.get(&mid, (size_t)nq) || !buf.get(&big, (size_t)nq)) {
    kdt_set_error("device allocation failed for sorting the lists");
    return KDT_ENOMEM;
  }
  k_zero_ctr<<<1, 64, 0, stream>>>(ctr);
  // twice the resident waves: the short rows wait on memory, not on the ALUs
  const unsigned gs = (unsigned)std::min<int64_t>((nq + 63) / 64, 256 * 64);
  k_rows_small<<<gs, 64, 0, stream>>>(in, out, off, nq, ctr, mid, big);
  k_rows_mid<<<512, kMidThreads, 0, stream>>>(in, out, off, ctr, mid);
  uint32_t h[2] = {0u, 0u};
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    kdt_set_error("sorting the lists failed");
    return KDT_EDEVICE;
  }
  const uint32_t nbig = h[1];
  if (nbig == 0) return KDT_OK;
  // rows above kMidMax entries: their concatenation through the radix sort
  int32_t* len = nullptr;
  int64_t* boff = nullptr;
  void* scan_tmp = nullptr;
  if (!buf.get(&len, nbig) || !buf.get(&boff, (size_t)nbig + 1) ||
      !buf.get((char**)&scan_tmp, scan_scratch_bytes(nbig))) {
    kdt_set_error("device allocation failed for sorting the lists");
    return KDT_ENOMEM;
  }
  k_big_len<<<(nbig + 255) / 256, 256, 0, stream>>>(big, nbig, off, len);
  int64_t tb = 0;
  if (exclusive_scan<int64_t>(len, boff, nbig, boff + nbig, scan_tmp, stream) != KDT_OK ||
      hipMemcpyAsync(&tb, boff + nbig, sizeof(tb), hipMemcpyDeviceToHost, stream) !=
          hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    kdt_set_error("sorting the long list rows failed");
    return KDT_EDEVICE;
  }
  uint32_t* keys[2] = {nullptr, nullptr};
  int32_t* vals[2] = {nullptr, nullptr};
  void* rs_tmp = nullptr;
  if (!buf.get(&keys[0], (size_t)tb) || !buf.get(&keys[1], (size_t)tb) ||
      !buf.get(&vals[0], (size_t)tb) || !buf.get(&vals[1], (size_t)tb) ||
      !buf.get((char**)&rs_tmp, radix_sort_scratch_bytes(tb))) {
    kdt_set_error("device allocation failed for sorting the long list rows");
    return KDT_ENOMEM;
  }
  const int kb = bits_below(key_limit), rb = bits_below(nbig);
  const bool composite = kb + rb <= 32;
  const unsigned gc = (unsigned)((tb + kBigChunk - 1) / kBigChunk);
  k_big_gather<<<gc, 256, 0, stream>>>(big, nbig, off, boff, tb, in, kb, composite ? 1 : 0,
                                       keys[0], vals[0]);
  const int32_t* sorted = nullptr;
  if (composite) {
    const int c = radix_sort_pairs(keys, vals, tb, 0, kb + rb, rs_tmp, stream);
    sorted = vals[c];
  } else {
    // by the entry, then stably by the row (the arrays swap roles)
    const int a = radix_sort_pairs(keys, vals, tb, 0, kb, rs_tmp, stream);
    uint32_t* k2[2] = {reinterpret_cast<uint32_t*>(vals[a]),
                       reinterpret_cast<uint32_t*>(vals[a ^ 1])};
    int32_t* v2[2] = {reinterpret_cast<int32_t*>(keys[a]), reinterpret_cast<int32_t*>(keys[a ^ 1])};
    const int c = radix_sort_pairs(k2, v2, tb, 0, rb, rs_tmp, stream);
    sorted = v2[c];
  }
  k_big_place<<<gc, 256, 0, stream>>>(big, nbig, off, boff, tb, sorted, out);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("sorting the long list rows failed");
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

}  // namespace kdt

extern "C" kdt_status kdt_debug_sort_rows(const int32_t* d_in, int32_t* d_out,
                                          const int64_t* d_off, int64_t nq, int64_t total,
                                          hipStream_t stream) {
  kdt_clear_error();
  if (nq < 0 || nq > INT32_MAX || total < 0 || total > INT32_MAX ||
      (total > 0 && (!d_in || !d_out || d_in == d_out)) || (nq > 0 && !d_off)) {
    kdt_set_error("kdt_debug_sort_rows: NULL or equal arrays, nq or total outside "
                  "[0, 2^31-1]");
    return KDT_EINVAL;
  }
  return kdt::sort_list_rows(d_in, d_out, d_off, nq, total, int64_t(1) << 31, stream);
}
