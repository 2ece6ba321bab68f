// Per-row sort of CSR lists: every row of a ball or box list (the input
// indices of the points inside one query's region) ascending.
//
// Rows come in four sizes, each sorted where it fits:
//   <= 64 entries     in registers: one wave per row, one entry per lane,
//                     a bitonic network over the lanes (shuffles), sized to
//                     the next power of two of the row;
//   <= kSmallMax      in LDS by the same 64-lane workgroup (bitonic);
//   <= kMidMax        in LDS by a 1024-lane workgroup (bitonic; 64 KiB);
//   longer            hipCUB's segmented sort over those rows only.
// A 64-lane workgroup walks chunks of 64 consecutive rows: one coalesced load
// gives the chunk's offsets, and the next row's entries are loaded while the
// current one is sorted.  Rows of the two larger classes are collected (by
// row id, through counters) for the later passes.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "kdt.h"
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

__global__ __launch_bounds__(kMidThreads) void k_rows_mid(const int32_t* __restrict__ in,
                                                          int32_t* __restrict__ out,
                                                          const int64_t* __restrict__ off,
                                                          const uint32_t* __restrict__ ctr,
                                                          const int32_t* __restrict__ rows) {
  __shared__ int32_t s[kMidMax];
  const uint32_t m = ctr[0];
  for (uint32_t i = blockIdx.x; i < m; i += gridDim.x) {
    const int64_t r = rows[i];
    const int64_t b = off[r], L = off[r + 1] - b;
    const int P = pow2_at_least(L);
    for (int e = threadIdx.x; e < P; e += kMidThreads) s[e] = e < L ? in[b + e] : INT_MAX;
    __syncthreads();
    lds_bitonic(s, P, threadIdx.x, kMidThreads);
    for (int e = threadIdx.x; e < L; e += kMidThreads) out[b + e] = s[e];
    __syncthreads();
  }
}

__global__ void k_big_bounds(const int32_t* __restrict__ rows, uint32_t nbig,
                             const int64_t* __restrict__ off, int64_t* __restrict__ begin,
                             int64_t* __restrict__ end) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbig) return;
  begin[i] = off[rows[i]];
  end[i] = off[rows[i] + 1];
}

}  // namespace

kdt_status sort_list_rows(const int32_t* in, int32_t* out, const int64_t* off, int64_t nq,
                          int64_t total, hipStream_t stream) {
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
  const unsigned gs = (unsigned)std::min<int64_t>((nq + 63) / 64, 256 * 32);
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
  // rows above kMidMax entries: hipCUB's segmented sort over those rows
  int64_t *bb = nullptr, *be = nullptr;
  void* tmp = nullptr;
  size_t tb = 0;
  if (!buf.get(&bb, nbig) || !buf.get(&be, nbig)) {
    kdt_set_error("device allocation failed for sorting the lists");
    return KDT_ENOMEM;
  }
  k_big_bounds<<<(nbig + 255) / 256, 256, 0, stream>>>(big, nbig, off, bb, be);
  if (hipcub::DeviceSegmentedSort::SortKeys(nullptr, tb, in, out, (int)total, (int)nbig, bb, be,
                                            stream) != hipSuccess) {
    kdt_set_error("sorting the long list rows failed");
    return KDT_EDEVICE;
  }
  if (!buf.get((char**)&tmp, tb)) {
    kdt_set_error("device allocation failed for sorting the lists");
    return KDT_ENOMEM;
  }
  if (hipcub::DeviceSegmentedSort::SortKeys(tmp, tb, in, out, (int)total, (int)nbig, bb, be,
                                            stream) != hipSuccess) {
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
  return kdt::sort_list_rows(d_in, d_out, d_off, nq, total, stream);
}
