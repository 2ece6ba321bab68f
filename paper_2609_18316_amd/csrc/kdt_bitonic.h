// kdt_bitonic.h -- the workgroup bitonic sort over LDS that the per-row
// sorts share (candidate keys of large-k rows, entries of CSR list rows).
#pragma once

#include <hip/hip_runtime.h>

namespace kdt {

// Key i of a row sort lives at LDS slot pad16(i): one unused slot after
// every 16 keys, so the runs of 16 that neighbouring lanes load start 17
// keys apart and a wave's run loads spread over all the banks, where
// unpadded they would all fall on the same few.  A sort of P keys needs
// P + P / 16 slots.
__host__ __device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

// The bitonic stages up to merges of 16 over one run held in registers, the
// run starting at key position `base` (directions from the positions).
template <class K>
__device__ __forceinline__ void run16_sort(K v[16], int base) {
#pragma unroll
  for (int k = 2; k <= 16; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int p = q ^ j;
        if (p > q) {
          const bool up = ((base + q) & k) == 0;
          const K a = v[q], c = v[p];
          const bool sw = (a > c) == up;
          v[q] = sw ? c : a;
          v[p] = sw ? a : c;
        }
      }
  }
}

// Ascending bitonic sort of keys [0, pn) (pn a power of two, 32 <= pn <= 16
// T; key i at s[pad16(i)], padding keys already in place) by the T threads
// of the workgroup, thread t owning the run of keys [16 t, 16 t + 16): the
// steps that stay inside a run (every step of the merges up to 16, and the
// last four of each larger merge) run in registers, one LDS load and store
// per run; the others in LDS.  65 instead of 105 LDS passes at pn = 16384.
// Starts and ends with the workgroup synchronised.
template <class K>
__device__ __forceinline__ void bitonic_runs16(K* s, int pn, int tid, int T) {
  const bool own = tid * 16 < pn;
  K v[16];
  __syncthreads();
  if (own) {
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = s[tid * 17 + q];
    run16_sort(v, tid * 16);
#pragma unroll
    for (int q = 0; q < 16; ++q) s[tid * 17 + q] = v[q];
  }
  __syncthreads();
  for (int k = 32; k <= pn; k <<= 1) {
    for (int j = k >> 1; j >= 16; j >>= 1) {
      for (int t = tid; t < pn / 2; t += T) {
        const int lo = 2 * t - (t & (j - 1));
        const int hi = lo + j;
        const K a = s[pad16(lo)], c = s[pad16(hi)];
        if ((a > c) == ((lo & k) == 0)) {
          s[pad16(lo)] = c;
          s[pad16(hi)] = a;
        }
      }
      __syncthreads();
    }
    if (own) {
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = s[tid * 17 + q];
      // the rest of merge k inside the run: steps 8, 4, 2, 1, direction from bit k
      const bool up = ((tid * 16) & k) == 0;
#pragma unroll
      for (int j = 8; j > 0; j >>= 1)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int p = q ^ j;
          if (p > q) {
            const K a = v[q], c = v[p];
            const bool sw = (a > c) == up;
            v[q] = sw ? c : a;
            v[p] = sw ? a : c;
          }
        }
#pragma unroll
      for (int q = 0; q < 16; ++q) s[tid * 17 + q] = v[q];
    }
    __syncthreads();
  }
}

}  // namespace kdt
