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

// One compare-exchange of a bitonic step: a keeps the smaller key when up.
template <class K>
__host__ __device__ __forceinline__ void bitonic_cx(K& a, K& b, bool up) {
  const K x = a, y = b;
  const bool sw = (x > y) == up;
  a = sw ? y : x;
  b = sw ? x : y;
}

// The bitonic stages up to merges of 16 over one run held in registers, the
// run starting at key position `base` (directions from the positions).
template <class K>
__host__ __device__ __forceinline__ void run16_sort(K v[16], int base) {
#pragma unroll
  for (int k = 2; k <= 16; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int p = q ^ j;
        if (p > q) bitonic_cx(v[q], v[p], ((base + q) & k) == 0);
      }
  }
}

// The per-thread parts of the workgroup sort below, one phase each (the
// workgroup synchronises between phases; within one, threads touch disjoint
// keys).  Thread t's run is keys [16 t, 16 t + 16); its strided set is the
// keys b + 16 q (q < 16) of the 256-key block t / 16, b = 256 (t / 16) +
// t % 16, whose pairs at steps 16 .. 128 of a merge lie inside the set.

// Merges up to 16 inside thread t's run.
template <class K>
__host__ __device__ __forceinline__ void bitonic_first_runs(K* s, int t) {
  K v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = s[t * 17 + q];
  run16_sort(v, t * 16);
#pragma unroll
  for (int q = 0; q < 16; ++q) s[t * 17 + q] = v[q];
}

// Step j of merge k over LDS: the pairs t, t + T, ... of the pn / 2.
template <class K>
__host__ __device__ __forceinline__ void bitonic_lds_step(K* s, int pn, int k, int j, int tid,
                                                          int T) {
  for (int t = tid; t < pn / 2; t += T) {
    const int lo = 2 * t - (t & (j - 1));
    const int hi = lo + j;
    K a = s[pad16(lo)], c = s[pad16(hi)];
    if ((a > c) == ((lo & k) == 0)) {
      s[pad16(lo)] = c;
      s[pad16(hi)] = a;
    }
  }
}

// Steps 128 (or k / 2 if smaller) down to 16 of merge k over thread t's
// strided set (needs keys in whole blocks of 256).
template <class K>
__host__ __device__ __forceinline__ void bitonic_strided_steps(K* s, int k, int t) {
  // key b + 16 q sits at slot pad16(b + 16 q) = slot0 + 17 q (t % 16 < 16),
  // and its bits from 16 up are (t / 16) << 8 | q << 4
  const int slot0 = (t >> 4) * 272 + (t & 15);
  const int high = (t >> 4) << 8;
  K v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = s[slot0 + 17 * q];
#pragma unroll
  for (int m = 3; m >= 0; --m) {  // step 16 << m, pairs q and q ^ (1 << m)
    if ((16 << m) < k) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int p = q ^ (1 << m);
        if (p > q) bitonic_cx(v[q], v[p], ((high | (q << 4)) & k) == 0);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) s[slot0 + 17 * q] = v[q];
}

// Steps 8, 4, 2, 1 of merge k (k >= 32) inside thread t's run: one direction
// for the whole run, from bit k of its position.
template <class K>
__host__ __device__ __forceinline__ void bitonic_run_steps(K* s, int k, int t) {
  K v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = s[t * 17 + q];
  const bool up = ((t * 16) & k) == 0;
#pragma unroll
  for (int j = 8; j > 0; j >>= 1)
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int p = q ^ j;
      if (p > q) bitonic_cx(v[q], v[p], up);
    }
#pragma unroll
  for (int q = 0; q < 16; ++q) s[t * 17 + q] = v[q];
}

// Ascending bitonic sort of keys [0, pn) (pn a power of two, 32 <= pn <= 16
// T; key i at s[pad16(i)], padding keys already in place) by the T threads
// of the workgroup.  Only the steps that cross a thread's keys go through
// LDS one pass each: every step of the merges up to 16 and steps 8 .. 1 of
// each larger merge run in registers over the thread's run, and, from pn =
// 256 on, steps 128 .. 16 over its strided set -- one LDS load and store per
// phase.  41 instead of 105 LDS passes at pn = 16384 (65 with the runs
// alone).  Starts and ends with the workgroup synchronised.
template <class K>
__device__ __forceinline__ void bitonic_runs16(K* s, int pn, int tid, int T) {
  const bool own = tid * 16 < pn;
  const bool strided = pn >= 256;
  __syncthreads();
  if (own) bitonic_first_runs(s, tid);
  __syncthreads();
  for (int k = 32; k <= pn; k <<= 1) {
    for (int j = k >> 1; j >= (strided ? 256 : 16); j >>= 1) {
      bitonic_lds_step(s, pn, k, j, tid, T);
      __syncthreads();
    }
    if (strided) {
      if (own) bitonic_strided_steps(s, k, tid);
      __syncthreads();
    }
    if (own) bitonic_run_steps(s, k, tid);
    __syncthreads();
  }
}

}  // namespace kdt
