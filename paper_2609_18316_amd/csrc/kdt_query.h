// kdt_query.h -- device-side tree view and traversal helpers shared by the
// query, grouping and batched kernels.
#pragma once

#include "kdt_internal.h"

namespace kdt {

constexpr int kMaxDepth = 32;  // levels <= 30 for n < 2^31 and leaf_size >= 2

struct TreeView {
  const float* rec;  // [n][rec_stride(D)] tree-ordered records
  const float* box;  // [n_nodes][2 * pad4(D)]
  int64_t n;
  int32_t levels;
};

template <int D>
struct Pt {
  float v[D];
};

template <int D>
__device__ __forceinline__ void load_box(const float* __restrict__ box, uint32_t node, float lo[D],
                                         float hi[D]) {
  constexpr int P = pad4(D);
  const float4* b = reinterpret_cast<const float4*>(box + (size_t)node * 2 * P);
#pragma unroll
  for (int q = 0; q < P / 4; ++q) {
    float4 l = b[q], h = b[P / 4 + q];
    if (4 * q + 0 < D) lo[4 * q + 0] = l.x, hi[4 * q + 0] = h.x;
    if (4 * q + 1 < D) lo[4 * q + 1] = l.y, hi[4 * q + 1] = h.y;
    if (4 * q + 2 < D) lo[4 * q + 2] = l.z, hi[4 * q + 2] = h.z;
    if (4 * q + 3 < D) lo[4 * q + 3] = l.w, hi[4 * q + 3] = h.w;
  }
}

// Smallest squared distance from p to the box: the same float32 operations,
// in the same axis order, as the point distance, so it never exceeds the
// rounded distance of any point inside the box.
template <int D>
__device__ __forceinline__ float box_mindist(const float lo[D], const float hi[D], const float p[D]) {
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float t = 0.0f;
    if (p[a] < lo[a]) t = lo[a] - p[a];
    else if (p[a] > hi[a]) t = p[a] - hi[a];
    float t2 = t * t;
    s = s + t2;
  }
  return s;
}

// Largest squared distance from p to the box (never below any point's).
template <int D>
__device__ __forceinline__ float box_maxdist(const float lo[D], const float hi[D], const float p[D]) {
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float t1 = fabsf(p[a] - lo[a]);
    float t2 = fabsf(p[a] - hi[a]);
    float t = t1 > t2 ? t1 : t2;
    float tt = t * t;
    s = s + tt;
  }
  return s;
}

// Squared Euclidean distance (Eq. 1, p = 2): float32, axes left to right,
// every operation rounded on its own (the library is built without FMA
// contraction).
template <int D>
__device__ __forceinline__ float sq_dist(const float* __restrict__ x, const float p[D]) {
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float t = x[a] - p[a];
    float t2 = t * t;
    s = s + t2;
  }
  return s;
}

template <int D>
__device__ __forceinline__ void load_rec(const float* __restrict__ rec, int64_t i, float x[D],
                                         int32_t& idx) {
  constexpr int S = rec_stride(D);
  const float4* r = reinterpret_cast<const float4*>(rec + i * S);
#pragma unroll
  for (int q = 0; q < S / 4; ++q) {
    float4 v = r[q];
    float w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int a = 4 * q + c;
      if (a < D) x[a] = w[c];
      if (a == D) idx = __float_as_int(w[c]);
    }
  }
}

// Key of an empty candidate slot: squared distance +inf, index 0xFFFFFFFF, so
// it sorts after every real point (indices are below 2^31).
constexpr uint64_t kEmptyKey = 0x7F800000FFFFFFFFull;

// Sorted register list of the KC smallest 64-bit keys (d2 bits << 32 | index).
// Only the last k slots are live: the first KC - k hold 0 and never move.
template <int KC>
struct TopK {
  uint64_t a[KC];
  __device__ __forceinline__ void init(int k) {
#pragma unroll
    for (int i = 0; i < KC; ++i) a[i] = (i < KC - k) ? 0ull : kEmptyKey;
  }
  __device__ __forceinline__ uint64_t worst() const { return a[KC - 1]; }
  __device__ __forceinline__ float worst_d2() const {
    return __uint_as_float((uint32_t)(a[KC - 1] >> 32));
  }
  // requires x < worst()
  __device__ __forceinline__ void insert(uint64_t x) {
#pragma unroll
    for (int i = KC - 1; i > 0; --i) {
      const uint64_t lo = a[i - 1];
      const uint64_t cur = a[i];
      a[i] = (x < lo) ? lo : ((x < cur) ? x : cur);
    }
    a[0] = (x < a[0]) ? x : a[0];
  }
};

__device__ __forceinline__ uint64_t make_key(float d2, int32_t idx) {
  return ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)idx;
}

}  // namespace kdt
