// kdt_torus.h -- the distance on the D-torus (periodic boundary conditions,
// Sec. 2.1 and Sec. 2.4) shared by the per-lane torus kernels and the
// wave-shared ball counts: the metric, a lower bound over a node box, and the
// torus ball as a query shape of the generic count traversal.
#pragma once

#include "kdt_query.h"

namespace kdt {

template <int D>
struct Torus {
  float L[D];
};

// Squared torus distance: per axis g = |x - p|, the way round L - g, the
// shorter of the two squared; summed left to right.
template <int D>
__device__ __forceinline__ float torus_sq_dist(const float* __restrict__ x, const float p[D],
                                               const Torus<D>& T) {
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float g = fabsf(x[a] - p[a]);
    const float w = T.L[a] - g;
    const float t = w < g ? w : g;
    const float t2 = t * t;
    s = s + t2;
  }
  return s;
}

// Lower bound of torus_sq_dist over the points of the box [lo, hi].  Below
// the box (lo > p) a point's gap lies between lo - p and hi - p, so its way
// round is at least L - (hi - p); above it, symmetrically.  Every step is a
// rounded operation that is monotone in the point's coordinate, so the bound
// never exceeds the rounded distance of any point inside.
template <int D>
__device__ __forceinline__ float torus_box_mindist(const float lo[D], const float hi[D],
                                                   const float p[D], const Torus<D>& T) {
  float s = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float below = lo[a] - p[a];
    const float above = p[a] - hi[a];
    float t = 0.0f;
    if (below > 0.0f) {
      const float w = T.L[a] - (hi[a] - p[a]);
      t = w < below ? w : below;
    } else if (above > 0.0f) {
      const float w = T.L[a] - (p[a] - lo[a]);
      t = w < above ? w : above;
    }
    const float t2 = t * t;
    s = s + t2;
  }
  return s;
}

// A closed ball on the torus: centre p, squared radius r2 and the periods
// (the same for all queries of a launch).  A node lies inside when its
// open-space farthest corner does: the torus distance never exceeds the open
// one, so that bound holds for every point of the node.
template <int D>
struct TorusBallShape {
  static constexpr int kFloats = D;
  float p[D];
  float r2;
  Torus<D> T;
  __device__ __forceinline__ bool cuts(const float lo[D], const float hi[D]) const {
    return torus_box_mindist<D>(lo, hi, p, T) <= r2;
  }
  __device__ __forceinline__ bool holds_box(const float lo[D], const float hi[D]) const {
    return box_maxdist<D>(lo, hi, p) <= r2;
  }
  __device__ __forceinline__ bool holds(const float x[D]) const {
    return torus_sq_dist<D>(x, p, T) <= r2;
  }
  __device__ __forceinline__ void pack(float* dst) const {
#pragma unroll
    for (int a = 0; a < D; ++a) dst[a] = p[a];
  }
  __device__ __forceinline__ TorusBallShape unpack(const float* src) const {
    TorusBallShape b;
#pragma unroll
    for (int a = 0; a < D; ++a) b.p[a] = src[a];
    b.r2 = r2;
    b.T = T;
    return b;
  }
};

// The torus metric for the wave-shared grouping: the point distance, its
// lower bound over a node, and the open farthest corner as the upper bound.
template <int D>
struct TorusMetric {
  Torus<D> T;
  __device__ __forceinline__ float dist(const float x[D], const float p[D]) const {
    return torus_sq_dist<D>(x, p, T);
  }
  __device__ __forceinline__ float mindist(const float lo[D], const float hi[D],
                                           const float p[D]) const {
    return torus_box_mindist<D>(lo, hi, p, T);
  }
  __device__ __forceinline__ float maxdist(const float lo[D], const float hi[D],
                                           const float p[D]) const {
    return box_maxdist<D>(lo, hi, p);
  }
};

// Torus grouping links through the wave-shared grouping traversal
// (kdt_packet.hip): conn flags nodes whose points are one component already.
template <int D>
kdt_status torus_fof_packet_launch(const TreeView& v, int leaf, float l2, const Torus<D>& T,
                                   int32_t* parent, uint32_t* conn, hipStream_t stream);

// Torus ball counts through the wave-shared count traversal (kdt_packet.hip);
// arguments as range_packet_launch (fill: CSR lists instead of counts).
template <int D>
kdt_status torus_range_packet_launch(const TreeView& v, int leaf, const float* d_q, int64_t nq,
                                     float r2, const Torus<D>& T, const int32_t* order,
                                     int32_t* d_count, uint32_t split_budget,
                                     hipStream_t stream, const FillOut* fill = nullptr);

}  // namespace kdt
