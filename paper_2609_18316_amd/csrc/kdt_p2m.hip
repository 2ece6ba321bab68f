// kdt_p2m.hip -- adaptive SPH particle-to-mesh deposit (Sec. 4.2) and its
// adjoint on gfx950.
//
// Each particle i spreads its mass over the cells whose centres lie within
// H_i = max(h_i, cell) with the M4 cubic spline w(q), q = 2 r / H_i, and the
// weights are normalised over the particle's in-grid cells (S_i), so the
// deposit conserves mass.  Forward: one workgroup takes 256 consecutive
// particles of the visiting order (tree order keeps them spatially compact),
// accumulates their deposits in a float64 LDS tile covering the union of their
// supports and flushes the tile into a float64 mesh with one atomic add per
// touched cell; a last pass rounds the mesh to float32.  Chunks whose union
// box does not fit the tile deposit with global float64 atomics.  Backward:
// one lane per particle gathers S, A = sum g w, B = sum grad w and
// C = sum g grad w (weights recomputed, float64 sums) -- no atomics.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kdt_internal.h"

namespace kdt {

constexpr int kPBlock = 256;
constexpr int kTile = 8192;  // float64 cells in the LDS tile (64 KiB)

struct GridDev {
  float lo[3];
  float cell;
  int32_t n[3];
};

__device__ __forceinline__ float m4_w(float q) {
  if (q < 1.0f) {
    float q2 = q * q;
    return 1.0f - 1.5f * q2 + 0.75f * q2 * q;
  }
  if (q < 2.0f) {
    float u = 2.0f - q;
    return 0.25f * u * u * u;
  }
  return 0.0f;
}

__device__ __forceinline__ float m4_dw(float q) {
  if (q < 1.0f) return -3.0f * q + 2.25f * q * q;
  if (q < 2.0f) {
    float u = 2.0f - q;
    return -0.75f * u * u;
  }
  return 0.0f;
}

// Cell index range [c0, c1] along one axis whose centres lie within H of x.
__device__ __forceinline__ void axis_range(float x, float H, float lo, float cell, int n, int& c0,
                                           int& c1) {
  const float inv = 1.0f / cell;
  int a = (int)ceilf((x - H - lo) * inv - 0.5f);
  int b = (int)floorf((x + H - lo) * inv - 0.5f);
  c0 = max(a, 0);
  c1 = min(b, n - 1);
}

struct Particle {
  float x[3];
  float m;
  float H;
  int c0[3], c1[3];
  bool ok;
};

__device__ __forceinline__ void load_particle(const GridDev& g, const float* __restrict__ x,
                                              const float* __restrict__ m,
                                              const float* __restrict__ h, int64_t i,
                                              Particle& p) {
  p.ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    p.x[a] = x[3 * i + a];
    const float top = g.lo[a] + g.cell * (float)g.n[a];
    p.ok &= (p.x[a] >= g.lo[a]) && (p.x[a] < top);
  }
  p.m = m ? m[i] : 0.0f;
  const float hi = h[i];
  p.ok &= hi >= 0.0f && isfinite(hi);
  p.H = fmaxf(hi, g.cell);
#pragma unroll
  for (int a = 0; a < 3; ++a) axis_range(p.x[a], p.H, g.lo[a], g.cell, g.n[a], p.c0[a], p.c1[a]);
  if (!p.ok) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      p.c0[a] = 0;
      p.c1[a] = -1;
    }
  }
}

// Visits every cell of the particle's support box with (flat index, w, dr, r).
template <typename F>
__device__ __forceinline__ void for_cells(const GridDev& g, const Particle& p, F&& f) {
  const float inv2h = 2.0f / p.H;
  for (int ix = p.c0[0]; ix <= p.c1[0]; ++ix) {
    const float dx = p.x[0] - (g.lo[0] + ((float)ix + 0.5f) * g.cell);
    for (int iy = p.c0[1]; iy <= p.c1[1]; ++iy) {
      const float dy = p.x[1] - (g.lo[1] + ((float)iy + 0.5f) * g.cell);
      const float dxy = dx * dx + dy * dy;
      const int64_t rowb = ((int64_t)ix * g.n[1] + iy) * g.n[2];
      for (int iz = p.c0[2]; iz <= p.c1[2]; ++iz) {
        const float dz = p.x[2] - (g.lo[2] + ((float)iz + 0.5f) * g.cell);
        const float r2 = dxy + dz * dz;
        const float r = sqrtf(r2);
        const float q = r * inv2h;
        if (q < 2.0f) f(rowb + iz, ix, iy, iz, q, dx, dy, dz, r);
      }
    }
  }
}

__global__ void k_zero_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void k_round_f32(const double* __restrict__ a, float* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)a[i];
}

__global__ __launch_bounds__(kPBlock) void k_p2m_fwd(GridDev g, const float* __restrict__ x,
                                                     const float* __restrict__ m,
                                                     const float* __restrict__ h, int64_t n,
                                                     const int32_t* __restrict__ order,
                                                     double* __restrict__ acc,
                                                     int32_t* __restrict__ bad) {
  __shared__ double tile[kTile];
  __shared__ int bmin[3], bmax[3];
  const int64_t t = (int64_t)blockIdx.x * kPBlock + threadIdx.x;
  Particle p;
  const bool live = t < n;
  if (live) {
    const int64_t i = order ? order[t] : t;
    load_particle(g, x, m, h, i, p);
    if (!p.ok) atomicOr(bad, 1);
  } else {
    p.ok = false;
    for (int a = 0; a < 3; ++a) {
      p.c0[a] = 0;
      p.c1[a] = -1;
    }
  }
  if (threadIdx.x < 3) {
    bmin[threadIdx.x] = INT32_MAX;
    bmax[threadIdx.x] = INT32_MIN;
  }
  __syncthreads();
  if (p.ok) {
    for (int a = 0; a < 3; ++a) {
      atomicMin(&bmin[a], p.c0[a]);
      atomicMax(&bmax[a], p.c1[a]);
    }
  }
  __syncthreads();
  const int ex = bmax[0] - bmin[0] + 1, ey = bmax[1] - bmin[1] + 1, ez = bmax[2] - bmin[2] + 1;
  const bool any = bmax[0] >= bmin[0];
  const bool use_tile = any && (int64_t)ex * ey * ez <= kTile;
  if (use_tile) {
    for (int c = threadIdx.x; c < ex * ey * ez; c += kPBlock) tile[c] = 0.0;
    __syncthreads();
  }
  if (p.ok) {
    float S = 0.0f;
    for_cells(g, p, [&](int64_t, int, int, int, float q, float, float, float, float) {
      S += m4_w(q);
    });
    const float f = p.m / S;
    if (use_tile) {
      for_cells(g, p, [&](int64_t, int ix, int iy, int iz, float q, float, float, float, float) {
        const float w = m4_w(q);
        if (w > 0.0f) {
          const int c = ((ix - bmin[0]) * ey + (iy - bmin[1])) * ez + (iz - bmin[2]);
          atomicAdd(&tile[c], (double)(f * w));
        }
      });
    } else {
      for_cells(g, p, [&](int64_t cidx, int, int, int, float q, float, float, float, float) {
        const float w = m4_w(q);
        if (w > 0.0f) unsafeAtomicAdd(acc + cidx, (double)(f * w));
      });
    }
  }
  if (use_tile) {
    __syncthreads();
    for (int c = threadIdx.x; c < ex * ey * ez; c += kPBlock) {
      const double v = tile[c];
      if (v != 0.0) {
        const int iz = c % ez, iy = (c / ez) % ey, ix = c / (ez * ey);
        const int64_t cidx = ((int64_t)(ix + bmin[0]) * g.n[1] + (iy + bmin[1])) * g.n[2] + (iz + bmin[2]);
        unsafeAtomicAdd(acc + cidx, v);
      }
    }
  }
}

__global__ __launch_bounds__(kPBlock) void k_p2m_bwd(GridDev g, const float* __restrict__ x,
                                                     const float* __restrict__ m,
                                                     const float* __restrict__ h, int64_t n,
                                                     const int32_t* __restrict__ order,
                                                     const float* __restrict__ gg,
                                                     float* __restrict__ gm,
                                                     float* __restrict__ gx,
                                                     int32_t* __restrict__ bad) {
  const int64_t t = (int64_t)blockIdx.x * kPBlock + threadIdx.x;
  if (t >= n) return;
  const int64_t i = order ? order[t] : t;
  Particle p;
  load_particle(g, x, m, h, i, p);
  if (!p.ok) {
    atomicOr(bad, 1);
    return;
  }
  const float inv2h = 2.0f / p.H;
  double S = 0.0, A = 0.0, B[3] = {0.0, 0.0, 0.0}, C[3] = {0.0, 0.0, 0.0};
  for_cells(g, p, [&](int64_t cidx, int, int, int, float q, float dx, float dy, float dz, float r) {
    const float w = m4_w(q);
    const double gc = (double)gg[cidx];
    S += (double)w;
    A += gc * (double)w;
    if (r > 0.0f) {
      const float fct = m4_dw(q) * inv2h / r;
      const double bx = (double)(fct * dx), by = (double)(fct * dy), bz = (double)(fct * dz);
      B[0] += bx;
      B[1] += by;
      B[2] += bz;
      C[0] += gc * bx;
      C[1] += gc * by;
      C[2] += gc * bz;
    }
  });
  const double G = A / S;
  if (gm) gm[i] = (float)G;
  if (gx) {
    const double f = (double)p.m / S;
#pragma unroll
    for (int a = 0; a < 3; ++a) gx[3 * i + a] = (float)(f * (C[a] - G * B[a]));
  }
}

static bool grid_ok(const kdt_grid* g) {
  return g && g->cell > 0.0f && std::isfinite(g->cell) && g->n[0] > 0 && g->n[1] > 0 &&
         g->n[2] > 0 && std::isfinite(g->lo[0]) && std::isfinite(g->lo[1]) &&
         std::isfinite(g->lo[2]);
}

static GridDev to_dev(const kdt_grid* g) {
  GridDev d;
  for (int a = 0; a < 3; ++a) {
    d.lo[a] = g->lo[a];
    d.n[a] = g->n[a];
  }
  d.cell = g->cell;
  return d;
}

}  // namespace kdt

using namespace kdt;

static kdt_status finish_bad_check(int32_t* d_bad, hipStream_t stream, const char* who) {
  int32_t bad = 0;
  hipError_t e = hipMemcpyAsync(&bad, d_bad, sizeof(bad), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  (void)hipFreeAsync(d_bad, stream);
  if (e != hipSuccess) {
    kdt_set_error("%s: %s", who, hipGetErrorString(e));
    return KDT_EDEVICE;
  }
  if (bad) {
    kdt_set_error("%s: a particle lies outside the grid or has an invalid smoothing length", who);
    return KDT_EINVAL;
  }
  return KDT_OK;
}

extern "C" kdt_status kdt_p2m(const float* d_x, const float* d_m, const float* d_h, int64_t n,
                              const kdt_grid* grid, const int32_t* d_order, float* d_grid,
                              hipStream_t stream) {
  kdt_clear_error();
  if (!d_x || !d_m || !d_h || !d_grid || n < 0 || !grid_ok(grid)) {
    kdt_set_error("kdt_p2m: NULL pointer, negative n or invalid grid");
    return KDT_EINVAL;
  }
  const int64_t cells = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  double* acc = nullptr;
  int32_t* bad = nullptr;
  if (hipMallocAsync((void**)&acc, sizeof(double) * cells, stream) != hipSuccess ||
      hipMallocAsync((void**)&bad, 256, stream) != hipSuccess) {
    kdt_set_error("kdt_p2m: cannot allocate the float64 accumulation mesh");
    return KDT_ENOMEM;
  }
  const unsigned gc = (unsigned)((cells + 255) / 256);
  k_zero_f64<<<gc, 256, 0, stream>>>(acc, cells);
  k_zero_f64<<<1, 32, 0, stream>>>(reinterpret_cast<double*>(bad), 1);
  if (n > 0)
    k_p2m_fwd<<<(unsigned)((n + kPBlock - 1) / kPBlock), kPBlock, 0, stream>>>(
        to_dev(grid), d_x, d_m, d_h, n, d_order, acc, bad);
  k_round_f32<<<gc, 256, 0, stream>>>(acc, d_grid, cells);
  (void)hipFreeAsync(acc, stream);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_p2m: kernel launch failed");
    return KDT_EDEVICE;
  }
  return finish_bad_check(bad, stream, "kdt_p2m");
}

extern "C" kdt_status kdt_p2m_backward(const float* d_x, const float* d_m, const float* d_h,
                                       int64_t n, const kdt_grid* grid, const int32_t* d_order,
                                       const float* d_ggrid, float* d_gm, float* d_gx,
                                       hipStream_t stream) {
  kdt_clear_error();
  if (!d_x || !d_m || !d_h || !d_ggrid || n < 0 || !grid_ok(grid)) {
    kdt_set_error("kdt_p2m_backward: NULL pointer, negative n or invalid grid");
    return KDT_EINVAL;
  }
  int32_t* bad = nullptr;
  if (hipMallocAsync((void**)&bad, 256, stream) != hipSuccess) {
    kdt_set_error("kdt_p2m_backward: allocation failed");
    return KDT_ENOMEM;
  }
  k_zero_f64<<<1, 32, 0, stream>>>(reinterpret_cast<double*>(bad), 1);
  if (n > 0 && (d_gm || d_gx))
    k_p2m_bwd<<<(unsigned)((n + kPBlock - 1) / kPBlock), kPBlock, 0, stream>>>(
        to_dev(grid), d_x, d_m, d_h, n, d_order, d_ggrid, d_gm, d_gx, bad);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("kdt_p2m_backward: kernel launch failed");
    return KDT_EDEVICE;
  }
  return finish_bad_check(bad, stream, "kdt_p2m_backward");
}
