// kdt_p2m.hip -- adaptive SPH particle-to-mesh deposit (Sec. 4.2) and its
// adjoint on gfx950.
//
// Each particle i spreads its mass over the cells whose centres lie within
// H_i = max(h_i, cell) with the M4 cubic spline w(q), q = 2 r / H_i, and the
// weights are normalised over the particle's in-grid cells (S_i), so the
// deposit conserves mass.
//
// On a periodic mesh (the periodic boundaries of Sec. 2.4 applied to the
// mesh) the box is a 3-torus of periods n_a * cell and a cell is reached the
// shorter way round.  Every H_i is below half of every period, so along each
// axis a support crosses at most one face: the particle is deposited as up
// to 8 images (itself, one period away along any subset of the axes whose
// face its support crosses), each clipped to the mesh like a particle of an
// open mesh.  An image keeps the particle's own coordinates and moves the
// cells instead: cell s of the image is measured from the centre of cell
// s + off (off = -n or +n cells), so no rounding of x + L enters the
// distances.  S_i sums over all images, so no support is dropped.
//
// Forward, as a binned deposit into LDS tiles of 16^3 cells:
//  1. one lane per particle (in visiting order) gathers it from the caller's
//     arrays, stores it packed for the later passes (x, y, z, h as one
//     float4), sums S_i over its support, keeps m_i / S_i and counts, per
//     tile, the particles whose support box overlaps it (wave-aggregated
//     atomics: the lanes of a wave hold nearby particles); the later passes
//     stream the packed copy instead of gathering again.  The tree entry
//     points read the positions from a tree's records and m, h in tree
//     order, so every pass streams contiguous arrays;
//  2. the host reads the per-tile counts, lays out the (tile, particle) lists
//     and cuts them into chunks of at most kChunk particles;
//  3. the particles are scattered into their tiles' lists;
//  4. one workgroup per chunk accumulates its particles' deposits inside its
//     tile in a float64 LDS tile and writes the tile out once: rounded to
//     float32 straight into the mesh when the tile is a single chunk, else as
//     a float64 partial;
//  5. tiles cut into several chunks sum their partials in chunk order.
// Every mesh cell is written exactly once and no global atomics touch the
// mesh.  Backward: one lane per particle gathers S, A = sum g w,
// B = sum grad w and C = sum g grad w (weights recomputed, float64 sums) --
// no atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "kdt_internal.h"

namespace kdt {

constexpr int kPBlock = 256;
constexpr int kT = 16;                      // tile edge in cells
constexpr int kTileCells = kT * kT * kT;    // float64 LDS tile: 32 KiB
constexpr int64_t kChunk = 4096;            // particles per deposit work item

// Scratch slots the deposit keeps on its stream between calls.
enum : int {
  kSlotParticles = 100,
  kSlotLists = 101,
  kSlotPartial = 102,
  kSlotFlag = 103,
  kSlotOrder = 104
};
// Calls without a particle order and at least this many particles order
// them by home tile first.
constexpr int64_t kSelfOrderMin = 1 << 16;

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct GridDev {
  float lo[3];
  float cell;
  int32_t n[3];
  int32_t periodic;  // 1: the mesh box is a 3-torus of periods n[a] * cell
  float L[3];        // the periods n[a] * cell
};

// Deposit schemes: the adaptive SPH kernel (M4, Sec. 4.2) and the fixed
// clouds the paper compares it with (Table 3; after Hockney and Eastwood):
// NGP, CIC and TSC spread a particle over 1, 2 and 3 cells per axis.
enum : int { kSph = 0, kNgp = 1, kCic = 2, kTsc = 3 };

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

// One image of a particle: its position, H, the cell offset of the image
// (cell s is measured from the centre of cell s + off; 0 for the particle
// itself) and its support's cell range clipped to the mesh (c0 > c1 on some
// axis: no cell).
struct Particle {
  float x[3];
  float m;
  float H;
  int off[3];
  int c0[3], c1[3];
  bool ok;
};

// A particle as the gather pass stores it: x, y, z, h.
__device__ __forceinline__ float4 load_packed(const float4* __restrict__ P, int64_t t) {
  return P[t];
}

// Position i of the caller's [n][3] array (XS = 3) or of a 3-d tree's
// records [n][4] (XS = 4: x, y, z and the point's index).
template <int XS>
__device__ __forceinline__ void load_position(const float* __restrict__ x, int64_t i, float p[3]) {
  if constexpr (XS == 4) {
    const float4 r = reinterpret_cast<const float4*>(x)[i];
    p[0] = r.x, p[1] = r.y, p[2] = r.z;
  } else {
    p[0] = x[3 * i], p[1] = x[3 * i + 1], p[2] = x[3 * i + 2];
  }
}

// Validity of a particle: inside the mesh box; for the adaptive kernel also
// h finite and >= 0, and on a periodic mesh H below half of every period.
template <int SCH = kSph>
__device__ __forceinline__ bool particle_ok(const GridDev& g, const float x[3], float h) {
  bool ok = SCH != kSph || (h >= 0.0f && isfinite(h));
  const float H = fmaxf(h, g.cell);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float top = g.lo[a] + g.L[a];
    ok &= (x[a] >= g.lo[a]) && (x[a] < top);
    if (SCH == kSph && g.periodic) ok &= 2.0f * H < g.L[a];
  }
  return ok;
}

// Per axis, the unclipped cell range [lo_c, hi_c] the particle can reach, and
// the one period offset whose image can reach cells (none if the support
// crosses no face).  For the fixed clouds also the stencil: cell base + j
// has weight cw[a][j] along axis a.
struct Images {
  int lo_c[3], hi_c[3];  // unclipped cell range of the support
  int off[3];            // cell offset of the axis's image: -n, +n, or 0
  int mask;              // bit a: axis a has an image; images = subsets of mask
  float cw[3][3];        // fixed clouds: per-axis weights from lo_c
};

template <int SCH>
__device__ __forceinline__ Images images_of(const GridDev& g, const float x[3], float H) {
  Images im;
  im.mask = 0;
  const float inv = 1.0f / g.cell;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if constexpr (SCH == kSph) {
      im.lo_c[a] = (int)ceilf((x[a] - H - g.lo[a]) * inv - 0.5f);
      im.hi_c[a] = (int)floorf((x[a] + H - g.lo[a]) * inv - 0.5f);
    } else if constexpr (SCH == kNgp) {
      // the cell holding the particle (decided in float32, as the oracle does)
      im.lo_c[a] = im.hi_c[a] = (int)floorf((x[a] - g.lo[a]) / g.cell);
      im.cw[a][0] = 1.0f;
    } else if constexpr (SCH == kCic) {
      const float sc = (x[a] - g.lo[a]) * inv - 0.5f;  // in cells from the first centre
      const float i0 = floorf(sc), f = sc - i0;
      im.lo_c[a] = (int)i0;
      im.hi_c[a] = im.lo_c[a] + 1;
      im.cw[a][0] = 1.0f - f;
      im.cw[a][1] = f;
    } else {
      const float sc = (x[a] - g.lo[a]) * inv - 0.5f;
      const float c = floorf(sc + 0.5f), u = sc - c;  // nearest centre, offset in [-1/2, 1/2)
      im.lo_c[a] = (int)c - 1;
      im.hi_c[a] = im.lo_c[a] + 2;
      im.cw[a][0] = 0.5f * (0.5f - u) * (0.5f - u);
      im.cw[a][1] = 0.75f - u * u;
      im.cw[a][2] = 0.5f * (0.5f + u) * (0.5f + u);
    }
    im.off[a] = 0;
    if (!g.periodic) continue;
    if (im.lo_c[a] < 0) {
      im.off[a] = -g.n[a];  // cells below the low face, stored one period up
      im.mask |= 1 << a;
    } else if (im.hi_c[a] > g.n[a] - 1) {
      im.off[a] = g.n[a];   // cells above the high face, stored one period down
      im.mask |= 1 << a;
    }
  }
  return im;
}

// Image `img` (a subset of im.mask) of the particle at x with smoothing
// length h: offsets and the clipped cell range (on an open mesh, image 0:
// the cells whose centres can lie within H, clipped to the mesh).
__device__ __forceinline__ void make_image(const GridDev& g, const float x[3], float h, float m,
                                           bool ok, const Images& im, int img, Particle& p) {
  p.ok = ok;
  p.m = m;
  p.H = fmaxf(h, g.cell);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    p.x[a] = x[a];
    p.off[a] = (img >> a) & 1 ? im.off[a] : 0;
    p.c0[a] = max(im.lo_c[a] - p.off[a], 0);
    p.c1[a] = min(im.hi_c[a] - p.off[a], g.n[a] - 1);
  }
  if (!p.ok) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      p.c0[a] = 0;
      p.c1[a] = -1;
    }
  }
}

// Calls f(Particle&, img) for every image of a particle (one on an open
// mesh or for a support that crosses no face).
template <typename F>
__device__ __forceinline__ void for_images(const GridDev& g, const float x[3], float h, float m,
                                           bool ok, F&& f) {
  const Images im = images_of<kSph>(g, x, fmaxf(h, g.cell));
  for (int img = 0; img < 8; ++img) {
    if ((img & ~im.mask) != 0) continue;
    Particle p;
    make_image(g, x, h, m, ok, im, img, p);
    f(p, img);
  }
}

// Visits every cell of the box [b0, b1] (a part of the particle's support
// box) whose centre lies within the support, with (flat index, ix, iy, iz, q,
// dx, dy, dz, r).  The same float operations for every cell, whichever part
// of the support box is visited, so a cell's weight does not depend on it.
//
// Rows are clipped to the support sphere before the exact test: a z-row is
// walked only over the cells within a chord of half-length
// sqrt(H^2 (1 + 2e-4) - dx^2 - dy^2) + 1e-3 cell, a margin far above the
// float rounding of q, so every cell with q < 2 is still visited (and the
// test q < 2 decides, as before); rows and planes farther than H are skipped.
template <typename F>
__device__ __forceinline__ void for_cells_in(const GridDev& g, const Particle& p, const int b0[3],
                                             const int b1[3], F&& f) {
  const float inv2h = 2.0f / p.H;
  const float H2 = p.H * p.H * 1.0002f;
  const float inv = 1.0f / g.cell;
  for (int ix = b0[0]; ix <= b1[0]; ++ix) {
    const float dx = p.x[0] - (g.lo[0] + ((float)(ix + p.off[0]) + 0.5f) * g.cell);
    if (dx * dx > H2) continue;
    for (int iy = b0[1]; iy <= b1[1]; ++iy) {
      const float dy = p.x[1] - (g.lo[1] + ((float)(iy + p.off[1]) + 0.5f) * g.cell);
      const float dxy = dx * dx + dy * dy;
      if (dxy > H2) continue;
      const float zr = sqrtf(H2 - dxy) + 1e-3f * g.cell;
      const int z0 = max(b0[2], (int)ceilf((p.x[2] - zr - g.lo[2]) * inv - 0.5f) - p.off[2]);
      const int z1 = min(b1[2], (int)floorf((p.x[2] + zr - g.lo[2]) * inv - 0.5f) - p.off[2]);
      const int64_t rowb = ((int64_t)ix * g.n[1] + iy) * g.n[2];
      for (int iz = z0; iz <= z1; ++iz) {
        const float dz = p.x[2] - (g.lo[2] + ((float)(iz + p.off[2]) + 0.5f) * g.cell);
        const float r2 = dxy + dz * dz;
        const float r = sqrtf(r2);
        const float q = r * inv2h;
        if (q < 2.0f) f(rowb + iz, ix, iy, iz, q, dx, dy, dz, r);
      }
    }
  }
}

template <typename F>
__device__ __forceinline__ void for_cells(const GridDev& g, const Particle& p, F&& f) {
  for_cells_in(g, p, p.c0, p.c1, f);
}

// Visits the cells of [b0, b1] that an image reaches with (flat index, ix,
// iy, iz, weight): the M4 profile w(q) for the adaptive kernel, the product
// of the per-axis stencil weights for the fixed clouds.
template <int SCH, typename F>
__device__ __forceinline__ void for_weights(const GridDev& g, const Particle& p, const Images& im,
                                            const int b0[3], const int b1[3], F&& f) {
  if constexpr (SCH == kSph) {
    for_cells_in(g, p, b0, b1, [&](int64_t c, int ix, int iy, int iz, float q, float, float,
                                   float, float) { f(c, ix, iy, iz, m4_w(q)); });
  } else {
    for (int ix = b0[0]; ix <= b1[0]; ++ix) {
      const float wx = im.cw[0][ix + p.off[0] - im.lo_c[0]];
      for (int iy = b0[1]; iy <= b1[1]; ++iy) {
        const float wxy = wx * im.cw[1][iy + p.off[1] - im.lo_c[1]];
        const int64_t rowb = ((int64_t)ix * g.n[1] + iy) * g.n[2];
        for (int iz = b0[2]; iz <= b1[2]; ++iz)
          f(rowb + iz, ix, iy, iz, wxy * im.cw[2][iz + p.off[2] - im.lo_c[2]]);
      }
    }
  }
}

__global__ void k_zero_f64(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}


struct TileGrid {
  int nt[3];  // tiles per axis
};

// Next tile of a lane's support box in x-major order; false past the last.
__device__ __forceinline__ bool next_tile(int c[3], const int t0[3], const int t1[3]) {
  if (++c[2] <= t1[2]) return true;
  c[2] = t0[2];
  if (++c[1] <= t1[1]) return true;
  c[1] = t0[1];
  return ++c[0] <= t1[0];
}

// Walks every lane's list of overlapped tiles in step: each round takes the
// current tile of the first unfinished lane and hands it, with the set of
// lanes currently at that tile, to `f` (called by the whole wave; the
// leader is the lowest such lane), then moves those lanes on.  Lanes of a
// wave hold nearby particles, so a wave needs few rounds.
template <typename F>
__device__ __forceinline__ void for_tiles_aggregated(const TileGrid& tg, const int t0[3],
                                                     const int t1[3], bool has, F&& f) {
  int c[3] = {t0[0], t0[1], t0[2]};
  bool more = has;
  for (;;) {
    const uint64_t act = __ballot(more);
    if (act == 0) break;
    const int tile = more ? (c[0] * tg.nt[1] + c[1]) * tg.nt[2] + c[2] : -1;
    const int leader = __ffsll((unsigned long long)act) - 1;
    const int lt = __shfl(tile, leader);
    const bool mine = more && tile == lt;
    const uint64_t same = __ballot(mine);
    f(lt, same, leader, mine);
    if (mine) more = next_tile(c, t0, t1);
  }
}

// Tiles overlapped by one image's support box; false (no tiles) for an
// invalid particle or an empty box.  The prep and scatter passes decide this
// identically, so the lists hold exactly the counted entries.
__device__ __forceinline__ bool tile_range(const Particle& p, int t0[3], int t1[3]) {
  bool has = p.ok;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    has &= p.c0[a] <= p.c1[a];
    t0[a] = p.c0[a] / kT;
    t1[a] = p.c1[a] / kT;
  }
  return has;
}

// Step 1: per particle (visiting position t): gathered from the caller's
// arrays (positions with XS floats per row) and stored packed,
// P[t] = (x, y, z, h); f = m / S over all its images; the per-tile entry
// counts (one per image and overlapped tile); the validity flag for a
// particle outside the box or with an invalid h, or for a tree whose
// deferred finiteness check failed (tree_bad).  The gather's scattered
// reads, if any, overlap the support sums.
template <int SCH, int XS>
__global__ __launch_bounds__(kPBlock) void k_p2m_prep(GridDev g, TileGrid tg,
                                                      const float* __restrict__ xin,
                                                      const float* __restrict__ min_,
                                                      const float* __restrict__ hin, int64_t n,
                                                      const int32_t* __restrict__ order,
                                                      const int32_t* __restrict__ tree_bad,
                                                      float4* __restrict__ P,
                                                      float* __restrict__ fbuf,
                                                      uint32_t* __restrict__ tcount,
                                                      int32_t* __restrict__ bad) {
  const int64_t t = xcd_block<kXcdRunP2M>() * kPBlock + threadIdx.x;
  float x[3] = {0.0f, 0.0f, 0.0f}, h = 0.0f, m = 0.0f;
  bool ok = false;
  if (t == 0 && tree_bad && *tree_bad) atomicOr(bad, 1);
  if (t < n) {
    const int64_t i = order ? order[t] : t;
    load_position<XS>(xin, i, x);
    h = hin ? hin[i] : 0.0f;
    m = min_[i];
    P[t] = make_float4(x[0], x[1], x[2], h);
    ok = particle_ok<SCH>(g, x, h);
    if (!ok) atomicOr(bad, 1);
  }
  // S in float64: a support of 10^5 cells (H near half the mesh) would
  // drift by 1e-5 in float32
  double S = 0.0;
  const Images im = images_of<SCH>(g, x, fmaxf(h, g.cell));
  // every lane walks the same image numbers (8 at most), so the tile
  // aggregation below runs with the whole wave
  for (int img = 0; img < 8; ++img) {
    const bool mine = t < n && (img & ~im.mask) == 0;
    if (!__any(mine)) continue;
    Particle p;
    make_image(g, x, h, m, ok && mine, im, img, p);
    int t0[3] = {0, 0, 0}, t1[3] = {-1, -1, -1};
    bool has = false;
    if (mine) {
      for_weights<SCH>(g, p, im, p.c0, p.c1,
                       [&](int64_t, int, int, int, float w) { S += (double)w; });
      has = tile_range(p, t0, t1);
    }
    for_tiles_aggregated(tg, t0, t1, has, [&](int tile, uint64_t same, int leader, bool) {
      if (lane_id() == leader) atomicAdd(tcount + tile, (uint32_t)__popcll(same));
    });
  }
  // a particle inside the mesh has its own cell centre within
  // sqrt(3)/2 cell <= H, so S > 0
  if (t < n) fbuf[t] = ok ? (float)((double)m / S) : 0.0f;
}

// The key of the self-ordering of an unordered call: the tile of the cell
// that holds each particle (wrapped on a periodic mesh); a particle outside
// the mesh of an open grid, or with a non-finite coordinate, gets the key
// n_tiles.  Only the speed depends on this order, never the deposit.
__global__ void k_p2m_tilekey(GridDev g, TileGrid tg, const float* __restrict__ x, int64_t n,
                              uint32_t n_tiles, uint32_t* __restrict__ keys,
                              int32_t* __restrict__ vals) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  int c[3];
  bool in = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float s = floorf((x[3 * t + a] - g.lo[a]) / g.cell);
    if (g.periodic && s == s) s -= floorf(s / (float)g.n[a]) * (float)g.n[a];
    in &= s >= 0.0f && s < (float)g.n[a];
    c[a] = in ? (int)s : 0;
  }
  keys[t] = in ? (uint32_t)(((c[0] / kT) * tg.nt[1] + c[1] / kT) * tg.nt[2] + c[2] / kT) : n_tiles;
  vals[t] = (int32_t)t;
}

// Step 3: every image appends its entry (visiting position, and on a
// periodic mesh the image in the low three bits) to the lists of the tiles
// its support box overlaps.
template <int SCH>
__global__ __launch_bounds__(kPBlock) void k_p2m_scatter(GridDev g, TileGrid tg,
                                                         const float4* __restrict__ P, int64_t n,
                                                         const int64_t* __restrict__ toff,
                                                         uint32_t* __restrict__ tfill,
                                                         int32_t* __restrict__ pairs) {
  const int64_t t = xcd_block<kXcdRunP2M>() * kPBlock + threadIdx.x;
  float x[3] = {0.0f, 0.0f, 0.0f}, h = 0.0f;
  bool ok = false;
  if (t < n) {
    const float4 v = load_packed(P, t);
    x[0] = v.x, x[1] = v.y, x[2] = v.z, h = v.w;
    ok = particle_ok<SCH>(g, x, h);
  }
  const Images im = images_of<SCH>(g, x, fmaxf(h, g.cell));
  for (int img = 0; img < 8; ++img) {
    const bool mine = t < n && (img & ~im.mask) == 0;
    if (!__any(mine)) continue;
    Particle p;
    make_image(g, x, h, 0.0f, ok && mine, im, img, p);
    int t0[3] = {0, 0, 0}, t1[3] = {-1, -1, -1};
    const bool has = mine && tile_range(p, t0, t1);
    const int32_t code = g.periodic ? (int32_t)(t * 8 + img) : (int32_t)t;
    for_tiles_aggregated(tg, t0, t1, has, [&](int tile, uint64_t same, int leader, bool on) {
      uint32_t base = 0;
      if (lane_id() == leader) base = atomicAdd(tfill + tile, (uint32_t)__popcll(same));
      base = (uint32_t)__shfl((int)base, leader);
      const int64_t at = toff[tile] + base + lanes_below(same);
      if (on && at < toff[tile + 1]) pairs[at] = code;
    });
  }
}

struct DepositChunk {
  int32_t tile;
  int32_t slot;  // -1: the tile's only chunk, written to the mesh; else its partial
  int64_t begin, end;
};

// Step 4: one workgroup per chunk of one tile's entry list.
template <int SCH>
__global__ __launch_bounds__(kPBlock) void k_p2m_tile(GridDev g, TileGrid tg,
                                                      const float4* __restrict__ P, int64_t n,
                                                      const float* __restrict__ fbuf,
                                                      const int32_t* __restrict__ pairs,
                                                      const DepositChunk* __restrict__ chunks,
                                                      float* __restrict__ mesh,
                                                      double* __restrict__ partial) {
  __shared__ double tile[kTileCells];
  const DepositChunk ck = chunks[blockIdx.x];
  const int tz = ck.tile % tg.nt[2], ty = (ck.tile / tg.nt[2]) % tg.nt[1],
            tx = ck.tile / (tg.nt[2] * tg.nt[1]);
  const int lo[3] = {tx * kT, ty * kT, tz * kT};
  const int hi[3] = {min(lo[0] + kT, g.n[0]) - 1, min(lo[1] + kT, g.n[1]) - 1,
                     min(lo[2] + kT, g.n[2]) - 1};
  for (int c = threadIdx.x; c < kTileCells; c += kPBlock) tile[c] = 0.0;
  __syncthreads();
  for (int64_t e = ck.begin + threadIdx.x; e < ck.end; e += kPBlock) {
    const int32_t code = pairs[e];
    const int64_t t = g.periodic ? (int64_t)((uint32_t)code >> 3) : (int64_t)code;
    const int img = g.periodic ? (code & 7) : 0;
    if ((uint64_t)t >= (uint64_t)n) continue;
    const float4 v = load_packed(P, t);
    const float x[3] = {v.x, v.y, v.z};
    const Images im = images_of<SCH>(g, x, fmaxf(v.w, g.cell));
    Particle p;
    make_image(g, x, v.w, 0.0f, true, im, img, p);
    const float f = fbuf[t];
    int b0[3], b1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      b0[a] = max(p.c0[a], lo[a]);
      b1[a] = min(p.c1[a], hi[a]);
    }
    for_weights<SCH>(g, p, im, b0, b1, [&](int64_t, int ix, int iy, int iz, float w) {
      if (w > 0.0f)
        atomicAdd(&tile[((ix - lo[0]) * kT + (iy - lo[1])) * kT + (iz - lo[2])], (double)(f * w));
    });
  }
  __syncthreads();
  for (int c = threadIdx.x; c < kTileCells; c += kPBlock) {
    const int lz = c % kT, ly = (c / kT) % kT, lx = c / (kT * kT);
    if (ck.slot >= 0) {
      partial[(int64_t)ck.slot * kTileCells + c] = tile[c];
    } else if (lo[0] + lx <= hi[0] && lo[1] + ly <= hi[1] && lo[2] + lz <= hi[2]) {
      mesh[((int64_t)(lo[0] + lx) * g.n[1] + (lo[1] + ly)) * g.n[2] + (lo[2] + lz)] = (float)tile[c];
    }
  }
}

struct SplitTile {
  int32_t tile;
  int32_t first_slot, n_slots;
};

// Step 5: tiles cut into several chunks add their partials in chunk order.
// Grid (split tiles, kTileCells / kPBlock): one thread per cell.
__global__ __launch_bounds__(kPBlock) void k_p2m_reduce(GridDev g, TileGrid tg,
                                                        const SplitTile* __restrict__ split,
                                                        const double* __restrict__ partial,
                                                        float* __restrict__ mesh) {
  const SplitTile st = split[blockIdx.x];
  const int tz = st.tile % tg.nt[2], ty = (st.tile / tg.nt[2]) % tg.nt[1],
            tx = st.tile / (tg.nt[2] * tg.nt[1]);
  const int c = blockIdx.y * kPBlock + threadIdx.x;
  const int lz = c % kT, ly = (c / kT) % kT, lx = c / (kT * kT);
  const int ix = tx * kT + lx, iy = ty * kT + ly, iz = tz * kT + lz;
  if (ix >= g.n[0] || iy >= g.n[1] || iz >= g.n[2]) return;
  const double* src = partial + (int64_t)st.first_slot * kTileCells + c;
  double v = 0.0;
  for (int s = 0; s < st.n_slots; ++s) v += src[(int64_t)s * kTileCells];
  mesh[((int64_t)ix * g.n[1] + iy) * g.n[2] + iz] = (float)v;
}

// The adjoint: one lane per particle (visiting position t, row order[t] or
// t of every per-particle array; positions with XS floats per row).
template <int XS>
__global__ __launch_bounds__(kPBlock) void k_p2m_bwd(GridDev g, const float* __restrict__ x,
                                                     const float* __restrict__ m,
                                                     const float* __restrict__ h, int64_t n,
                                                     const int32_t* __restrict__ order,
                                                     const int32_t* __restrict__ tree_bad,
                                                     const float* __restrict__ gg,
                                                     float* __restrict__ gm,
                                                     float* __restrict__ gx,
                                                     int32_t* __restrict__ bad) {
  const int64_t t = xcd_block<kXcdRunP2M>() * kPBlock + threadIdx.x;
  if (t == 0 && tree_bad && *tree_bad) atomicOr(bad, 1);
  if (t >= n) return;
  const int64_t i = order ? order[t] : t;
  float xi[3];
  load_position<XS>(x, i, xi);
  const float hi = h[i], mi = m[i];
  if (!particle_ok(g, xi, hi)) {
    atomicOr(bad, 1);
    return;
  }
  const float inv2h = 2.0f / fmaxf(hi, g.cell);
  double S = 0.0, A = 0.0, B[3] = {0.0, 0.0, 0.0}, C[3] = {0.0, 0.0, 0.0};
  for_images(g, xi, hi, mi, true, [&](const Particle& p, int) {
    for_cells(g, p, [&](int64_t cidx, int, int, int, float q, float dx, float dy, float dz,
                        float r) {
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
  });
  const double G = A / S;
  if (gm) gm[i] = (float)G;
  if (gx) {
    const double f = (double)mi / S;
#pragma unroll
    for (int a = 0; a < 3; ++a) gx[3 * i + a] = (float)(f * (C[a] - G * B[a]));
  }
}

static bool grid_ok(const kdt_grid* g) {
  return g && g->cell > 0.0f && std::isfinite(g->cell) && g->n[0] > 0 && g->n[1] > 0 &&
         g->n[2] > 0 && std::isfinite(g->lo[0]) && std::isfinite(g->lo[1]) &&
         std::isfinite(g->lo[2]) && (g->periodic == 0 || g->periodic == 1);
}

static GridDev to_dev(const kdt_grid* g) {
  GridDev d;
  for (int a = 0; a < 3; ++a) {
    d.lo[a] = g->lo[a];
    d.n[a] = g->n[a];
    d.L[a] = g->cell * (float)g->n[a];
  }
  d.cell = g->cell;
  d.periodic = g->periodic;
  return d;
}

}  // namespace kdt

using namespace kdt;

// Reads the device-side validity flag back, waits for the stream and
// reports the flag.
static kdt_status read_bad_flag(const int32_t* d_bad, hipStream_t stream, const char* who,
                                bool tree) {
  int32_t bad = 0;
  hipError_t e = hipMemcpyAsync(&bad, d_bad, sizeof(bad), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    kdt_set_error("%s: %s", who, hipGetErrorString(e));
    return KDT_EDEVICE;
  }
  if (bad) {
    kdt_set_error("%s: a particle lies outside the grid or has an invalid smoothing length "
                  "(on a periodic mesh H must stay below half of every period)%s", who,
                  tree ? ", or the tree's points hold a non-finite coordinate" : "");
    return KDT_EINVAL;
  }
  return KDT_OK;
}

namespace {

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

namespace {
// Calls f with the scheme as a compile-time constant.
template <typename F>
void by_scheme(int sch, F&& f) {
  switch (sch) {
    case kNgp: f(std::integral_constant<int, kNgp>()); break;
    case kCic: f(std::integral_constant<int, kCic>()); break;
    case kTsc: f(std::integral_constant<int, kTsc>()); break;
    default: f(std::integral_constant<int, kSph>()); break;
  }
}
}  // namespace

// An unordered call's particles in home-tile order (k_p2m_tilekey, then the
// library's radix sort), so that a wave's particles share their tiles: the
// per-tile counters are then updated once per wave, not once per lane.  The
// order lives in the stream's scratch (slot kSlotOrder).
static kdt_status self_order(const GridDev& g, const int32_t gn[3], const float* d_x, int64_t n,
                             hipStream_t stream, const char* who, const int32_t** order) {
  TileGrid tg;
  int64_t n_tiles = 1;
  for (int a = 0; a < 3; ++a) {
    tg.nt[a] = (gn[a] + kT - 1) / kT;
    n_tiles *= tg.nt[a];
  }
  int bits = 1;
  while (bits < 31 && (int64_t(1) << bits) <= n_tiles) ++bits;
  const size_t a4 = align256(sizeof(uint32_t) * (size_t)n);
  char* s = static_cast<char*>(
      stream_scratch(stream, kSlotOrder, 4 * a4 + radix_sort_scratch_bytes(n)));
  if (!s) {
    kdt_set_error("%s: device allocation failed for the particle order", who);
    return KDT_ENOMEM;
  }
  uint32_t* keys[2] = {reinterpret_cast<uint32_t*>(s), reinterpret_cast<uint32_t*>(s + a4)};
  int32_t* vals[2] = {reinterpret_cast<int32_t*>(s + 2 * a4),
                      reinterpret_cast<int32_t*>(s + 3 * a4)};
  k_p2m_tilekey<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(g, tg, d_x, n,
                                                                 (uint32_t)n_tiles, keys[0],
                                                                 vals[0]);
  const int cur = radix_sort_pairs(keys, vals, n, 0, bits, s + 4 * a4, stream);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("%s: ordering the particles failed", who);
    return KDT_EDEVICE;
  }
  *order = vals[cur];
  return KDT_OK;
}

// Where a deposit's particles come from: the caller's arrays (positions
// [n][3]; row order[t], or t, of every array for visiting position t), or a
// 3-d tree's records [n][4] with m and h in tree order (xs = 4, no order).
struct Source {
  const float* x;
  const float* m;
  const float* h;             // NULL for the fixed clouds
  const int32_t* order;
  int xs;                     // floats per position row: 3 or 4
  const int32_t* tree_bad;    // the tree's deferred finiteness flag, or NULL
  bool may_self_order;        // an unordered call of the caller's arrays
};

// The binned deposit of either scheme; `who` names the entry point in
// messages.
static kdt_status p2m_forward(int sch, const char* who, Source src, int64_t n,
                              const kdt_grid* grid, float* d_grid, hipStream_t stream) {
  if (!d_grid || n < 0 || !grid_ok(grid) ||
      (n > 0 && (!src.x || !src.m || (sch == kSph && !src.h)))) {
    kdt_set_error("%s: NULL pointer, negative n or invalid grid", who);
    return KDT_EINVAL;
  }
  if (n > INT32_MAX || (grid->periodic && n >= (int64_t(1) << 28))) {
    kdt_set_error("%s: n = %lld above %s", who, (long long)n,
                  grid->periodic ? "2^28 - 1 (periodic mesh)" : "2^31 - 1");
    return KDT_EUNSUPPORTED;
  }
  const GridDev g = to_dev(grid);
  TileGrid tg;
  int64_t n_tiles = 1;
  for (int a = 0; a < 3; ++a) {
    tg.nt[a] = (grid->n[a] + kT - 1) / kT;
    n_tiles *= tg.nt[a];
  }
  if (n_tiles > INT32_MAX / 2) {
    kdt_set_error("%s: mesh too large (%lld tiles of %d^3 cells)", who, (long long)n_tiles, kT);
    return KDT_EUNSUPPORTED;
  }
  if (src.may_self_order && !src.order && n >= kSelfOrderMin) {
    const kdt_status st = self_order(g, grid->n, src.x, n, stream, who, &src.order);
    if (st != KDT_OK) return st;
  }
  // scratch kept on the stream between calls: the packed particles, m / S
  // and the tile counters (+ the validity flag) in one slot; the lists and
  // chunk tables in a second; float64 partial tiles in a third
  const size_t a_p = align256(sizeof(float4) * (size_t)n);
  const size_t a_n = align256(sizeof(float) * (size_t)n);
  const size_t a_t = align256(sizeof(uint32_t) * ((size_t)n_tiles + 64));
  char* s0 = static_cast<char*>(stream_scratch(stream, kSlotParticles, a_p + a_n + a_t));
  if (!s0) {
    kdt_set_error("%s: device allocation failed", who);
    return KDT_ENOMEM;
  }
  float4* P = reinterpret_cast<float4*>(s0);
  float* fbuf = reinterpret_cast<float*>(s0 + a_p);
  uint32_t* tcount = reinterpret_cast<uint32_t*>(s0 + a_p + a_n);
  int32_t* bad = reinterpret_cast<int32_t*>(tcount + n_tiles);
  const unsigned gt = (unsigned)((n_tiles + 64 + 255) / 256);
  k_fill_u32<<<gt, 256, 0, stream>>>(tcount, n_tiles + 64, 0u);
  const unsigned gp = (unsigned)((n + kPBlock - 1) / kPBlock);
  if (n > 0)
    by_scheme(sch, [&](auto c) {
      constexpr int S = decltype(c)::value;
      if (src.xs == 4)
        k_p2m_prep<S, 4><<<gp, kPBlock, 0, stream>>>(g, tg, src.x, src.m, src.h, n, src.order,
                                                     src.tree_bad, P, fbuf, tcount, bad);
      else
        k_p2m_prep<S, 3><<<gp, kPBlock, 0, stream>>>(g, tg, src.x, src.m, src.h, n, src.order,
                                                     src.tree_bad, P, fbuf, tcount, bad);
    });
  // the per-tile counts size the lists: read them back (with the check flag)
  std::vector<uint32_t> cnt((size_t)n_tiles + 1);
  hipError_t e = hipMemcpyAsync(cnt.data(), tcount, sizeof(uint32_t) * (n_tiles + 1),
                                hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    kdt_set_error("%s: %s", who, hipGetErrorString(e));
    return KDT_EDEVICE;
  }
  if (cnt[n_tiles] != 0) {
    kdt_set_error("%s: a particle lies outside the grid or has an invalid smoothing "
                  "length (on a periodic mesh H must stay below half of every period)%s", who,
                  src.tree_bad ? ", or the tree's points hold a non-finite coordinate" : "");
    return KDT_EINVAL;
  }
  // lay out the lists and cut them into chunks; tiles of several chunks get
  // consecutive partial slots (the chunk grows if the partials would pass 1 GiB)
  std::vector<int64_t> toff((size_t)n_tiles + 1);
  int64_t total = 0;
  for (int64_t t = 0; t < n_tiles; ++t) {
    toff[t] = total;
    total += cnt[t];
  }
  toff[n_tiles] = total;
  int64_t chunk = kChunk;
  auto slots_for = [&](int64_t c) {
    int64_t s = 0;
    for (int64_t t = 0; t < n_tiles; ++t) {
      const int64_t k = (cnt[t] + c - 1) / c;
      if (k > 1) s += k;
    }
    return s;
  };
  while (slots_for(chunk) * (int64_t)sizeof(double) * kTileCells > (int64_t(1) << 30)) chunk *= 2;
  std::vector<DepositChunk> chunks;
  std::vector<SplitTile> split;
  int32_t slots = 0;
  chunks.reserve((size_t)n_tiles);
  for (int64_t t = 0; t < n_tiles; ++t) {
    const int64_t k = std::max<int64_t>(1, (cnt[t] + chunk - 1) / chunk);
    if (k == 1) {
      chunks.push_back({(int32_t)t, -1, toff[t], toff[t] + cnt[t]});
      continue;
    }
    split.push_back({(int32_t)t, slots, (int32_t)k});
    for (int64_t c = 0; c < k; ++c) {
      const int64_t b = toff[t] + c * chunk;
      chunks.push_back({(int32_t)t, slots++, b, std::min<int64_t>(b + chunk, toff[t] + cnt[t])});
    }
  }
  // largest chunks first, so the long ones do not form the tail of the launch
  // (the launch order changes nothing in the results: slots are fixed above)
  std::stable_sort(chunks.begin(), chunks.end(), [](const DepositChunk& a, const DepositChunk& b) {
    return a.end - a.begin > b.end - b.begin;
  });
  const size_t a_pairs = align256(sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1));
  const size_t a_toff = align256(sizeof(int64_t) * ((size_t)n_tiles + 1));
  const size_t a_chunks = align256(sizeof(DepositChunk) * std::max<size_t>(chunks.size(), 1));
  const size_t a_split = align256(sizeof(SplitTile) * std::max<size_t>(split.size(), 1));
  char* s1 = static_cast<char*>(
      stream_scratch(stream, kSlotLists, a_pairs + a_toff + a_chunks + a_split));
  double* partial = static_cast<double*>(
      stream_scratch(stream, kSlotPartial, sizeof(double) * kTileCells * std::max(slots, 1)));
  if (!s1 || !partial) {
    kdt_set_error("%s: device allocation failed (%lld particle-tile pairs)", who, (long long)total);
    return KDT_ENOMEM;
  }
  int32_t* pairs = reinterpret_cast<int32_t*>(s1);
  int64_t* d_toff = reinterpret_cast<int64_t*>(s1 + a_pairs);
  DepositChunk* d_chunks = reinterpret_cast<DepositChunk*>(s1 + a_pairs + a_toff);
  SplitTile* d_split = reinterpret_cast<SplitTile*>(s1 + a_pairs + a_toff + a_chunks);
  e = hipMemcpyAsync(d_toff, toff.data(), sizeof(int64_t) * (n_tiles + 1), hipMemcpyHostToDevice,
                     stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_chunks, chunks.data(), sizeof(DepositChunk) * chunks.size(),
                       hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && !split.empty())
    e = hipMemcpyAsync(d_split, split.data(), sizeof(SplitTile) * split.size(),
                       hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) {
    kdt_set_error("%s: %s", who, hipGetErrorString(e));
    return KDT_EDEVICE;
  }
  k_fill_u32<<<gt, 256, 0, stream>>>(tcount, n_tiles, 0u);  // reused as list fill counters
  by_scheme(sch, [&](auto c) {
    constexpr int S = decltype(c)::value;
    if (n > 0) k_p2m_scatter<S><<<gp, kPBlock, 0, stream>>>(g, tg, P, n, d_toff, tcount, pairs);
    k_p2m_tile<S><<<(unsigned)chunks.size(), kPBlock, 0, stream>>>(g, tg, P, n, fbuf, pairs,
                                                                   d_chunks, d_grid, partial);
  });
  if (!split.empty())
    k_p2m_reduce<<<dim3((unsigned)split.size(), kTileCells / kPBlock), kPBlock, 0, stream>>>(
        g, tg, d_split, partial, d_grid);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("%s: kernel launch failed", who);
    return KDT_EDEVICE;
  }
  // the host tables above must outlive their copies
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    kdt_set_error("%s: %s", who, hipGetErrorString(e));
    return KDT_EDEVICE;
  }
  return KDT_OK;
}

extern "C" kdt_status kdt_p2m(const float* d_x, const float* d_m, const float* d_h, int64_t n,
                              const kdt_grid* grid, const int32_t* d_order, float* d_grid,
                              hipStream_t stream) {
  kdt_clear_error();
  return p2m_forward(kSph, "kdt_p2m", Source{d_x, d_m, d_h, d_order, 3, nullptr, true}, n, grid,
                     d_grid, stream);
}

// A fixed cloud's scheme and, on a periodic mesh, the cells per axis it
// needs; false (and the error set) otherwise.
static bool cloud_ok(const char* who, const kdt_grid* grid, int32_t scheme) {
  if (scheme < kNgp || scheme > kTsc) {
    kdt_set_error("%s: scheme %d is not 1 (NGP), 2 (CIC) or 3 (TSC)", who, scheme);
    return false;
  }
  if (grid && grid->periodic)
    for (int a = 0; a < 3; ++a)
      if (grid->n[a] < scheme) {
        kdt_set_error("%s: a periodic mesh needs at least %d cells per axis", who, scheme);
        return false;
      }
  return true;
}

extern "C" kdt_status kdt_p2m_cloud(const float* d_x, const float* d_m, int64_t n,
                                    const kdt_grid* grid, int32_t scheme, const int32_t* d_order,
                                    float* d_grid, hipStream_t stream) {
  kdt_clear_error();
  if (!cloud_ok("kdt_p2m_cloud", grid, scheme)) return KDT_EINVAL;
  return p2m_forward(scheme, "kdt_p2m_cloud", Source{d_x, d_m, nullptr, d_order, 3, nullptr, true},
                     n, grid, d_grid, stream);
}

static kdt_status p2m_backward(const char* who, Source src, int64_t n, const kdt_grid* grid,
                               const float* d_ggrid, float* d_gm, float* d_gx,
                               hipStream_t stream) {
  if (n < 0 || !grid_ok(grid) || (n > 0 && (!src.x || !src.m || !src.h || !d_ggrid))) {
    kdt_set_error("%s: NULL pointer, negative n or invalid grid", who);
    return KDT_EINVAL;
  }
  if (n == 0 || (!d_gm && !d_gx)) return KDT_OK;
  int32_t* bad = static_cast<int32_t*>(stream_scratch(stream, kSlotFlag, 256));
  if (!bad) {
    kdt_set_error("%s: allocation failed", who);
    return KDT_ENOMEM;
  }
  k_zero_f64<<<1, 32, 0, stream>>>(reinterpret_cast<double*>(bad), 1);
  if (src.may_self_order && !src.order && n >= kSelfOrderMin) {
    const kdt_status st = self_order(to_dev(grid), grid->n, src.x, n, stream, who, &src.order);
    if (st != KDT_OK) return st;
  }
  const unsigned gp = (unsigned)((n + kPBlock - 1) / kPBlock);
  if (src.xs == 4)
    k_p2m_bwd<4><<<gp, kPBlock, 0, stream>>>(to_dev(grid), src.x, src.m, src.h, n, src.order,
                                             src.tree_bad, d_ggrid, d_gm, d_gx, bad);
  else
    k_p2m_bwd<3><<<gp, kPBlock, 0, stream>>>(to_dev(grid), src.x, src.m, src.h, n, src.order,
                                             src.tree_bad, d_ggrid, d_gm, d_gx, bad);
  if (hipGetLastError() != hipSuccess) {
    kdt_set_error("%s: kernel launch failed", who);
    return KDT_EDEVICE;
  }
  return read_bad_flag(bad, stream, who, src.tree_bad != nullptr);
}

extern "C" kdt_status kdt_p2m_backward(const float* d_x, const float* d_m, const float* d_h,
                                       int64_t n, const kdt_grid* grid, const int32_t* d_order,
                                       const float* d_ggrid, float* d_gm, float* d_gx,
                                       hipStream_t stream) {
  kdt_clear_error();
  return p2m_backward("kdt_p2m_backward", Source{d_x, d_m, d_h, d_order, 3, nullptr, true}, n,
                      grid, d_ggrid, d_gm, d_gx, stream);
}

// A tree the tree-ordered deposit can read: 3-d float32 coordinates, records
// of 4 floats; false (and the error set) otherwise.
static bool p2m_tree_ok(const kdt_tree* tree, const char* who) {
  if (!tree) {
    kdt_set_error("%s: NULL tree", who);
    return false;
  }
  if (refuse_f64(tree, who)) return false;
  if (tree->d != 3 || tree->stride != 4) {
    kdt_set_error("%s: the deposit needs a tree of 3-d points (this one has d = %d)", who,
                  tree->d);
    return false;
  }
  return true;
}

extern "C" kdt_status kdt_p2m_tree(const kdt_tree* tree, const float* d_m, const float* d_h,
                                   const kdt_grid* grid, int32_t scheme, float* d_grid,
                                   hipStream_t stream) {
  kdt_clear_error();
  if (!p2m_tree_ok(tree, "kdt_p2m_tree")) return tree ? KDT_EUNSUPPORTED : KDT_EINVAL;
  if (scheme != kSph && !cloud_ok("kdt_p2m_tree", grid, scheme)) return KDT_EINVAL;
  return p2m_forward(scheme, "kdt_p2m_tree",
                     Source{tree->rec, d_m, scheme == kSph ? d_h : nullptr, nullptr, 4,
                            tree->flag, false},
                     tree->n, grid, d_grid, stream);
}

extern "C" kdt_status kdt_p2m_tree_backward(const kdt_tree* tree, const float* d_m,
                                            const float* d_h, const kdt_grid* grid,
                                            const float* d_ggrid, float* d_gm, float* d_gx,
                                            hipStream_t stream) {
  kdt_clear_error();
  if (!p2m_tree_ok(tree, "kdt_p2m_tree_backward")) return tree ? KDT_EUNSUPPORTED : KDT_EINVAL;
  return p2m_backward("kdt_p2m_tree_backward",
                      Source{tree->rec, d_m, d_h, nullptr, 4, tree->flag, false}, tree->n, grid,
                      d_ggrid, d_gm, d_gx, stream);
}
