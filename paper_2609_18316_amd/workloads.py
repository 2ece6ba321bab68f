"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module only draws random numbers: it holds none of the k-d tree, query,
grouping or deposit arithmetic, so both the HIP path and the CPU oracle can be
fed the same bytes without sharing any of the method's code.

The paper benchmarks on procedural mocks (uniform points in a hypercube of
side L, §3.1; a clustered mock of Gaussian groups plus a uniform background,
§4.1).  The generators below are the stand-ins for those workloads:

* ``uniform``   -- points uniform in [0, 1)^d (the §3.1 uniform mock, L = 1).
* ``normal``    -- standard-normal points in d dimensions.
* ``clustered`` -- 2000 isotropic Gaussian halos (80 % of the points) plus a
  20 % uniform background in [0, 1)^3, the §4.1 style of clustered mock.
* ``grf``       -- the §3.1 inhomogeneous mock: particles placed in proportion
  to a Gaussian-random-field density (spectral index -2) on a grid of about
  N^(1/3) cells per side.
* ``masses``    -- particle masses for the particle-to-mesh deposit (§4.2).
* ``batch_sizes`` -- log-uniform sizes for many independent point sets.

All draws use ``numpy.random.Generator(PCG64(seed))``.  Uniform float32 draws
are multiples of 2^-24, which makes equal squared distances (ties) common.
"""
from __future__ import annotations

import numpy as np

N_HALOS = 2000
HALO_FRACTION = 0.8
SIGMA_RANGE = (0.002, 0.02)
MASS_RANGE = (1.0, 1.0e3)
MASS_SLOPE = -1.9


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(n: int, d: int, seed: int) -> np.ndarray:
    """``n`` points uniform in [0, 1)^d, float32, row-major ``[n][d]``."""
    return _rng(seed).random((n, d), dtype=np.float32)


def normal(n: int, d: int, seed: int) -> np.ndarray:
    """``n`` standard-normal points in d dimensions, float32 ``[n][d]``."""
    return _rng(seed).standard_normal((n, d), dtype=np.float32)


def _hamilton_split(total: int, weights: np.ndarray) -> np.ndarray:
    """Integer shares of ``total`` proportional to ``weights`` (largest remainder).

    Each share is the floor of its exact quota; the points left over go one
    each to the largest fractional parts, ties to the lower halo id.
    """
    quota = weights / weights.sum() * total
    base = np.floor(quota).astype(np.int64)
    left = total - int(base.sum())
    frac = quota - base
    order = np.lexsort((np.arange(len(frac)), -frac))
    base[order[:left]] += 1
    return base


def clustered(n: int, seed: int) -> np.ndarray:
    """Clustered 3-D mock: Gaussian halos plus a uniform background.

    * 2000 halo centres uniform in [0, 1)^3;
    * halo scale sigma log-uniform in [0.002, 0.02], independent of mass;
    * halo mass from a power law dN/dM ~ M^-1.9 on [1, 1e3] (inverse CDF);
    * floor(0.8 n) halo points split between halos in proportion to mass;
    * halo points at centre + sigma * N(0, I) in float64, wrapped into [0, 1)
      and rounded to float32 (a value that rounds to 1.0 becomes 0.0);
    * the remaining points uniform in [0, 1)^3;
    * finally a seeded random permutation, so the index carries no structure.
    """
    rng = _rng(seed)
    centres = rng.random((N_HALOS, 3))
    lo, hi = np.log10(SIGMA_RANGE[0]), np.log10(SIGMA_RANGE[1])
    sigma = 10.0 ** rng.uniform(lo, hi, N_HALOS)
    a = MASS_SLOPE + 1.0
    u = rng.random(N_HALOS)
    m_lo, m_hi = MASS_RANGE
    mass = (m_lo ** a + u * (m_hi ** a - m_lo ** a)) ** (1.0 / a)
    n_halo = int(np.floor(HALO_FRACTION * n))
    counts = _hamilton_split(n_halo, mass)
    owner = np.repeat(np.arange(N_HALOS), counts)
    z = rng.standard_normal((n_halo, 3))
    x = centres[owner] + sigma[owner, None] * z
    x -= np.floor(x)
    x32 = x.astype(np.float32)
    x32[x32 >= np.float32(1.0)] = np.float32(0.0)
    bg = rng.random((n - n_halo, 3), dtype=np.float32)
    pts = np.concatenate([x32, bg], axis=0)
    perm = rng.permutation(n)
    return np.ascontiguousarray(pts[perm])


GRF_INDEX = -2.0


def grf_density(nx: int, seed: int, index: float = GRF_INDEX) -> np.ndarray:
    """Density on an ``nx``^3 periodic grid from a Gaussian random field with
    power spectrum P(k) ~ |k|^index (the §3.1 mock uses index -2).

    White noise is drawn on the grid, filtered in Fourier space by
    sqrt(P(k)) (the k = 0 mode removed), and transformed back, giving a field
    delta with zero mean.  The paper does not say how delta becomes a
    (non-negative) density; the reading here is the lognormal map
    rho = exp(delta / std(delta)), float64, mean not normalised.
    """
    rng = _rng(seed)
    white = rng.standard_normal((nx, nx, nx))
    f = np.fft.rfftn(white)
    k = np.fft.fftfreq(nx) * nx
    kz = np.fft.rfftfreq(nx) * nx
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (index / 4.0)  # sqrt(P) = |k|^(index / 2)
    delta = np.fft.irfftn(f * amp, s=(nx, nx, nx), axes=(0, 1, 2))
    sd = delta.std()
    return np.exp(delta / sd) if sd > 0 else np.ones_like(delta)  # a 1^3 grid has no field


def grf(n: int, seed: int, index: float = GRF_INDEX) -> np.ndarray:
    """The §3.1 inhomogeneous mock: ``n`` points in [0, 1)^3, float32.

    * density from ``grf_density`` on nx = floor(n^(1/3)) cells per side, so
      the mean spacing of the points is about one cell;
    * per cell, a share of the n points proportional to its density (largest
      remainder, ties to the lower cell index);
    * each point at its cell's corner plus a uniform shift inside the cell,
      in float64, rounded to float32 (a value that rounds to 1.0 becomes 0.0);
    * finally a seeded random permutation.
    """
    nx = max(1, int(np.floor(n ** (1.0 / 3.0) + 1e-9)))
    rho = grf_density(nx, seed, index).reshape(-1)
    counts = _hamilton_split(n, rho)
    rng = _rng(seed + 1)
    cell = np.repeat(np.arange(nx ** 3), counts)
    ijk = np.stack(np.unravel_index(cell, (nx, nx, nx)), axis=1).astype(np.float64)
    x = (ijk + rng.random((n, 3))) / nx
    x32 = x.astype(np.float32)
    x32[x32 >= np.float32(1.0)] = np.float32(0.0)
    return np.ascontiguousarray(x32[rng.permutation(n)])


def masses(n: int, seed: int) -> np.ndarray:
    """Particle masses uniform in [0.5, 1.5), float32."""
    return (_rng(seed).random(n, dtype=np.float32) + np.float32(0.5)).astype(np.float32)


def batch_sizes(n_sets: int, lo_exp: float, hi_exp: float, seed: int) -> np.ndarray:
    """``n_sets`` set sizes ``round(10 ** U(lo_exp, hi_exp))`` as int64."""
    e = _rng(seed).uniform(lo_exp, hi_exp, n_sets)
    return np.rint(10.0 ** e).astype(np.int64)


def batched_clustered(sizes: np.ndarray, seed_base: int) -> tuple[np.ndarray, np.ndarray]:
    """Concatenate ``clustered(sizes[s], seed_base + s)`` for every set.

    Returns the points ``[sum n_s][3]`` float32 and ``offsets[n_sets + 1]``
    int64 (set s owns rows ``offsets[s]:offsets[s+1]``).
    """
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    out = np.empty((int(offsets[-1]), 3), dtype=np.float32)
    for s, n_s in enumerate(sizes):
        out[offsets[s]:offsets[s + 1]] = clustered(int(n_s), seed_base + s)
    return out, offsets


def sample_indices(n: int, m: int, seed: int) -> np.ndarray:
    """``m`` distinct indices in [0, n) (sorted), for sampled parity checks."""
    m = min(m, n)
    return np.sort(_rng(seed).choice(n, size=m, replace=False)).astype(np.int64)
