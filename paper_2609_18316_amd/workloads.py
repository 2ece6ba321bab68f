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
