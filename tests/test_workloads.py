"""The seeded workload generators: sizes, ranges, determinism, and the
statistics each one is defined by (Sec. 3.1 uniform and inhomogeneous mocks,
Sec. 4.1 style clustered mock)."""
import numpy as np

from paper_2609_18316_amd import workloads


def test_grf_mock_shape_range_and_determinism():
    for n in (1, 7, 1000, 20011):
        x = workloads.grf(n, 3)
        assert x.shape == (n, 3) and x.dtype == np.float32
        assert (x >= 0).all() and (x < 1).all()
        np.testing.assert_array_equal(x, workloads.grf(n, 3))
    assert not np.array_equal(workloads.grf(1000, 3), workloads.grf(1000, 4))


def test_grf_counts_follow_the_density():
    """Per cell, the number of points is the density's share of n, rounded by
    largest remainder (so within one of the exact quota)."""
    n = 30000
    nx = int(np.floor(n ** (1 / 3) + 1e-9))
    rho = workloads.grf_density(nx, 5).reshape(-1)
    x = workloads.grf(n, 5)
    ijk = np.minimum((x.astype(np.float64) * nx).astype(np.int64), nx - 1)
    counts = np.bincount(np.ravel_multi_index(ijk.T, (nx, nx, nx)), minlength=nx ** 3)
    quota = rho / rho.sum() * n
    assert counts.sum() == n
    assert (np.abs(counts - quota) < 1.0 + 1e-9).all()
    # an inhomogeneous field: the densest cells hold many times the mean
    assert counts.max() > 8 * n / nx ** 3


def test_grf_field_has_the_requested_spectral_index():
    """The log-density is the filtered Gaussian field: its power spectrum
    falls as |k|^-2 (fitted slope over the resolved shells)."""
    nx = 64
    delta = np.log(workloads.grf_density(nx, 7))
    p = np.abs(np.fft.fftn(delta)) ** 2
    k = np.fft.fftfreq(nx) * nx
    kk = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
    shells = np.arange(2, 20)
    pk = np.array([p[(kk >= s - 0.5) & (kk < s + 0.5)].mean() for s in shells])
    slope = np.polyfit(np.log(shells), np.log(pk), 1)[0]
    assert abs(slope - workloads.GRF_INDEX) < 0.15, slope
    assert abs(np.mean(delta)) < 1e-9 and abs(np.std(delta) - 1.0) < 1e-9


def test_clustered_and_uniform_ranges():
    x = workloads.clustered(5000, 2)
    assert x.shape == (5000, 3) and (x >= 0).all() and (x < 1).all()
    u = workloads.uniform(1000, 4, 1)
    assert (u >= 0).all() and (u < 1).all()
    # uniform draws sit on the 2^-24 lattice
    assert np.array_equal(u, np.round(u.astype(np.float64) * 2 ** 24) / 2 ** 24)
