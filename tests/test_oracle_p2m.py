"""Pins for the oracle's adaptive SPH particle-to-mesh deposit (Sec. 4.2) and
its adjoint, against properties the M4 spline and the deposit must have."""
import numpy as np
import pytest

import oracle

G16 = dict(lo=(0.0, 0.0, 0.0), cell=1.0 / 16, shape=(16, 16, 16))


def _particles(n, seed, hmax=0.2):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.random((n, 3))
    m = rng.random(n) + 0.5
    h = rng.random(n) * hmax
    return x, m, h


def test_m4_normalisation_and_smoothness():
    # 4 pi int_0^2 w(q) q^2 dq = pi for the M4 spline (Monaghan & Lattanzio 1985)
    q = np.linspace(0.0, 2.0, 20001)
    w = np.array([oracle.m4_w(v) for v in q])
    f = w * q * q
    integral = 4.0 * np.pi * np.sum((f[1:] + f[:-1]) * 0.5 * np.diff(q))
    assert abs(integral - np.pi) < 1e-7
    assert oracle.m4_w(0.0) == 1.0 and oracle.m4_dw(0.0) == 0.0
    assert oracle.m4_w(2.0) == 0.0 and oracle.m4_w(2.5) == 0.0
    eps = 1e-7
    for b in (1.0, 2.0):  # C2 at the branch points
        assert abs(oracle.m4_w(b - eps) - oracle.m4_w(b + eps)) < 1e-6
        assert abs(oracle.m4_dw(b - eps) - oracle.m4_dw(b + eps)) < 1e-6
        d2l = (oracle.m4_dw(b - eps) - oracle.m4_dw(b - 2e-4)) / (2e-4 - eps)
        d2r = (oracle.m4_dw(b + 2e-4) - oracle.m4_dw(b + eps)) / (2e-4 - eps)
        assert abs(d2l - d2r) < 1e-2
    for v in np.linspace(0.01, 1.99, 37):  # w' is the derivative of w
        fd = (oracle.m4_w(v + 1e-6) - oracle.m4_w(v - 1e-6)) / 2e-6
        assert abs(fd - oracle.m4_dw(v)) < 1e-6


def test_mass_conservation_and_linearity():
    x, m, h = _particles(200, 1)
    rho = oracle.p2m(x, m, h, **G16)
    assert abs(rho.sum() - m.sum()) < 1e-10 * m.sum()
    assert (rho >= 0).all()
    m2 = np.random.Generator(np.random.PCG64(9)).random(200)
    a = oracle.p2m(x, m + 2.0 * m2, h, **G16)
    b = rho + 2.0 * oracle.p2m(x, m2, h, **G16)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)


def test_support_box_equals_whole_grid_scan():
    x, m, h = _particles(150, 2, hmax=0.3)
    np.testing.assert_allclose(oracle.p2m(x, m, h, **G16),
                               oracle.p2m(x, m, h, brute=True, **G16), rtol=1e-13, atol=1e-16)


def test_particle_at_cell_centre_with_unit_support():
    c = 1.0 / 16
    x = np.array([[5.5 * c, 7.5 * c, 9.5 * c]])
    rho = oracle.p2m(x, [2.0], [c], **G16)  # H = cell: neighbours sit at q = 2
    assert rho[5, 7, 9] == pytest.approx(2.0, rel=1e-15)
    assert np.count_nonzero(rho) == 1
    rho = oracle.p2m(x, [1.0], [0.0], **G16)  # h below the cell size is floored
    assert rho[5, 7, 9] == pytest.approx(1.0, rel=1e-15)


def test_particle_at_cell_vertex_splits_in_eight():
    c = 1.0 / 16
    x = np.array([[8 * c, 4 * c, 11 * c]])
    rho = oracle.p2m(x, [1.0], [0.0], **G16)
    nz = np.argwhere(rho > 0)
    assert len(nz) == 8
    np.testing.assert_allclose(rho[rho > 0], 0.125, rtol=1e-14)
    assert set(map(tuple, nz)) == {(i, j, k) for i in (7, 8) for j in (3, 4) for k in (10, 11)}


def test_cell_centre_with_double_support_has_m4_ratios():
    """H = 2 cells: face neighbours sit at q = 1 where w = 1/4 of w(0)."""
    c = 1.0 / 16
    x = np.array([[6.5 * c, 6.5 * c, 6.5 * c]])
    rho = oracle.p2m(x, [1.0], [2 * c], **G16)
    self_ = rho[6, 6, 6]
    faces = [rho[5, 6, 6], rho[7, 6, 6], rho[6, 5, 6], rho[6, 7, 6], rho[6, 6, 5], rho[6, 6, 7]]
    np.testing.assert_allclose(np.array(faces) / self_, 0.25, rtol=1e-13)
    edges = [rho[5, 5, 6], rho[7, 6, 7], rho[6, 5, 7]]
    np.testing.assert_allclose(edges, edges[0], rtol=1e-13)
    assert rho[4, 6, 6] == 0.0  # q = 2
    assert np.count_nonzero(rho) == 1 + 6 + 12 + 8


def test_boundary_particle_keeps_its_mass():
    c = 1.0 / 16
    x = np.array([[0.1 * c, 15.9 * c, 0.3 * c]])
    rho = oracle.p2m(x, [1.5], [3 * c], **G16)
    assert rho.sum() == pytest.approx(1.5, rel=1e-14)


def test_rejects_particles_outside_the_grid():
    with pytest.raises(ValueError):
        oracle.p2m(np.array([[1.0, 0.5, 0.5]]), [1.0], [0.1], **G16)


def _loss_grad_fd(x, m, h, g, eps):
    dx = np.zeros_like(x)
    for i in range(x.shape[0]):
        for e in range(3):
            xp = x.copy()
            xm = x.copy()
            xp[i, e] += eps
            xm[i, e] -= eps
            lp = float((g * oracle.p2m(xp, m, h, **G16)).sum())
            lm = float((g * oracle.p2m(xm, m, h, **G16)).sum())
            dx[i, e] = (lp - lm) / (2 * eps)
    return dx


def test_adjoint_matches_central_differences():
    rng = np.random.Generator(np.random.PCG64(21))
    x = 0.15 + 0.7 * rng.random((12, 3))
    m = rng.random(12) + 0.5
    h = 0.05 + 0.15 * rng.random(12)
    g = rng.standard_normal(G16["shape"])
    dm, dx = oracle.p2m_backward(x, m, h, g=g, **G16)
    # the central-difference error falls like eps^2 (about 9e-4 relative at
    # eps = 1e-3 cell, 9e-8 at 1e-5 cell), so a small step is used
    fd = _loss_grad_fd(x, m, h, g, eps=1e-5 / 16)
    np.testing.assert_allclose(dx, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())
    # dL/dm by differences in m (exact up to rounding: rho is linear in m)
    for i in range(3):
        mp = m.copy()
        mp[i] += 1e-3
        lp = float((g * oracle.p2m(x, mp, h, **G16)).sum())
        l0 = float((g * oracle.p2m(x, m, h, **G16)).sum())
        assert (lp - l0) / 1e-3 == pytest.approx(dm[i], rel=1e-8)


def test_adjoint_dot_product_and_constant_gradient():
    x, m, h = _particles(80, 5)
    g = np.random.Generator(np.random.PCG64(6)).standard_normal(G16["shape"])
    rho = oracle.p2m(x, m, h, **G16)
    dm, dx = oracle.p2m_backward(x, m, h, g=g, **G16)
    assert float((g * rho).sum()) == pytest.approx(float((dm * m).sum()), rel=1e-12)
    dm1, dx1 = oracle.p2m_backward(x, m, h, g=np.ones(G16["shape"]), **G16)
    np.testing.assert_allclose(dm1, 1.0, rtol=1e-13)
    assert np.abs(dx1).max() < 1e-11
