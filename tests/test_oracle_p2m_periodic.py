"""Pins for the oracle's periodic particle-to-mesh deposit: the mesh of
Sec. 4.2 on the periodic boundaries of Sec. 2.4 (a 3-torus of periods
n_a * cell; cell distances the shorter way round per axis, as the torus metric
of the queries of Sec. 2.1), and its adjoint."""
import numpy as np
import pytest

import oracle

CELL = 1.0 / 16
SHAPES = ((16, 16, 16), (16, 12, 20))


def _particles(n, seed, shape, hmax):
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.array(shape) * CELL
    x = rng.random((n, 3)) * L
    # a third of them hugging a face, an edge or a corner
    k = n // 3
    x[:k] = (rng.random((k, 3)) * 0.06 - 0.03) % L
    m = rng.random(n) + 0.5
    h = rng.random(n) * hmax
    return x, m, h


@pytest.mark.parametrize("shape", SHAPES)
def test_support_box_equals_whole_mesh_minimum_image(shape):
    """The support loop (unwrapped cell indices, nearest copy) against every
    cell of the mesh measured the shorter way round on each axis."""
    hmax = 0.49 * min(shape) * CELL
    x, m, h = _particles(60, 3, shape, hmax)
    # supports of almost half a period, from every part of a cell: the cells
    # half a period away are reached on one side only
    frac = np.linspace(0.05, 0.95, 10)
    xe = np.stack([(3 + frac) * CELL, (5 + frac[::-1]) * CELL, (7 + frac) * CELL], axis=1)
    x = np.concatenate([x, xe])
    m = np.concatenate([m, np.ones(10)])
    h = np.concatenate([h, np.full(10, hmax)])
    a = oracle.p2m(x, m, h, (0, 0, 0), CELL, shape, periodic=True)
    b = oracle.p2m(x, m, h, (0, 0, 0), CELL, shape, periodic=True, brute=True)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("shape", SHAPES)
def test_no_mass_is_dropped(shape):
    x, m, h = _particles(200, 4, shape, 0.3 * min(shape) * CELL)
    rho = oracle.p2m(x, m, h, (0, 0, 0), CELL, shape, periodic=True)
    assert abs(rho.sum() - m.sum()) <= 1e-12 * m.sum()
    # the open mesh does drop the support beyond the faces, so the two differ
    rho_open = oracle.p2m(x, m, h, (0, 0, 0), CELL, shape)
    assert np.abs(rho - rho_open).max() > 1e-3


@pytest.mark.parametrize("shift", ((1, 0, 0), (0, 5, 0), (3, 11, 7), (15, 15, 15)))
def test_translation_by_whole_cells_rolls_the_mesh(shift):
    shape = (16, 16, 16)
    x, m, h = _particles(80, 5, shape, 0.4)
    L = np.array(shape) * CELL
    y = (x + np.array(shift) * CELL) % L
    a = oracle.p2m(x, m, h, (0, 0, 0), CELL, shape, periodic=True)
    b = oracle.p2m(y, m, h, (0, 0, 0), CELL, shape, periodic=True)
    np.testing.assert_allclose(np.roll(a, shift, axis=(0, 1, 2)), b, rtol=1e-9, atol=1e-12)


def test_equals_open_deposit_away_from_the_faces():
    shape = (16, 16, 16)
    rng = np.random.Generator(np.random.PCG64(6))
    h = rng.random(50) * 0.2
    H = np.maximum(h, CELL)
    x = H[:, None] + 2 * CELL + rng.random((50, 3)) * (1.0 - 2 * H[:, None] - 4 * CELL)
    m = rng.random(50) + 0.5
    a = oracle.p2m(x, m, h, (0, 0, 0), CELL, shape, periodic=True)
    b = oracle.p2m(x, m, h, (0, 0, 0), CELL, shape)
    np.testing.assert_array_equal(a, b)


def test_particle_on_the_box_vertex_splits_over_the_eight_corner_cells():
    shape = (16, 16, 16)
    rho = oracle.p2m(np.zeros((1, 3)), np.array([2.0]), np.array([CELL]), (0, 0, 0), CELL,
                     shape, periodic=True)
    corners = [(i, j, k) for i in (0, 15) for j in (0, 15) for k in (0, 15)]
    for c in corners:
        assert abs(rho[c] - 0.25) < 1e-14
    assert abs(rho.sum() - 2.0) < 1e-14


def test_support_of_half_a_period_is_refused():
    shape = (16, 12, 20)
    x = np.array([[0.5, 0.3, 0.6]])
    with pytest.raises(ValueError):
        oracle.p2m(x, np.ones(1), np.array([0.5 * 12 * CELL]), (0, 0, 0), CELL, shape,
                   periodic=True)
    oracle.p2m(x, np.ones(1), np.array([0.49 * 12 * CELL]), (0, 0, 0), CELL, shape,
               periodic=True)


def test_adjoint_finite_differences_dot_product_and_constant_gradient():
    shape = (16, 12, 20)
    x, m, h = _particles(12, 7, shape, 0.3)
    rng = np.random.Generator(np.random.PCG64(8))
    g = rng.standard_normal(shape)
    kw = dict(lo=(0, 0, 0), cell=CELL, shape=shape, periodic=True)
    dm, dx = oracle.p2m_backward(x, m, h, g=g, **kw)
    loss = lambda xx, mm: float((g * oracle.p2m(xx, mm, h, **kw)).sum())
    eps = 1e-5 * CELL
    L = np.array(shape) * CELL
    for i in range(len(m)):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] = (xp[i, a] + eps) % L[a]
            xm[i, a] = (xm[i, a] - eps) % L[a]
            fd = (loss(xp, m) - loss(xm, m)) / (2 * eps)
            assert abs(fd - dx[i, a]) <= 1e-6 * max(1.0, abs(dx[i, a])), (i, a, fd, dx[i, a])
    # linear in m: <g, P2M(m)> = <dL/dm, m>
    assert abs(loss(x, m) - float(dm @ m)) <= 1e-12 * abs(loss(x, m))
    # a constant upstream gradient: no mass leaves the torus, nothing moves
    dm1, dx1 = oracle.p2m_backward(x, m, h, g=np.ones(shape), **kw)
    np.testing.assert_allclose(dm1, 1.0, rtol=1e-13)
    assert np.abs(dx1).max() < 1e-12
