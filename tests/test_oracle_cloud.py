"""Pins for the oracle's fixed-cloud deposits (NGP, CIC, TSC: the comparison
schemes of Sec. 4.2 and Table 3): the shape functions against their closed
forms and moments, the per-axis stencils against the shape functions over the
whole mesh, conservation, and the patterns of particles at cell centres and
vertices."""
import numpy as np
import pytest

import oracle

SCHEMES = ("ngp", "cic", "tsc")
CELL = 1.0 / 16


def _w(scheme, s):
    """Weights W(j - s) of the cells j around s (integer offsets -3..3)."""
    j = np.floor(s) + np.arange(-3, 5)
    return j, np.array([oracle.cloud_shape(scheme, v) for v in j - s])


@pytest.mark.parametrize("scheme", SCHEMES)
def test_shape_functions_partition_unity_and_moments(scheme):
    rng = np.random.Generator(np.random.PCG64(1))
    for s in np.concatenate([rng.random(200) * 10 - 5, [0.0, 0.5, -0.5, 0.25, 1.75]]):
        j, w = _w(scheme, s)
        assert abs(w.sum() - 1.0) < 1e-14
        assert (w >= 0).all()
        v = j - s
        if scheme != "ngp":
            assert abs((w * v).sum()) < 1e-13           # centre of mass kept
        if scheme == "cic":
            f = s - np.floor(s)
            assert abs((w * v * v).sum() - f * (1 - f)) < 1e-13
        if scheme == "tsc":
            assert abs((w * v * v).sum() - 0.25) < 1e-13  # the cloud's variance
    # values at the centre and the support edges
    c = {"ngp": 1.0, "cic": 1.0, "tsc": 0.75}[scheme]
    assert oracle.cloud_shape(scheme, 0.0) == c
    edge = {"ngp": 0.5, "cic": 1.0, "tsc": 1.5}[scheme]
    assert oracle.cloud_shape(scheme, -edge) == 0.0
    assert oracle.cloud_shape(scheme, edge + 1e-9) == 0.0
    # NGP: a particle on a cell face belongs to the cell above it (the cell
    # whose centre is half a cell above: v = +1/2)
    assert oracle.cloud_shape(scheme, edge) == (1.0 if scheme == "ngp" else 0.0)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("periodic", (False, True))
def test_stencil_equals_the_shape_function_over_the_whole_mesh(scheme, periodic):
    rng = np.random.Generator(np.random.PCG64(2))
    shape = (16, 12, 20)
    L = np.array(shape) * CELL
    x = rng.random((80, 3)) * L
    x[:20] = (rng.random((20, 3)) * 0.04 - 0.02) % L  # near faces and corners
    m = rng.random(80) + 0.5
    a = oracle.p2m_cloud(x, m, (0, 0, 0), CELL, shape, scheme, periodic=periodic)
    b = oracle.p2m_cloud(x, m, (0, 0, 0), CELL, shape, scheme, periodic=periodic, brute=True)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)
    assert abs(a.sum() - m.sum()) < 1e-12 * m.sum()


def test_ngp_particle_on_a_face_goes_to_the_cell_above():
    shape = (16, 16, 16)
    x = np.array([[5.0, 7.5, 0.0]]) * CELL
    for brute in (False, True):
        rho = oracle.p2m_cloud(x, np.ones(1), (0, 0, 0), CELL, shape, "ngp", brute=brute)
        assert rho[5, 7, 0] == 1.0


def test_particle_at_a_cell_centre():
    shape = (16, 16, 16)
    x = np.array([[5.5, 7.5, 9.5]]) * CELL
    for scheme in ("ngp", "cic"):
        rho = oracle.p2m_cloud(x, np.ones(1), (0, 0, 0), CELL, shape, scheme)
        assert rho[5, 7, 9] == 1.0 and rho.sum() == 1.0
    rho = oracle.p2m_cloud(x, np.ones(1), (0, 0, 0), CELL, shape, "tsc")
    w1 = np.array([0.125, 0.75, 0.125])
    np.testing.assert_allclose(rho[4:7, 6:9, 8:11], np.einsum("i,j,k->ijk", w1, w1, w1),
                               rtol=1e-14)
    assert abs(rho.sum() - 1.0) < 1e-14


def test_cic_particle_on_a_vertex_splits_in_eight():
    shape = (16, 16, 16)
    x = np.array([[6.0, 6.0, 6.0]]) * CELL  # between the centres 5.5 and 6.5
    rho = oracle.p2m_cloud(x, np.array([8.0]), (0, 0, 0), CELL, shape, "cic")
    np.testing.assert_allclose(rho[5:7, 5:7, 5:7], 1.0, rtol=1e-14)
    # periodic box corner: the eight corner cells
    rho = oracle.p2m_cloud(np.zeros((1, 3)), np.array([8.0]), (0, 0, 0), CELL, shape, "cic",
                           periodic=True)
    for c in [(i, j, k) for i in (0, 15) for j in (0, 15) for k in (0, 15)]:
        assert abs(rho[c] - 1.0) < 1e-14


@pytest.mark.parametrize("scheme", ("cic", "tsc"))
def test_centre_of_mass_is_kept_inside_the_mesh(scheme):
    rng = np.random.Generator(np.random.PCG64(3))
    shape = (16, 16, 16)
    x = (3 + rng.random((30, 3)) * 10) * CELL
    for p in x:
        rho = oracle.p2m_cloud(p[None, :], np.ones(1), (0, 0, 0), CELL, shape, scheme)
        idx = np.argwhere(rho > 0)
        centres = (idx + 0.5) * CELL
        com = (rho[rho > 0][:, None] * centres).sum(axis=0)
        np.testing.assert_allclose(com, p, atol=1e-13)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_translation_by_whole_cells_rolls_a_periodic_mesh(scheme):
    rng = np.random.Generator(np.random.PCG64(4))
    shape = (16, 16, 16)
    x = rng.random((50, 3))
    m = rng.random(50) + 0.5
    shift = (3, 15, 7)
    y = (x + np.array(shift) * CELL) % 1.0
    a = oracle.p2m_cloud(x, m, (0, 0, 0), CELL, shape, scheme, periodic=True)
    b = oracle.p2m_cloud(y, m, (0, 0, 0), CELL, shape, scheme, periodic=True)
    np.testing.assert_allclose(np.roll(a, shift, axis=(0, 1, 2)), b, rtol=1e-9, atol=1e-12)
