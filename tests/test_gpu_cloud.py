"""GPU parity of the fixed-cloud deposits (NGP, CIC, TSC: the schemes the
adaptive deposit is compared with in Sec. 4.2 and Table 3) against the
float64 oracle, to the deposit's tolerance: per cell
|rho32 - rho64| <= 1e-5 max(|rho64|, mean cell mass), total mass within
1e-5.  NGP decides its cell in float32 on both sides, so it is exact."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_18316_amd import kdt, workloads
from tests.gpu_util import dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [((16, 16, 16), 1.0 / 16), ((32, 24, 40), 1.0 / 32), ((64, 64, 64), 1.0 / 64)]


def _close(g, o, total):
    mean = total / o.size
    err = np.abs(g.astype(np.float64) - o)
    bound = 1e-5 * np.maximum(np.abs(o), mean)
    assert (err <= bound).all(), float((err / bound).max())
    assert abs(float(g.astype(np.float64).sum()) - total) <= 1e-5 * total


def _points(n, shape, cell, seed):
    L = np.array(shape, np.float64) * cell
    x = (workloads.clustered(n, seed).astype(np.float64) * L).astype(np.float32)
    return np.minimum(x, np.nextafter(L.astype(np.float32), 0))


@pytest.mark.parametrize("scheme", ("ngp", "cic", "tsc"))
@pytest.mark.parametrize("periodic", (False, True))
@pytest.mark.parametrize("n,shape,cell", [(n,) + sc for n in (1, 777, 20000) for sc in SHAPES]
                         + [(300000,) + SHAPES[2]])
def test_cloud_matches_float64_oracle(scheme, periodic, n, shape, cell):
    dev()
    say(f"{scheme} periodic={periodic} n={n} shape={shape}")
    x = _points(n, shape, cell, seed=600 + n)
    m = workloads.masses(n, 601 + n)
    o = oracle.p2m_cloud(x, m, (0, 0, 0), cell, shape, scheme, periodic=periodic)
    t = kdt.build(to_dev(x))
    for order in (t.perm_ptr, None):
        g = kdt.p2m_cloud(to_dev(x), to_dev(m), (0, 0, 0), cell, shape, scheme,
                          order_ptr=order, periodic=periodic)
        g = to_host(g)
        _close(g, o, float(m.astype(np.float64).sum()))
        if scheme == "ngp":
            np.testing.assert_allclose(g, o, rtol=1e-6, atol=0)
    t.close()


def test_cloud_particles_on_faces_and_cell_centres():
    dev()
    shape, cell = (16, 16, 16), 1.0 / 16
    x = (np.array([[5.0, 7.5, 0.0], [0.0, 0.0, 0.0], [15.5, 15.5, 15.5], [8.0, 8.0, 8.0]])
         * cell).astype(np.float32)
    m = np.array([1.0, 2.0, 3.0, 4.0], np.float32)
    for scheme in ("ngp", "cic", "tsc"):
        for periodic in (False, True):
            o = oracle.p2m_cloud(x, m, (0, 0, 0), cell, shape, scheme, periodic=periodic)
            g = to_host(kdt.p2m_cloud(to_dev(x), to_dev(m), (0, 0, 0), cell, shape, scheme,
                                      periodic=periodic))
            _close(g, o, 10.0)


def test_cloud_errors_and_empty_input():
    dev()
    x = to_dev(np.array([[0.5, 0.5, 0.5]], np.float32))
    m = to_dev(np.ones(1, np.float32))
    with pytest.raises(kdt.KdtError) as e:
        kdt.load()
        g = kdt.make_grid((0, 0, 0), 1 / 16, (16, 16, 16))
        out = torch.empty((16, 16, 16), device=dev())
        kdt._check(kdt.load().kdt_p2m_cloud(kdt._ptr(x), kdt._ptr(m), 1, kdt.C.byref(g), 4,
                                            None, kdt._ptr(out), kdt._stream()))
    assert e.value.status == kdt.KDT_EINVAL
    with pytest.raises(kdt.KdtError) as e:  # a periodic TSC needs 3 cells per axis
        kdt.p2m_cloud(x, m, (0, 0, 0), 0.5, (2, 2, 2), "tsc", periodic=True)
    assert e.value.status == kdt.KDT_EINVAL
    with pytest.raises(kdt.KdtError) as e:  # outside the mesh
        kdt.p2m_cloud(to_dev(np.array([[0.5, 0.5, 1.5]], np.float32)), m, (0, 0, 0), 1 / 16,
                      (16, 16, 16), "cic")
    assert e.value.status == kdt.KDT_EINVAL
    z = kdt.p2m_cloud(x[:0], m[:0], (0, 0, 0), 1 / 16, (16, 16, 16), "tsc")
    assert float(z.abs().sum()) == 0.0
