"""The matrix-core filter of the wave kNN (d = 8, 16) must never drop a
point that belongs in the answer: it marks candidates with fp32 MFMA dot
products and a rounding margin, and the exact float32 distances decide.
These cases put the decision within a few ulps or make the norm expansion
cancel badly; results must stay bit-identical to the oracle."""
import numpy as np
import pytest

import oracle
from paper_2609_18316_amd import kdt
from tests.gpu_util import dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _shells(d, n_centres, per_shell, seed):
    """Points on thin shells around random centres (radius 0.3, relative
    spread 1e-6): many distances tie within a few ulps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.random((n_centres, d))
    pts = []
    for c in centres:
        v = rng.standard_normal((per_shell, d))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        r = 0.3 * (1.0 + 1e-6 * rng.standard_normal((per_shell, 1)))
        pts.append(c + r * v)
    return np.concatenate(pts).astype(np.float32), centres.astype(np.float32)


@pytest.mark.parametrize("d", (8, 16))
@pytest.mark.parametrize("k", (1, 16, 64))
def test_filter_keeps_near_ties(d, k):
    dev()
    x, centres = _shells(d, 40, 150, seed=31 + d)
    rng = np.random.Generator(np.random.PCG64(32 + d))
    q = (centres + 1e-7 * rng.standard_normal(centres.shape)).astype(np.float32)
    say(f"shell near-ties d={d} k={k}")
    oi, od = oracle.knn_brute(x, q, k)
    for leaf in (16, 64):
        t = kdt.build(to_dev(x), leaf_size=leaf)
        gi, gd = t.knn(to_dev(q), k, traversal=2)
        np.testing.assert_array_equal(to_host(gi), oi)
        np.testing.assert_array_equal(to_host(gd), od)
        t.close()


@pytest.mark.parametrize("d", (8, 16))
@pytest.mark.parametrize("offset", (1e3, -3e4))
def test_filter_far_from_the_origin(d, offset):
    """|q|^2 and |p|^2 dwarf the distances: the expansion cancels and the
    filter keeps almost everything, which must still give exact results."""
    dev()
    rng = np.random.Generator(np.random.PCG64(33 + d))
    x = (rng.random((6000, d)) + offset).astype(np.float32)
    q = (rng.random((500, d)) + offset).astype(np.float32)
    say(f"far from the origin d={d} offset={offset:g}")
    oi, od = oracle.knn_brute(x, q, 16)
    t = kdt.build(to_dev(x), leaf_size=64)
    gi, gd = t.knn(to_dev(q), 16, traversal=2)
    np.testing.assert_array_equal(to_host(gi), oi)
    np.testing.assert_array_equal(to_host(gd), od)
    gi, gd = t.knn(None, 16, traversal=2)
    oi, od = oracle.knn_brute(x, x, 16)
    np.testing.assert_array_equal(to_host(gi), oi)
    np.testing.assert_array_equal(to_host(gd), od)
