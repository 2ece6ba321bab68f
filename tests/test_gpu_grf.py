"""Queries on the paper's inhomogeneous mock (Sec. 3.1: particles placed by a
Gaussian-random-field density of spectral index -2): kNN, ball counts and
lists, and friends-of-friends at the paper's b = 0.03 and the batched
workload's b = 0.2, on median and sliding-midpoint trees, against the
oracle."""
import numpy as np
import pytest

import oracle
from paper_2609_18316_amd import kdt, workloads
from tests.gpu_util import dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu

T = oracle.host_threads()


@pytest.mark.parametrize("n", (20011, 200000))
@pytest.mark.parametrize("rule", (kdt.SPLIT_MEDIAN, kdt.SPLIT_MIDPOINT))
def test_queries_on_the_grf_mock(n, rule):
    dev()
    x = workloads.grf(n, 31)
    q = workloads.uniform(20000, 3, 32)
    ot = oracle.Tree(x, 16)
    t = kdt.build(to_dev(x), leaf_size=32, split_rule=rule)
    for k in (8, 32):
        say(f"GRF n={n} rule={rule} kNN k={k}")
        oi, od = ot.knn(q, k, threads=T)
        gi, gd = t.knn(to_dev(q), k)
        np.testing.assert_array_equal(to_host(gi), oi)
        np.testing.assert_array_equal(to_host(gd), od)
    oi, od = ot.knn(x, 32, threads=T)
    np.testing.assert_array_equal(to_host(t.knn(None, 32, kth_only=2)), np.sqrt(od[:, -1]))
    r = float(np.float32(2.0 * n ** (-1.0 / 3.0)))
    say(f"GRF n={n} rule={rule} balls r={r}")
    np.testing.assert_array_equal(to_host(t.range(to_dev(q), r)), ot.range(q, r, threads=T))
    oc, ooff, oidx = ot.range(q[:3000], r, lists=True)
    gc, goff, gidx = t.range(to_dev(q[:3000]), r, lists=True)
    np.testing.assert_array_equal(to_host(goff), ooff)
    np.testing.assert_array_equal(to_host(gidx), oidx)
    for b in (0.03, 0.2):
        l = float(np.float32(b * n ** (-1.0 / 3.0)))
        say(f"GRF n={n} rule={rule} FoF b={b}")
        np.testing.assert_array_equal(to_host(t.fof(l)), ot.fof(l))
    t.close()
