"""GPU parity for kNN with k above the 64 register entries (the ball-and-sort
path; Sec. 3.3 measures k up to 10^4) against the oracle's brute force on the
same seeded inputs: identical (index, d2) lists, k-th-only modes, padding when
k exceeds n, degenerate point sets, clustered data and query orders."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_18316_amd import kdt, workloads
from tests import cases
from tests.gpu_util import dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _check(t, x, q, k):
    """External queries (q) and self queries against brute force, all modes."""
    for queries, ref in ((q, q), (None, x)):
        oi, od = oracle.knn_brute(x, ref, k)
        arg = None if queries is None else to_dev(queries)
        gi, gd = t.knn(arg, k)
        np.testing.assert_array_equal(to_host(gi), oi)
        np.testing.assert_array_equal(to_host(gd), od)
        np.testing.assert_array_equal(to_host(t.knn(arg, k, kth_only=1)), od[:, -1])
        np.testing.assert_array_equal(to_host(t.knn(arg, k, kth_only=2)), np.sqrt(od[:, -1]))


@pytest.mark.parametrize("d", kdt.DIMS)
@pytest.mark.parametrize("kind", cases.KINDS)
def test_large_k_equals_brute_force(kind, d):
    dev()
    for n in (1, 70, 3001):
        x = cases.points(kind, n, d, seed=7 * n + d)
        q = cases.points(kind, 200, d, seed=13 * n + d)
        t = kdt.build(to_dev(x), leaf_size=16)
        for k in sorted({65, 100, 257, n + 3}):
            if k <= kdt.MAX_K:
                continue
            say(f"large k d={d} kind={kind} n={n} k={k}")
            if n <= 1200:
                _check(t, x, q, k)
            else:
                # self queries of all n points would take the oracle long: sample rows
                oi, od = oracle.knn_brute(x, q, k)
                gi, gd = t.knn(to_dev(q), k)
                np.testing.assert_array_equal(to_host(gi), oi)
                np.testing.assert_array_equal(to_host(gd), od)
                rows = workloads.sample_indices(n, 300, seed=k)
                si, sd = t.knn(None, k)
                oi, od = oracle.knn_brute(x, x[rows], k)
                np.testing.assert_array_equal(to_host(si)[rows], oi)
                np.testing.assert_array_equal(to_host(sd)[rows], od)
                kth = to_host(t.knn(None, k, kth_only=1))
                np.testing.assert_array_equal(kth[rows], od[:, -1])


def test_large_k_clustered_leaf_sizes():
    """Clustered mock-catalogue points: radii from the 64th neighbour are far
    too small or large in places, so the growth rounds and chunking matter."""
    dev()
    x = workloads.clustered(40000, seed=17)
    q = np.concatenate([x[workloads.sample_indices(40000, 200, seed=3)],
                        workloads.uniform(100, 3, seed=4)])
    ref = {k: oracle.knn_brute(x, q, k) for k in (65, 500, 2000)}
    for leaf in (8, 32, 100):
        t = kdt.build(to_dev(x), leaf_size=leaf)
        for k, (oi, od) in ref.items():
            say(f"large k clustered leaf={leaf} k={k}")
            gi, gd = t.knn(to_dev(q), k)
            np.testing.assert_array_equal(to_host(gi), oi)
            np.testing.assert_array_equal(to_host(gd), od)


def test_large_k_far_queries_and_identical_points():
    """Queries far outside the root box, and a tree of identical points (the
    64th-neighbour radius is zero there)."""
    dev()
    x = workloads.uniform(5000, 3, seed=21)
    q = (workloads.uniform(50, 3, seed=22) * 1e4 + 1e5).astype(np.float32)
    t = kdt.build(to_dev(x), leaf_size=16)
    say("large k far queries")
    oi, od = oracle.knn_brute(x, q, 300)
    gi, gd = t.knn(to_dev(q), 300)
    np.testing.assert_array_equal(to_host(gi), oi)
    np.testing.assert_array_equal(to_host(gd), od)
    same = np.full((700, 2), 0.25, np.float32)
    t = kdt.build(to_dev(same), leaf_size=8)
    for k in (65, 700, 701):
        say(f"large k identical points k={k}")
        oi, od = oracle.knn_brute(same, same, k)
        gi, gd = t.knn(None, k)
        np.testing.assert_array_equal(to_host(gi), oi)
        np.testing.assert_array_equal(to_host(gd), od)


def test_large_k_query_orders_agree():
    """Sorted, unsorted and caller-given query orders give the same rows."""
    dev()
    x = workloads.normal(20000, 3, seed=31)
    q = workloads.normal(3000, 3, seed=32)
    t = kdt.build(to_dev(x), leaf_size=32)
    say("large k query orders")
    oi, od = oracle.knn_brute(x, q, 129)
    qd = to_dev(q)
    order = t.query_order(qd, kind=0)
    for kw in ({}, {"sort_queries": False}, {"order": order}):
        gi, gd = t.knn(qd, 129, **kw)
        np.testing.assert_array_equal(to_host(gi), oi)
        np.testing.assert_array_equal(to_host(gd), od)


def test_large_k_limits_and_empty():
    dev()
    x = workloads.uniform(100, 3, seed=1)
    t = kdt.build(to_dev(x))
    with pytest.raises(kdt.KdtError) as e:
        t.knn(None, kdt.MAX_K_SORTED + 1, kth_only=1)
    assert e.value.status == kdt.KDT_EUNSUPPORTED
    q = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    gi, gd = t.knn(q, 1000)
    assert gi.shape == (0, 1000) and gd.shape == (0, 1000)


def test_large_k_lattice_ties():
    """A coarse lattice where most distances tie: ties at and across the k-th
    place are broken by index, as in the oracle."""
    dev()
    rng = np.random.Generator(np.random.PCG64(8))
    x = (rng.integers(0, 8, (20000, 3)) / 8.0).astype(np.float32)
    q = (rng.integers(0, 8, (500, 3)) / 8.0).astype(np.float32)
    t = kdt.build(to_dev(x), leaf_size=32)
    for k in (65, 1000, 5000):
        say(f"large k lattice ties k={k}")
        oi, od = oracle.knn_brute(x, q, k)
        gi, gd = t.knn(to_dev(q), k)
        np.testing.assert_array_equal(to_host(gi), oi)
        np.testing.assert_array_equal(to_host(gd), od)
        # the k-th distance alone is selected, not sorted: equal distances at
        # and around the k-th place are the hard case
        np.testing.assert_array_equal(to_host(t.knn(to_dev(q), k, kth_only=1)), od[:, -1])
        np.testing.assert_array_equal(to_host(t.knn(to_dev(q), k, kth_only=2)),
                                      np.sqrt(od[:, -1]))


def test_large_k_rows_beyond_the_lds_sort():
    """Rows whose candidate ball holds more keys than one workgroup sorts in
    LDS (16384): the k smallest are selected first.  Coincident points (the
    ball of every query holds them all) and a 1/32 lattice (masses of equal
    distances, ties by index) at k = 1000 and 9000; also k = 16384 itself."""
    dev()
    rng = np.random.Generator(np.random.PCG64(77))
    same = np.full((20000, 3), 0.5, np.float32)
    lat = (rng.integers(0, 8, size=(40000, 3)) / 32.0).astype(np.float32)
    for x, ks in ((same, (1000, 9000, 16384)), (lat, (1000, 9000))):
        q = np.concatenate([x[:20], (rng.integers(0, 8, size=(20, 3)) / 32.0 + 1 / 64.0)
                            .astype(np.float32)])
        t = kdt.build(to_dev(x), leaf_size=32)
        for k in ks:
            say(f"large k={k} on {len(x)} points with wide candidate rows")
            oi, od = oracle.knn_brute(x, q, k)
            gi, gd = t.knn(to_dev(q), k)
            np.testing.assert_array_equal(to_host(gi), oi)
            np.testing.assert_array_equal(to_host(gd), od)
        t.close()


def test_large_k_rows_beyond_the_register_select():
    """Rows of more than 32768 candidate keys, more than the widest row sort
    holds in registers: the select reads them from global memory each digit
    pass and stops once the kept keys fit the sort.  40000 coincident points
    (every key ties on distance: the passes go down into the index bits) and
    a tight cluster of 40000 seen from afar (the whole cluster is in every
    ball, distinct distances); k = 1000, 9000 and 16384."""
    dev()
    rng = np.random.Generator(np.random.PCG64(78))
    same = np.full((40000, 3), 0.25, np.float32)
    tight = (0.5 + 1e-3 * rng.standard_normal((40000, 3))).astype(np.float32)
    far = np.array([[0.9, 0.1, 0.2], [0.05, 0.95, 0.5], [0.5, 0.5, 0.98]], np.float32)
    for x, q in ((same, np.concatenate([same[:4], far])), (tight, far)):
        t = kdt.build(to_dev(x), leaf_size=32)
        for k in (1000, 9000, 16384):
            say(f"large k={k} on {len(x)} points, every ball holding all of them")
            oi, od = oracle.knn_brute(x, q, k)
            gi, gd = t.knn(to_dev(q), k)
            np.testing.assert_array_equal(to_host(gi), oi)
            np.testing.assert_array_equal(to_host(gd), od)
        t.close()
