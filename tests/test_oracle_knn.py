"""Pins for the oracle's kNN (Sec. 2.3, Algorithm 2) against what the
mathematics fixes: brute force, a full sort, exact integer lattice distances
and a hand-derived example."""
import numpy as np
import pytest

import oracle
from tests import cases, golden_io

SIZES = (1, 2, 7, 31, 32, 33, 100, 1000)


@pytest.mark.parametrize("kind", cases.KINDS)
@pytest.mark.parametrize("d", (2, 3, 4, 8, 16))
def test_tree_knn_equals_brute_force(kind, d):
    for n in SIZES:
        x = cases.points(kind, n, d, seed=10 * n + d)
        q = np.concatenate([x[: min(n, 40)], cases.points(kind, 20, d, seed=999 + d)])
        for leaf in (1, 4, 16):
            t = oracle.Tree(x, leaf)
            for k in sorted({1, 8, 32, n, n + 3}):
                it, dt = t.knn(q, k)
                ib, db = oracle.knn_brute(x, q, k)
                np.testing.assert_array_equal(it, ib)
                np.testing.assert_array_equal(dt, db)


def test_k_equals_n_is_a_full_sort():
    """With k = n the answer is every point, sorted by (d2, index)."""
    x = cases.points("lattice", 300, 3, seed=5)
    q = cases.points("lattice", 25, 3, seed=6)
    idx, d2 = oracle.Tree(x, 8).knn(q, x.shape[0])
    for s in range(q.shape[0]):
        dd = np.array([oracle.sq_dist(x[i], q[s]) for i in range(x.shape[0])], np.float32)
        order = np.lexsort((np.arange(x.shape[0]), dd))
        np.testing.assert_array_equal(idx[s], order)
        np.testing.assert_array_equal(d2[s], dd[order])


def test_lattice_distances_match_integer_arithmetic():
    """On a 1/16 lattice every float32 squared distance is exact, so the
    result must equal the one computed with integer arithmetic."""
    rng = np.random.Generator(np.random.PCG64(3))
    for d in (2, 3, 8, 16):
        xi = rng.integers(0, 16, (500, d))
        qi = rng.integers(0, 16, (40, d))
        x = (xi / 16.0).astype(np.float32)
        q = (qi / 16.0).astype(np.float32)
        k = 12
        idx, d2 = oracle.Tree(x, 8).knn(q, k)
        for s in range(q.shape[0]):
            di = ((xi - qi[s]) ** 2).sum(axis=1)
            order = np.lexsort((np.arange(len(di)), di))[:k]
            np.testing.assert_array_equal(idx[s], order)
            np.testing.assert_array_equal(d2[s].astype(np.float64) * 256.0, di[order])


def test_hand_derived_example():
    pts, rows = golden_io.knn_line()
    t = oracle.Tree(pts, 1)
    for qv, k, iv, dv in rows:
        for idx, d2 in (t.knn(qv[None, :], k), oracle.knn_brute(pts, qv[None, :], k)):
            np.testing.assert_array_equal(idx[0], iv)
            np.testing.assert_array_equal(d2[0], dv)


def test_padding_when_k_exceeds_n():
    x = cases.points("uniform", 5, 3, seed=1)
    idx, d2 = oracle.Tree(x, 2).knn(x, 9)
    assert (idx[:, 5:] == -1).all() and np.isinf(d2[:, 5:]).all()
    assert sorted(idx[0, :5]) == list(range(5))


def test_invariants_on_clustered_points():
    from paper_2609_18316_amd import workloads
    x = workloads.clustered(20000, seed=7)
    q = workloads.uniform(500, 3, seed=8)
    k = 32
    idx, d2 = oracle.Tree(x, 32).knn(q, k)
    # rows ascending by (d2, idx)
    for s in range(q.shape[0]):
        keys = list(zip(d2[s].tolist(), idx[s].tolist()))
        assert keys == sorted(keys)
        assert len(set(idx[s].tolist())) == k
    # a closed ball through the k-th neighbour holds at least k points
    cnt = oracle.range_brute(x, q[:50], 0.0)
    assert (cnt == 0).all()
    for s in range(50):
        r = np.float32(np.sqrt(np.float64(d2[s, -1])))
        while np.float32(r * r) < d2[s, -1]:
            r = np.nextafter(r, np.float32(np.inf))
        assert oracle.range_brute(x, q[s:s + 1], float(r))[0] >= k
    ib, db = oracle.knn_brute(x, q[:50], k)
    np.testing.assert_array_equal(idx[:50], ib)
    np.testing.assert_array_equal(d2[:50], db)


def test_large_k_lattice_ties_match_integer_arithmetic():
    """k well above 64 on a coarse 1/8 lattice, where most distances tie: the
    order is (exact integer d2, index), as the definition fixes."""
    rng = np.random.Generator(np.random.PCG64(8))
    xi = rng.integers(0, 8, (900, 3))
    qi = rng.integers(0, 8, (30, 3))
    x = (xi / 8.0).astype(np.float32)
    q = (qi / 8.0).astype(np.float32)
    for k in (65, 300, 900, 905):
        idx, d2 = oracle.knn_brute(x, q, k)
        for s in range(q.shape[0]):
            di = ((xi - qi[s]) ** 2).sum(axis=1)
            order = np.lexsort((np.arange(len(di)), di))[:k]
            m = len(order)
            np.testing.assert_array_equal(idx[s, :m], order)
            np.testing.assert_array_equal(d2[s, :m].astype(np.float64) * 64.0, di[order])
            assert np.all(idx[s, m:] == -1) and np.all(np.isinf(d2[s, m:]))


def test_query_slices_on_threads_change_nothing():
    """The oracle's queries may run in contiguous slices on host threads (the
    CPU baseline and the large parity checks do): results are the same."""
    rng = np.random.Generator(np.random.PCG64(77))
    x = rng.random((3000, 3), dtype=np.float32)
    q = rng.random((1001, 3), dtype=np.float32)
    t = oracle.Tree(x, 8)
    for a, b in zip(t.knn(q, 9), t.knn(q, 9, threads=7)):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(t.range(q, 0.05), t.range(q, 0.05, threads=5))
    for a, b in zip(oracle.knn_brute(x, q, 4), oracle.knn_brute(x, q, 4, threads=3)):
        np.testing.assert_array_equal(a, b)
