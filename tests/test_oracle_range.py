"""Pins for the oracle's ball query (Sec. 2.3, Algorithm 3)."""
import numpy as np
import pytest

import oracle
from tests import cases, golden_io


@pytest.mark.parametrize("kind", cases.KINDS)
@pytest.mark.parametrize("d", (2, 3, 4, 8, 16))
def test_tree_range_equals_brute_force(kind, d):
    for n in (1, 7, 33, 1000):
        x = cases.points(kind, n, d, seed=7 * n + d)
        q = np.concatenate([x[: min(n, 30)], cases.points(kind, 15, d, seed=77 + d)])
        for leaf in (1, 16):
            t = oracle.Tree(x, leaf)
            for r in (0.0, 0.05, 0.2, 0.5, 3.0):
                ct, ot, lt = t.range(q, r, lists=True)
                cb, ob, lb = oracle.range_brute(x, q, r, lists=True)
                np.testing.assert_array_equal(ct, cb)
                np.testing.assert_array_equal(ot, ob)
                np.testing.assert_array_equal(lt, lb)


def test_lattice_counts_closed_form():
    """Ball counts around an interior point of Z^3 equal 1 + sum r3(m)."""
    g = np.arange(-4, 5)
    grid = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    x = (grid / 16.0).astype(np.float32)
    q = np.zeros((1, 3), np.float32)
    t = oracle.Tree(x, 4)
    for r2, expect in golden_io.range_lattice():
        r = np.float32(np.sqrt(r2 + 0.5) / 16.0)
        assert t.range(q, float(r))[0] == expect
        assert oracle.range_brute(x, q, float(r))[0] == expect


def test_infinite_and_zero_radius():
    x = cases.points("duplicates", 400, 3, seed=2)
    t = oracle.Tree(x, 8)
    assert (t.range(x, np.inf) == 400).all()
    mult = np.array([(x == x[i]).all(axis=1).sum() for i in range(400)])
    np.testing.assert_array_equal(t.range(x, 0.0), mult)


def test_self_query_sum_is_n_plus_twice_the_pairs():
    """With queries = points, sum of counts = n + 2 #{i<j : d2 <= r^2}."""
    rng = np.random.Generator(np.random.PCG64(4))
    xi = rng.integers(0, 32, (600, 3))
    x = (xi / 32.0).astype(np.float32)
    r2_int = 9  # (3/32)^2, exact
    r = float(np.float32(3.0 / 32.0))
    diff = xi[:, None, :] - xi[None, :, :]
    di = (diff ** 2).sum(-1)
    pairs = int(np.triu(di <= r2_int, 1).sum())
    counts = oracle.Tree(x, 16).range(x, r)
    assert int(counts.sum()) == 600 + 2 * pairs


def test_lists_sorted_and_consistent_with_knn():
    from paper_2609_18316_amd import workloads
    x = workloads.clustered(30000, seed=3)
    q = workloads.uniform(300, 3, seed=4)
    t = oracle.Tree(x, 32)
    c, off, lst = t.range(q, 0.02, lists=True)
    for s in range(q.shape[0]):
        row = lst[off[s]:off[s + 1]]
        assert (np.diff(row) > 0).all()
    k = 5
    idx, d2 = t.knn(q, k)
    r2 = np.float32(0.02) * np.float32(0.02)
    for s in range(q.shape[0]):
        inside = d2[s] <= r2
        row = set(lst[off[s]:off[s + 1]].tolist())
        assert set(idx[s][inside].tolist()) <= row
        if c[s] >= k:
            assert inside.all()
