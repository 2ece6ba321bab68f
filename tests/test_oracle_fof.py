"""Pins for the oracle's friends-of-friends grouping (Sec. 4.1)."""
import numpy as np
import pytest

import oracle
from tests import cases, golden_io


@pytest.mark.parametrize("kind", cases.KINDS)
@pytest.mark.parametrize("d", (2, 3, 8))
def test_tree_fof_equals_brute_force(kind, d):
    for n in (1, 2, 33, 700):
        x = cases.points(kind, n, d, seed=3 * n + d)
        t = oracle.Tree(x, 8)
        for l in (0.0, 0.03, 0.1, 0.3):
            np.testing.assert_array_equal(t.fof(l), oracle.fof_brute(x, l))


def test_hand_derived_example():
    x, l, expect = golden_io.fof_groups()
    np.testing.assert_array_equal(oracle.fof_brute(x, l), expect)
    np.testing.assert_array_equal(oracle.Tree(x, 1).fof(l), expect)


def test_zero_length_groups_exact_duplicates():
    x = cases.points("duplicates", 500, 3, seed=11)
    lab = oracle.Tree(x, 8).fof(0.0)
    for i in range(500):
        same = np.nonzero((x == x[i]).all(axis=1))[0]
        assert lab[i] == same.min()


def test_length_above_diameter_gives_one_group():
    x = cases.points("uniform", 800, 3, seed=12)
    lab = oracle.Tree(x, 8).fof(2.0)
    assert (lab == 0).all()


def test_invariants_clustered():
    from paper_2609_18316_amd import workloads
    n = 20000
    x = workloads.clustered(n, seed=13)
    l = float(np.float32(0.2 * (1.0 / n) ** (1.0 / 3.0)))
    t = oracle.Tree(x, 32)
    lab = t.fof(l)
    i = np.arange(n)
    assert (lab <= i).all()
    assert (lab[lab] == lab).all()
    c, off, lst = t.range(x, l, lists=True)
    owner = np.repeat(i, c)
    assert (lab[owner] == lab[lst]).all()
    # a group's label is one of its members and is its smallest index
    for g in np.unique(lab)[:200]:
        members = np.nonzero(lab == g)[0]
        assert members.min() == g


def test_chain_threshold_is_inclusive():
    x = np.zeros((10, 2), np.float32)
    x[:, 0] = np.arange(10, dtype=np.float32) * np.float32(0.125)
    perm = np.random.Generator(np.random.PCG64(1)).permutation(10)
    x = x[perm]
    assert (oracle.fof_brute(x, 0.125) == 0).all()
    below = float(np.nextafter(np.float32(0.125), np.float32(0)))
    np.testing.assert_array_equal(oracle.fof_brute(x, below), np.arange(10))
