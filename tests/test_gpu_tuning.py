"""leaf_size = 0 and traversal = 0 through the C ABI: the library's tuning
table (what kdt_tuning_get reports) decides the leaf size of kdt_build and the
traversal of kdt_knn, kdt_tuning_set replaces an entry for the process, and a
batched plan with leaf_size 0 gives every set the leaf size of its own size.
Results never depend on the choice: each case is checked against the
oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_18316_amd import autotune, kdt, workloads
from tests.gpu_util import dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _levels(n, leaf):
    L = 0
    while -(-n // (1 << L)) > leaf:
        L += 1
    return L


def test_table_lookup_matches_the_stored_table():
    dev()
    for name, e in autotune.load_table().items():
        d, l2, k, kind = autotune._parse_key(name)
        leaf, qpw, depth = kdt.tuning_get(d, 1 << l2, k)
        # the preferred kind of each shape is the one compiled in first
        same = [v for nm, v in autotune.load_table().items() if autotune._parse_key(nm)[:3] == (d, l2, k)]
        assert (leaf, qpw) in [(v["leaf_size"], v["queries_per_wave"]) for v in same], name
        assert depth == _levels(1 << l2, leaf) + 1


def test_zero_leaf_size_builds_with_the_tuned_leaf():
    dev()
    x = workloads.clustered(20011, 3)
    q = workloads.uniform(1500, 3, 4)
    ot = oracle.Tree(x, 8)
    oi, od = ot.knn(q, 8)
    try:
        _tuned_builds(x, q, oi, od)
    finally:
        kdt.tuning_set(3, 20011, 8, 0, 0)
    with pytest.raises(kdt.KdtError):
        kdt.tuning_set(3, 100, 8, 1, 1)
    with pytest.raises(kdt.KdtError):
        kdt.tuning_set(5, 100, 8, 16, 1)
    with pytest.raises(kdt.KdtError):
        kdt.tuning_set(3, 100, 8, 16, 32)


def _tuned_builds(x, q, oi, od):
    for leaf, qpw in ((12, 64), (40, 1), (7, 64)):
        kdt.tuning_set(3, 20011, 8, leaf, qpw)
        assert kdt.tuning_get(3, 20011, 8)[:2] == (leaf, qpw)
        t = kdt.build(to_dev(x), leaf_size=0, tune_k=8)
        say(f"tuned leaf {leaf}, {qpw} queries per traversal: tree leaf {t.info.leaf_size}")
        assert t.info.leaf_size == leaf and t.info.levels == _levels(20011, leaf)
        gi, gd = t.knn(to_dev(q), 8)  # traversal 0: the tuned one
        np.testing.assert_array_equal(to_host(gi), oi)
        np.testing.assert_array_equal(to_host(gd), od)
        t.close()


def test_batch_plan_with_tuned_leaf_per_set():
    dev()
    sizes = np.array([900, 5000, 20000, 70000, 1500], np.int64)
    buckets = list(zip((10, 12, 14, 16), (8, 16, 24, 48)))
    for e, leaf in buckets:
        kdt.tuning_set(3, 1 << e, 8, leaf, 64)
    try:
        _batch_with_tuned_leaves(sizes)
    finally:
        for e, _ in buckets:
            kdt.tuning_set(3, 1 << e, 8, 0, 0)


def _batch_with_tuned_leaves(sizes):
    x, off = workloads.batched_clustered(sizes, 7000)
    lens = np.array([np.float32(0.2 * n ** (-1.0 / 3.0)) for n in sizes], np.float32)
    plan = kdt.BatchPlan(off, 3, 8, leaf_size=0)
    xt, lt = to_dev(x), to_dev(lens)
    for use_graph in (1, 2, 0):
        say(f"batched plan, per-set tuned leaves, use_graph={use_graph}")
        idx, d2, lab = plan.launch(xt, lt, use_graph=use_graph)
        idx, d2, lab = to_host(idx), to_host(d2), to_host(lab)
        for s in range(len(sizes)):
            a, b = off[s], off[s + 1]
            oi, od = oracle.knn_brute(x[a:b], x[a:b], 8) if b - a <= 5000 else \
                oracle.Tree(x[a:b], 16).knn(x[a:b], 8)
            np.testing.assert_array_equal(idx[a:b], oi)
            np.testing.assert_array_equal(d2[a:b], od)
            np.testing.assert_array_equal(lab[a:b], oracle.Tree(x[a:b], 16).fof(float(lens[s])))
    plan.close()
