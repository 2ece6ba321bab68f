"""kdt_knn_noalloc -- kNN whose only scratch (the query order) lives in the
library's static device array -- must give exactly what kdt_knn gives, call
after call (the array keeps the previous call's contents), and refuse what
does not fit with a clear error."""
import numpy as np
import pytest
import torch

from paper_2609_18316_amd import kdt, workloads
from tests.gpu_util import dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _points(d, n, seed):
    return workloads.clustered(n, seed) if d == 3 else workloads.uniform(n, d, seed)


def _noalloc(tree, q, k, kth_only=0, **kw):
    nq = tree.n if q is None else q.shape[0]
    d2 = torch.empty((nq,) if kth_only else (nq, k), dtype=torch.float32, device=dev())
    idx = None if kth_only else torch.empty((nq, k), dtype=torch.int32, device=dev())
    tree.knn_noalloc(q, k, d2, idx, kth_only=kth_only, **kw)
    return d2 if kth_only else (idx, d2)


def _same(a, b):
    if isinstance(a, tuple):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(to_host(x), to_host(y))
    else:
        np.testing.assert_array_equal(to_host(a), to_host(b))


@pytest.mark.parametrize("d,leaf,traversal,k", ((3, 32, 0, 32), (3, 32, 2, 8), (8, 24, 1, 16),
                                                (16, 64, 0, 16), (2, 16, 0, 64)))
def test_noalloc_equals_knn_on_consecutive_calls(d, leaf, traversal, k):
    """Two calls in a row, the second with fewer queries (the scratch still
    holds the first call's keys), plus k-th-only and self queries."""
    tree = kdt.build(to_dev(_points(d, 60000, 21 + d)), leaf_size=leaf)
    for nq, seed in ((50000, 31), (3001, 32), (1, 33)):
        q = to_dev(workloads.uniform(nq, d, seed + d))
        say(f"noalloc d={d} leaf={leaf} traversal={traversal} k={k} nq={nq}")
        _same(_noalloc(tree, q, k, traversal=traversal), tree.knn(q, k, traversal=traversal))
        _same(_noalloc(tree, q, k, kth_only=2, traversal=traversal),
              tree.knn(q, k, kth_only=2, traversal=traversal))
        _same(_noalloc(tree, q, k, sort_queries=False, traversal=traversal),
              tree.knn(q, k, sort_queries=False, traversal=traversal))
    _same(_noalloc(tree, None, k, traversal=traversal), tree.knn(None, k, traversal=traversal))
    tree.close()


def test_noalloc_at_its_limit_and_beyond():
    """KDT_NOALLOC_MAX_SORTED queries are ordered in the static scratch; one
    more is refused unless the queries need no ordering."""
    dev()
    lim = kdt.NOALLOC_MAX_SORTED
    x = _points(3, 1 << 20, 41)
    tree = kdt.build(to_dev(x), leaf_size=32)
    q = to_dev(workloads.uniform(lim + 1, 3, 42))
    say(f"noalloc limit nq={lim}")
    _same(_noalloc(tree, q[:lim], 8), tree.knn(q[:lim], 8))
    say(f"noalloc beyond the limit nq={lim + 1}")
    with pytest.raises(kdt.KdtError) as e:
        _noalloc(tree, q, 8)
    assert e.value.status == kdt.KDT_ECAPACITY
    _same(_noalloc(tree, q, 8, sort_queries=False), tree.knn(q, 8, sort_queries=False))
    order = tree.query_order(q)
    _same(_noalloc(tree, q, 8, order=order), tree.knn(q, 8))
    # a smaller call after the failed one still matches
    _same(_noalloc(tree, q[:777], 8), tree.knn(q[:777], 8))
    tree.close()


def test_noalloc_refuses_what_would_allocate():
    dev()
    x = _points(3, 5000, 51)
    tree = kdt.build(to_dev(x))
    q = to_dev(workloads.uniform(100, 3, 52))
    with pytest.raises(kdt.KdtError) as e:
        _noalloc(tree, q, 65)
    assert e.value.status == kdt.KDT_EUNSUPPORTED
    opts = kdt.QueryOpts(1, 0, None, 0, kdt._periods(1.0, 3))
    d2 = torch.empty((100, 8), dtype=torch.float32, device=dev())
    rc = kdt.load().kdt_knn_noalloc(tree._h, kdt._ptr(q), 100, 8, None, kdt._ptr(d2), 0,
                                    kdt.C.byref(opts), kdt._stream())
    assert rc == kdt.KDT_EUNSUPPORTED
    # an empty query set is fine and touches nothing
    tree.knn_noalloc(q[:0], 8, torch.empty((0, 8), dtype=torch.float32, device=dev()))
    tree.close()
