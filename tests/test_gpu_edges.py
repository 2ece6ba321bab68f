"""Edge cases through the C ABI: empty query and particle sets, a one-point
tree, queries far outside the tree's box (down to squared distances that
overflow to +inf), and degenerate batches."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_18316_amd import kdt, workloads
from tests.gpu_util import dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_empty_query_sets_are_no_ops():
    d = dev()
    x = workloads.uniform(1000, 3, seed=21)
    t = kdt.build(to_dev(x))
    q = torch.empty((0, 3), dtype=torch.float32, device=d)
    for trav in (0, 1, 2):
        idx, d2 = t.knn(q, 8, traversal=trav)
        assert idx.shape == (0, 8) and d2.shape == (0, 8)
        assert t.knn(q, 8, kth_only=2, traversal=trav).shape == (0,)
    assert t.range(q, 0.1).shape == (0,)
    c, off, lst = t.range(q, 0.1, lists=True)
    assert c.numel() == 0 and to_host(off).tolist() == [0] and lst.numel() == 0
    for kind in (0, 1):
        assert t.query_order(q, kind=kind).shape == (0,)
    with pytest.raises(kdt.KdtError):  # k is still checked
        t.knn(q, 0)


def test_empty_particle_set_gives_an_empty_mesh():
    d = dev()
    z3 = torch.empty((0, 3), dtype=torch.float32, device=d)
    z = torch.empty(0, dtype=torch.float32, device=d)
    rho = kdt.p2m(z3, z, z, (0, 0, 0), 1 / 16, (16, 16, 16))
    assert rho.shape == (16, 16, 16) and (to_host(rho) == 0).all()
    gm, gx = kdt.p2m_backward(z3, z, z, (0, 0, 0), 1 / 16, (16, 16, 16),
                              torch.ones((16, 16, 16), device=d))
    assert gm.shape == (0,) and gx.shape == (0, 3)


def test_one_point_tree():
    dev()
    x = np.array([[0.25, 0.5, 0.75]], np.float32)
    t = kdt.build(to_dev(x))
    assert t.info.levels == 0
    idx, d2 = t.knn(None, 3)
    np.testing.assert_array_equal(to_host(idx), [[0, -1, -1]])
    np.testing.assert_array_equal(to_host(d2), [[0.0, np.inf, np.inf]])
    q = workloads.uniform(100, 3, seed=22)
    oi, od = oracle.Tree(x, 32).knn(q, 2)
    for trav in (1, 2):
        gi, gd = t.knn(to_dev(q), 2, traversal=trav)
        np.testing.assert_array_equal(to_host(gi), oi)
        np.testing.assert_array_equal(to_host(gd), od)
    np.testing.assert_array_equal(to_host(t.range(to_dev(q), 0.3)), oracle.range_brute(x, q, 0.3))
    np.testing.assert_array_equal(to_host(t.fof(0.1)), [0])


@pytest.mark.parametrize("scale", (1e3, 1e19, 1e30))
def test_queries_far_outside_the_box(scale):
    """Far queries: the Hilbert key clamps them to the box edge, every node is
    far, and at 1e19 / 1e30 the float32 squared distances overflow to +inf,
    where ties are decided by the index alone."""
    dev()
    x = workloads.clustered(5000, seed=23)
    rng = np.random.Generator(np.random.PCG64(24))
    q = (rng.standard_normal((300, 3)) * scale).astype(np.float32)
    say(f"far queries at scale {scale:g}")
    t = kdt.build(to_dev(x))
    oi, od = oracle.knn_brute(x, q, 8)
    for trav in (1, 2):
        gi, gd = t.knn(to_dev(q), 8, traversal=trav)
        np.testing.assert_array_equal(to_host(gi), oi)
        np.testing.assert_array_equal(to_host(gd), od)
    r = float(scale) * 3
    np.testing.assert_array_equal(to_host(t.range(to_dev(q), r)), oracle.range_brute(x, q, r))


def test_batch_degenerate_sets():
    dev()
    off = np.array([0, 3, 3, 10], np.int64)  # the second set is empty
    with pytest.raises(kdt.KdtError) as e:
        kdt.BatchPlan(off, 3, 4)
    assert e.value.status == kdt.KDT_EINVAL
    # single points and tiny sets: k larger than every set pads each row
    sizes = [1, 2, 5]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = workloads.uniform(int(off[-1]), 3, seed=25)
    plan = kdt.BatchPlan(off, 3, 8)
    lens = to_dev(np.full(len(sizes), 0.5, np.float32))
    idx, d2, lab = (to_host(a) for a in plan.launch(to_dev(x), lens))
    for s, n in enumerate(sizes):
        xs = x[off[s]:off[s + 1]]
        oi, od = oracle.knn_brute(xs, xs, 8)
        np.testing.assert_array_equal(idx[off[s]:off[s + 1]], oi)
        np.testing.assert_array_equal(d2[off[s]:off[s + 1]], od)
        np.testing.assert_array_equal(lab[off[s]:off[s + 1]], oracle.fof_brute(xs, 0.5))
    plan.close()
