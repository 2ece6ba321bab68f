"""Work in tree order: self-query rows written in the tree's order
(tree_rows), per-point arrays moved between input and tree order (gather,
scatter), and the deposit and its adjoint over a tree's points with masses,
smoothing lengths and gradients in tree order (Sec. 4.2 on the particles as
the tree holds them).

Every result is compared with the oracle on the same seeded inputs, rows
permuted by the tree order: kNN and balls bit-exact, the deposit to its
tolerance (per cell |rho32 - rho64| <= 1e-5 max(|rho64|, mean cell mass),
total mass within 1e-5; dm to the same per-element rule, dx to 1e-4 in
relative L2 norm)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_18316_amd import kdt, workloads
from tests.gpu_util import dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu

RULES = (kdt.SPLIT_MEDIAN, kdt.SPLIT_MIDPOINT)


def _points(n, d, seed):
    x = workloads.clustered(n, seed)
    return x if d == 3 else np.ascontiguousarray(np.tile(x, (1, 6))[:, :d])


@pytest.mark.parametrize("d", (2, 3, 8))
@pytest.mark.parametrize("rule", RULES)
def test_knn_tree_rows_equal_the_oracle(d, rule):
    dev()
    for n in (1, 4097, 20011):
        x = _points(n, d, 50 + n + d)
        t = kdt.build(to_dev(x), leaf_size=16, split_rule=rule)
        perm = t.export()["perm"]
        xp = x[perm]
        for k in sorted({1, 8, min(33, n), 64}):
            oi, od = oracle.knn_brute(x, xp, k)
            for trav in (1, 2):
                say(f"tree-row kNN d={d} rule={rule} n={n} k={k} traversal={trav}")
                gi, gd = t.knn(None, k, traversal=trav, tree_rows=True)
                np.testing.assert_array_equal(to_host(gi), oi)
                np.testing.assert_array_equal(to_host(gd), od)
                kth = to_host(t.knn(None, k, kth_only=1, traversal=trav, tree_rows=True))
                np.testing.assert_array_equal(kth, od[:, k - 1])
                hs = to_host(t.knn(None, k, kth_only=2, traversal=trav, tree_rows=True))
                np.testing.assert_array_equal(hs, np.sqrt(od[:, k - 1]))
        t.close()


def test_knn_tree_rows_large_k_torus_and_noalloc():
    dev()
    n = 6000
    x = workloads.clustered(n, 61)
    t = kdt.build(to_dev(x), leaf_size=16)
    perm = t.export()["perm"]
    xp = x[perm]
    say("tree-row kNN k = 100 (ball-and-sort path)")
    oi, od = oracle.knn_brute(x, xp, 100)
    gi, gd = t.knn(None, 100, tree_rows=True)
    np.testing.assert_array_equal(to_host(gi), oi)
    np.testing.assert_array_equal(to_host(gd), od)
    say("tree-row kNN on the torus")
    oi, od = oracle.knn_brute(x, xp, 16, period=1.0)
    gi, gd = t.knn(None, 16, period=1.0, tree_rows=True)
    np.testing.assert_array_equal(to_host(gi), oi)
    np.testing.assert_array_equal(to_host(gd), od)
    say("tree-row kNN without allocation")
    oi, od = oracle.knn_brute(x, xp, 8)
    d2 = torch.empty((n, 8), dtype=torch.float32, device=dev())
    idx = torch.empty((n, 8), dtype=torch.int32, device=dev())
    t.knn_noalloc(None, 8, d2, idx, tree_rows=True)
    np.testing.assert_array_equal(to_host(idx), oi)
    np.testing.assert_array_equal(to_host(d2), od)
    t.close()


@pytest.mark.parametrize("rule", RULES)
def test_range_tree_rows_equal_the_oracle(rule):
    dev()
    n = 20011
    x = workloads.clustered(n, 71)
    t = kdt.build(to_dev(x), leaf_size=16, split_rule=rule)
    perm = t.export()["perm"]
    xp = x[perm]
    for r in (0.0, 0.004, 0.02):
        for trav in (1, 2):
            say(f"tree-row balls rule={rule} r={r} traversal={trav}")
            oc, ooff, oidx = oracle.range_brute(x, xp, r, lists=True)
            np.testing.assert_array_equal(to_host(t.range(None, r, traversal=trav,
                                                          tree_rows=True)), oc)
            gc, goff, gidx = t.range(None, r, lists=True, traversal=trav, tree_rows=True)
            np.testing.assert_array_equal(to_host(goff), ooff)
            np.testing.assert_array_equal(to_host(gidx), oidx)
    if rule == kdt.SPLIT_MEDIAN:
        say("tree-row balls on the torus")
        oc, ooff, oidx = oracle.range_brute(x, xp, 0.01, lists=True, period=1.0)
        gc, goff, gidx = t.range(None, 0.01, lists=True, period=1.0, tree_rows=True)
        np.testing.assert_array_equal(to_host(gc), oc)
        np.testing.assert_array_equal(to_host(goff), ooff)
        np.testing.assert_array_equal(to_host(gidx), oidx)
    t.close()


def test_f64_tree_rows_equal_the_oracle():
    dev()
    n = 5000
    rng = np.random.Generator(np.random.PCG64(81))
    x = rng.random((n, 3))
    t = kdt.build_f64(torch.from_numpy(x).to(dev()), leaf_size=16)
    perm = t.export()["perm"]
    oi, od = oracle.knn_brute_f64(x, x[perm], 12)
    gi, gd = t.knn(None, 12, tree_rows=True)
    np.testing.assert_array_equal(to_host(gi), oi)
    np.testing.assert_array_equal(to_host(gd), od)
    oc, ooff, oidx = oracle.range_brute_f64(x, x[perm], 0.03, lists=True)
    gc, goff, gidx = t.range(None, 0.03, lists=True, tree_rows=True)
    np.testing.assert_array_equal(to_host(gc), oc)
    np.testing.assert_array_equal(to_host(goff), ooff)
    np.testing.assert_array_equal(to_host(gidx), oidx)
    t.close()


def test_tree_rows_errors():
    dev()
    x = workloads.clustered(500, 91)
    t = kdt.build(to_dev(x), leaf_size=8)
    for call in (lambda: t.knn(to_dev(x[:5]), 4, tree_rows=True),
                 lambda: t.range(to_dev(x[:5]), 0.1, tree_rows=True)):
        with pytest.raises(kdt.KdtError) as e:
            call()
        assert e.value.status == kdt.KDT_EINVAL
    opts = kdt.QueryOpts(1, 0, None, 0, None, 2)
    d2 = torch.empty(500, dtype=torch.float32, device=dev())
    with pytest.raises(kdt.KdtError) as e:
        kdt._check(kdt.load().kdt_knn(t._h, None, 500, 4, None, kdt._ptr(d2), 1,
                                      kdt.C.byref(opts), kdt._stream()))
    assert e.value.status == kdt.KDT_EINVAL
    t.close()


@pytest.mark.parametrize("n", (1, 2, 4097, 300007))
def test_gather_and_scatter(n):
    dev()
    x = workloads.clustered(n, 100 + n)
    t = kdt.build(to_dev(x), leaf_size=16)
    perm = t.export()["perm"]
    rng = np.random.Generator(np.random.PCG64(n))
    for shape, dtype in (((n,), np.float32), ((n, 3), np.float32), ((n, 5), np.int32),
                         ((n, 1), np.int32)):
        say(f"gather/scatter n={n} shape={shape} {dtype.__name__}")
        a = rng.standard_normal(shape).astype(np.float32).view(np.float32)
        if dtype == np.int32:
            a = rng.integers(-2 ** 31, 2 ** 31, size=shape, dtype=np.int64).astype(np.int32)
        g = to_host(t.gather(to_dev(a)))
        np.testing.assert_array_equal(g, a[perm])
        back = to_host(t.scatter(to_dev(g)))
        np.testing.assert_array_equal(back, a)
    t.close()


def test_gather_errors():
    dev()
    x = workloads.clustered(100, 3)
    t = kdt.build(to_dev(x), leaf_size=8)
    a = to_dev(np.zeros(100, np.float32))
    for width in (0, 4097):
        with pytest.raises(kdt.KdtError) as e:
            kdt._check(kdt.load().kdt_tree_gather(t._h, kdt._ptr(a), width, kdt._ptr(a),
                                                  kdt._stream()))
        assert e.value.status == kdt.KDT_EINVAL
    with pytest.raises(kdt.KdtError) as e:  # in place
        kdt._check(kdt.load().kdt_tree_scatter(t._h, kdt._ptr(a), 1, kdt._ptr(a),
                                               kdt._stream()))
    assert e.value.status == kdt.KDT_EINVAL
    t.close()


# ---------------------------------------------------------------------------
# the deposit over a tree's points
# ---------------------------------------------------------------------------

def _close_rho(g, o, m_total):
    mean = m_total / o.size
    err = np.abs(g.astype(np.float64) - o)
    bound = 1e-5 * np.maximum(np.abs(o), mean)
    assert (err <= bound).all(), float((err / bound).max())
    assert abs(float(g.astype(np.float64).sum()) - m_total) <= 1e-5 * m_total


def _tree_setup(n, scale, seed, rule=kdt.SPLIT_MEDIAN, k=32):
    """Clustered points scaled to the box [0, scale), a tree over them, m in
    input order, h in tree order (tree-row k-th distances) and h in input
    order for the oracle."""
    x = (workloads.clustered(n, seed).astype(np.float64) * scale).astype(np.float32)
    x = np.minimum(x, np.nextafter(np.float32(scale), np.float32(0)))
    m = workloads.masses(n, seed + 1)
    t = kdt.build(to_dev(x), leaf_size=16, split_rule=rule)
    perm = t.export()["perm"]
    h_tree = t.knn(None, min(k, n), kth_only=2, tree_rows=True)
    h_in = np.empty(n, np.float32)
    h_in[perm] = to_host(h_tree)
    return x, m, t, perm, h_tree, h_in


@pytest.mark.parametrize("rule", RULES)
@pytest.mark.parametrize("n,cells", [(1, 16), (777, 16), (20000, 32), (300000, 64)])
def test_tree_deposit_matches_the_oracle(n, cells, rule):
    dev()
    say(f"tree deposit n={n} cells={cells} rule={rule}")
    x, m, t, perm, h_tree, h_in = _tree_setup(n, 1.0, 100 + n, rule)
    shape, lo, cell = (cells,) * 3, (0.0, 0.0, 0.0), 1.0 / cells
    o = oracle.p2m(x, m, h_in, lo, cell, shape)
    g = kdt.p2m_tree(t, t.gather(to_dev(m)), h_tree, lo, cell, shape)
    _close_rho(to_host(g), o, float(m.astype(np.float64).sum()))
    t.close()


@pytest.mark.parametrize("shape,cell", [((16, 16, 16), 1.0 / 16), ((32, 24, 40), 1.0 / 32)])
def test_tree_deposit_periodic_matches_the_oracle(shape, cell):
    dev()
    n = 20000
    L = np.array(shape, np.float64) * cell
    x = (workloads.clustered(n, 7).astype(np.float64) * L).astype(np.float32)
    x = np.minimum(x, np.nextafter(L.astype(np.float32), 0))
    m = workloads.masses(n, 8)
    t = kdt.build(to_dev(x), leaf_size=16)
    perm = t.export()["perm"]
    h_tree = torch.clamp(t.knn(None, 32, kth_only=2, tree_rows=True), max=float(0.45 * L.min()))
    h_in = np.empty(n, np.float32)
    h_in[perm] = to_host(h_tree)
    say(f"periodic tree deposit shape={shape}")
    o = oracle.p2m(x, m, h_in, (0, 0, 0), cell, shape, periodic=True)
    mt = t.gather(to_dev(m))
    g = kdt.p2m_tree(t, mt, h_tree, (0, 0, 0), cell, shape, periodic=True)
    _close_rho(to_host(g), o, float(m.astype(np.float64).sum()))
    rng = np.random.Generator(np.random.PCG64(9))
    up = rng.standard_normal(shape).astype(np.float32)
    om, ox = oracle.p2m_backward(x, m, h_in, (0, 0, 0), cell, shape, up, periodic=True)
    gm, gx = kdt.p2m_tree_backward(t, mt, h_tree, (0, 0, 0), cell, shape, to_dev(up),
                                   periodic=True)
    gm, gx = to_host(gm).astype(np.float64), to_host(gx).astype(np.float64)
    scale = np.abs(om).mean()
    assert (np.abs(gm - om[perm]) <= 1e-5 * np.maximum(np.abs(om[perm]), scale)).all()
    assert np.linalg.norm(gx - ox[perm]) <= 1e-4 * np.linalg.norm(ox)
    t.close()


@pytest.mark.parametrize("scheme", ("ngp", "cic", "tsc"))
@pytest.mark.parametrize("periodic", (False, True))
def test_tree_cloud_deposit_matches_the_oracle(scheme, periodic):
    dev()
    n, cells = 20000, 32
    x, m, t, perm, _, _ = _tree_setup(n, 1.0, 300, k=8)
    say(f"tree {scheme} deposit periodic={periodic}")
    o = oracle.p2m_cloud(x, m, (0, 0, 0), 1.0 / cells, (cells,) * 3, scheme, periodic=periodic)
    g = to_host(kdt.p2m_tree(t, t.gather(to_dev(m)), None, (0, 0, 0), 1.0 / cells, (cells,) * 3,
                             scheme=scheme, periodic=periodic))
    _close_rho(g, o, float(m.astype(np.float64).sum()))
    if scheme == "ngp":
        np.testing.assert_allclose(g, o, rtol=1e-6, atol=0)
    t.close()


@pytest.mark.parametrize("rule", RULES)
@pytest.mark.parametrize("n,cells", [(777, 16), (20000, 32)])
def test_tree_adjoint_matches_the_oracle(n, cells, rule):
    dev()
    say(f"tree adjoint n={n} cells={cells} rule={rule}")
    x, m, t, perm, h_tree, h_in = _tree_setup(n, 1.0, 200 + n, rule)
    shape, lo, cell = (cells,) * 3, (0.0, 0.0, 0.0), 1.0 / cells
    rng = np.random.Generator(np.random.PCG64(7))
    up = rng.standard_normal(shape).astype(np.float32)
    om, ox = oracle.p2m_backward(x, m, h_in, lo, cell, shape, up)
    gm, gx = kdt.p2m_tree_backward(t, t.gather(to_dev(m)), h_tree, lo, cell, shape, to_dev(up))
    # back in input order through the library's scatter
    gm, gx = to_host(t.scatter(gm)).astype(np.float64), to_host(t.scatter(gx)).astype(np.float64)
    scale = np.abs(om).mean()
    assert (np.abs(gm - om) <= 1e-5 * np.maximum(np.abs(om), scale)).all()
    assert np.linalg.norm(gx - ox) <= 1e-4 * np.linalg.norm(ox)
    t.close()


def test_tree_deposit_errors():
    dev()
    n = 1000
    x = workloads.clustered(n, 5)
    m = to_dev(workloads.masses(n, 6))
    h = to_dev(np.full(n, 0.01, np.float32))
    grid = ((0, 0, 0), 1.0 / 16, (16, 16, 16))
    # a NaN found by the deferred check of the build
    bad = x.copy()
    bad[123, 2] = np.nan
    t = kdt.build(to_dev(bad), leaf_size=16, check_finite="deferred")
    for call in (lambda: kdt.p2m_tree(t, m, h, *grid),
                 lambda: kdt.p2m_tree_backward(t, m, h, *grid, torch.ones((16,) * 3,
                                                                          device=dev()))):
        with pytest.raises(kdt.KdtError) as e:
            call()
        assert e.value.status == kdt.KDT_EINVAL
    t.close()
    # a point outside the mesh box
    t = kdt.build(to_dev(x), leaf_size=16)
    with pytest.raises(kdt.KdtError) as e:
        kdt.p2m_tree(t, m, h, (0.5, 0, 0), 1.0 / 16, (16, 16, 16))
    assert e.value.status == kdt.KDT_EINVAL
    # an unknown scheme
    g = kdt.make_grid(*grid)
    out = torch.empty((16,) * 3, device=dev())
    with pytest.raises(kdt.KdtError) as e:
        kdt._check(kdt.load().kdt_p2m_tree(t._h, kdt._ptr(m), kdt._ptr(h), kdt.C.byref(g), 4,
                                           kdt._ptr(out), kdt._stream()))
    assert e.value.status == kdt.KDT_EINVAL
    t.close()
    # trees the deposit cannot read: d != 3, float64 coordinates
    t2 = kdt.build(to_dev(np.ascontiguousarray(x[:, :2])), leaf_size=16)
    t64 = kdt.build_f64(torch.from_numpy(x.astype(np.float64)).to(dev()), leaf_size=16)
    for tt in (t2, t64):
        with pytest.raises(kdt.KdtError) as e:
            kdt.p2m_tree(tt, m, h, *grid)
        assert e.value.status == kdt.KDT_EUNSUPPORTED
        tt.close()
