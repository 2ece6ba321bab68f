"""GPU parity at the full workload sizes, in the launch configuration bench.py
times: every row the oracle can follow in seconds (its queries run in
contiguous slices on the host's cores), sampled rows elsewhere, and properties
that hold at any size where it cannot follow."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from paper_2609_18316_amd import kdt, workloads
from tests.gpu_util import dev, say, to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N = 1 << 24
NQ = 1 << 22
T = oracle.host_threads()


@pytest.fixture(scope="module")
def clustered():
    dev()
    say("generating 2^24 clustered points and 2^22 queries")
    x = workloads.clustered(N, seed=2)
    q = workloads.uniform(NQ, 3, seed=102)
    xt, qt = to_dev(x), to_dev(q)
    tree = kdt.build(xt, leaf_size=0, tune_k=32)  # the tuned leaf size, as the bench
    say("oracle tree over 2^24 points")
    ot = oracle.Tree(x, 32)
    return x, q, xt, qt, tree, ot


def test_knn_and_counts_full_size_every_row(clustered):
    """The headline workload: kNN k = 32 and r = 0.01 counts of all 2^22
    queries against the oracle, row by row."""
    x, q, xt, qt, tree, ot = clustered
    say("kNN k=32 of 2^22 queries + r=0.01 counts")
    order = tree.query_order(qt)
    idx, d2 = tree.knn(qt, 32, order=order)
    cnt = tree.range(qt, 0.01)
    idx, d2, cnt = to_host(idx), to_host(d2), to_host(cnt)
    say(f"oracle kNN of all 2^22 queries on {T} threads")
    oi, od = ot.knn(q, 32, threads=T)
    np.testing.assert_array_equal(idx, oi)
    np.testing.assert_array_equal(d2, od)
    say(f"oracle counts of all 2^22 queries on {T} threads")
    np.testing.assert_array_equal(cnt, ot.range(q, 0.01, threads=T))


def test_midpoint_tree_full_size(clustered):
    """The paper's split rule on the GPU at 2^24 clustered points: the whole
    tree equals the oracle's (which builds with that rule), and kNN k = 32 and
    r = 0.01 counts of all 2^22 queries over it equal the oracle's."""
    from tests.test_gpu_midpoint import assert_same_tree
    x, q, xt, qt, tree, ot = clustered
    leaf = kdt.tuning_get(3, N, 32)[0]
    say(f"sliding-midpoint tree over 2^24 points, leaf {leaf} (the bench's)")
    mt = kdt.build(xt, leaf_size=leaf, split_rule=kdt.SPLIT_MIDPOINT)
    omt = ot if leaf == 32 else oracle.Tree(x, leaf)
    say(f"{mt.info.n_nodes} nodes, depth {mt.info.levels}; comparing with the oracle's tree")
    assert mt.info.levels == omt.depth
    assert_same_tree(mt.export(), omt.export())
    del omt
    idx, d2 = mt.knn(qt, 32)
    cnt = mt.range(qt, 0.01)
    idx, d2, cnt = to_host(idx), to_host(d2), to_host(cnt)
    say(f"oracle kNN and counts of all 2^22 queries on {T} threads")
    oi, od = ot.knn(q, 32, threads=T)
    np.testing.assert_array_equal(idx, oi)
    np.testing.assert_array_equal(d2, od)
    np.testing.assert_array_equal(cnt, ot.range(q, 0.01, threads=T))
    mt.close()


def test_ball_lists_full_size(clustered):
    """CSR lists of the r = 0.01 balls of all 2^22 queries on the 2^24-point
    tree (Algorithm 3 with lists): offsets equal the running sum of the
    oracle's counts on every row; on every row the listed indices ascend, are
    distinct and lie in the closed ball (d2 <= r2, float32 in the oracle's
    summation order), which with the counts makes each list the exact ball;
    2^14 sampled rows also equal the oracle's lists."""
    x, q, xt, qt, tree, ot = clustered
    r = 0.01
    say("ball lists r=0.01 of 2^22 queries")
    cnt, off, idx = tree.range(qt, r, lists=True)
    cnt, off, idx = to_host(cnt), to_host(off), to_host(idx)
    say(f"{len(idx)} pairs; oracle counts of all 2^22 queries on {T} threads")
    oc = ot.range(q, r, threads=T)
    np.testing.assert_array_equal(cnt, oc)
    assert off[0] == 0
    np.testing.assert_array_equal(np.diff(off), oc.astype(np.int64))
    assert off[-1] == len(idx)
    r2 = np.float32(r) * np.float32(r)
    row = np.repeat(np.arange(NQ, dtype=np.int64), oc)
    step = 1 << 24
    for s in range(0, len(idx), step):
        i, w = idx[s:s + step], row[s:s + step]
        assert i.min() >= 0 and i.max() < N
        dx = x[i] - q[w]
        d2 = (dx[:, 0] * dx[:, 0] + dx[:, 1] * dx[:, 1]) + dx[:, 2] * dx[:, 2]
        assert (d2 <= r2).all()
        # ascending and distinct within each row
        same_row = w[1:] == w[:-1]
        assert (i[1:][same_row] > i[:-1][same_row]).all()
    sample = workloads.sample_indices(NQ, 1 << 14, seed=61)
    say("oracle lists of 2^14 sampled rows")
    sc, soff, sidx = ot.range(q[sample], r, lists=True)
    for j, row_id in enumerate(sample):
        np.testing.assert_array_equal(idx[off[row_id]:off[row_id + 1]], sidx[soff[j]:soff[j + 1]])


def test_box_counts_full_size_sampled(clustered):
    """2^16 boxes of side 0.002-0.04 on the 2^24-point tree; 48 sampled rows
    checked against the oracle's definition."""
    x, q, xt, qt, tree, ot = clustered
    rng = np.random.Generator(np.random.PCG64(51))
    c = rng.random((1 << 16, 3), dtype=np.float32)
    half = ((0.002 + 0.038 * rng.random((1 << 16, 3))) / 2).astype(np.float32)
    lo, hi = (c - half).astype(np.float32), (c + half).astype(np.float32)
    say("box counts of 2^16 boxes on 2^24 points")
    cnt = to_host(tree.box(to_dev(lo), to_dev(hi)))
    s = workloads.sample_indices(1 << 16, 48, seed=52)
    np.testing.assert_array_equal(cnt[s], oracle.box_brute(x, lo[s], hi[s]))


def test_self_knn_and_smoothing_full_size_sampled(clustered):
    x, q, xt, qt, tree, ot = clustered
    say("self kNN k=32 of 2^24 points, k-th distance")
    h = to_host(tree.knn(None, 32, kth_only=2))
    s = workloads.sample_indices(N, 1 << 20, seed=8)
    say(f"oracle self kNN of 2^20 sampled points on {T} threads")
    oi, od = ot.knn(x[s], 32, threads=T)
    np.testing.assert_array_equal(h[s], np.sqrt(od[:, -1]))
    assert (od[:, 0] == 0).all()


@pytest.mark.parametrize("k", [1000, 10_000])
def test_large_k_full_size_sampled(clustered, k):
    """kNN with k in the ball-and-sort range on the 2^24 clustered points: the
    first 10^5 uniform queries (as timed) and 2000 queries on cluster points,
    whose first candidate balls hold far more than k points and shrink once
    before the sort; full sorted rows compared on 200 sampled queries."""
    x, q, xt, qt, tree, ot = clustered
    on = x[workloads.sample_indices(N, 2000, seed=9)]
    for name, qs in (("uniform", q[:100_000]), ("in clusters", on)):
        say(f"large k={k} of {len(qs)} {name} queries on 2^24 points")
        gi, gd = tree.knn(to_dev(qs), k)
        s = workloads.sample_indices(len(qs), 200, seed=10)
        st = torch.from_numpy(s).to(gi.device)
        hi, hd = to_host(gi[st]), to_host(gd[st])
        del gi, gd
        say(f"oracle tree kNN k={k} of the 200 sampled rows on {T} threads")
        oi, od = ot.knn(qs[s], k, threads=T)
        np.testing.assert_array_equal(hi, oi)
        np.testing.assert_array_equal(hd, od)


def test_fof_full_size_properties_and_sampled_components(clustered):
    x, q, xt, qt, tree, ot = clustered
    l = float(np.float32(0.2 * (1.0 / N) ** (1.0 / 3.0)))
    say(f"FoF of 2^24 points, l={l}")
    lab = to_host(tree.fof(l))
    i = np.arange(N)
    assert (lab <= i).all()
    assert (lab[lab] == lab).all()
    s = workloads.sample_indices(N, 2000, seed=9)
    c, off, lst = ot.range(x[s], l, lists=True)
    owner = np.repeat(np.arange(len(s)), c)
    assert (lab[lst] == lab[s][owner]).all()
    # exact components of small groups, by breadth-first search with oracle ball queries
    checked = 0
    for p in s[:400]:
        seen = {int(p)}
        frontier = [int(p)]
        ok = True
        while frontier and ok:
            cc, oo, ll = ot.range(x[frontier], l, lists=True)
            nxt = set(ll.tolist()) - seen
            seen |= nxt
            frontier = sorted(nxt)
            ok = len(seen) <= 3000
        if ok:
            assert lab[p] == min(seen)
            assert (lab[sorted(seen)] == lab[p]).all()
            checked += 1
    assert checked > 100


def test_deposit_full_size_subvolume_and_adjoint_sample(clustered):
    x, q, xt, qt, tree, ot = clustered
    g = 256
    cell = 1.0 / g
    m = workloads.masses(N, seed=5)
    mt = to_dev(m)
    h = tree.knn(None, 32, kth_only=2)
    say("P2M forward 2^24 particles on 256^3")
    rho = to_host(kdt.p2m(xt, mt, h, (0, 0, 0), cell, (g, g, g), order_ptr=tree.perm_ptr))
    hh = to_host(h)
    # the same deposit in tree order, as the step runs it: smoothing lengths
    # written in tree order, masses gathered, positions from the tree
    say("P2M forward in tree order")
    h_t = tree.knn(None, 32, kth_only=2, tree_rows=True)
    np.testing.assert_array_equal(to_host(tree.scatter(h_t)), hh)
    m_t = tree.gather(mt)
    rho_t = to_host(kdt.p2m_tree(tree, m_t, h_t, (0, 0, 0), cell, (g, g, g)))
    total = float(m.astype(np.float64).sum())
    for r in (rho, rho_t):
        assert abs(float(r.astype(np.float64).sum()) - total) <= 1e-5 * total
    mean = total / rho.size
    for lo_c in ((100, 100, 100), (3, 250, 17), (128, 64, 200)):
        lo = np.array(lo_c) * cell
        hi = (np.array(lo_c) + 16) * cell
        H = np.maximum(hh, np.float32(cell)).astype(np.float64)
        near = np.all((x >= lo - H[:, None] - cell) & (x < hi + H[:, None] + cell), axis=1)
        sel = np.nonzero(near)[0]
        say(f"oracle deposit of {len(sel)} particles around cells {lo_c}")
        o = oracle.p2m(x[sel], m[sel], hh[sel], (0, 0, 0), cell, (g, g, g))
        a, b, c = lo_c
        og = o[a:a + 16, b:b + 16, c:c + 16]
        gt = rho_t[a:a + 16, b:b + 16, c:c + 16].astype(np.float64)
        assert (np.abs(gt - og) <= 1e-5 * np.maximum(np.abs(og), mean)).all()
        gg = rho[a:a + 16, b:b + 16, c:c + 16].astype(np.float64)
        err = np.abs(gg - og)
        assert (err <= 1e-5 * np.maximum(np.abs(og), mean)).all()
        # the measured errors, for the record: against max(|rho64|, mean) and
        # purely relative on cells above 10^-3 of the mean
        big = np.abs(og) > 1e-3 * mean
        say(f"  max error / max(|rho64|, mean) {(err / np.maximum(np.abs(og), mean)).max():.3e}; "
            f"max relative error on {int(big.sum())} cells above 1e-3 mean "
            f"{(err[big] / np.abs(og[big])).max() if big.any() else 0.0:.3e}")
    say("P2M adjoint 2^24 particles")
    gen = torch.Generator(device=xt.device).manual_seed(11)
    up = torch.randn((g, g, g), device=xt.device, generator=gen)
    gm, gx = kdt.p2m_backward(xt, mt, h, (0, 0, 0), cell, (g, g, g), up, order_ptr=tree.perm_ptr)
    s = workloads.sample_indices(N, 2048, seed=12)
    om, ox = oracle.p2m_backward(x[s], m[s], hh[s], (0, 0, 0), cell, (g, g, g), to_host(up))
    gm_s, gx_s = to_host(gm)[s].astype(np.float64), to_host(gx)[s].astype(np.float64)
    assert (np.abs(gm_s - om) <= 1e-5 * np.maximum(np.abs(om), np.abs(om).mean())).all()
    assert np.linalg.norm(gx_s - ox) <= 1e-4 * np.linalg.norm(ox)
    say("P2M adjoint in tree order")
    gm_t, gx_t = kdt.p2m_tree_backward(tree, m_t, h_t, (0, 0, 0), cell, (g, g, g), up)
    gm_s = to_host(tree.scatter(gm_t))[s].astype(np.float64)
    gx_s = to_host(tree.scatter(gx_t))[s].astype(np.float64)
    assert (np.abs(gm_s - om) <= 1e-5 * np.maximum(np.abs(om), np.abs(om).mean())).all()
    assert np.linalg.norm(gx_s - ox) <= 1e-4 * np.linalg.norm(ox)


def test_periodic_deposit_full_size_corner_and_faces(clustered):
    """The 256^3 deposit on the periodic mesh: sub-volumes at a corner and on
    faces, where supports wrap, against the oracle over the particles within
    reach the shorter way round; total mass exact; the adjoint on a sample."""
    x, q, xt, qt, tree, ot = clustered
    g = 256
    cell = 1.0 / g
    m = workloads.masses(N, seed=5)
    mt = to_dev(m)
    h = tree.knn(None, 32, kth_only=2)
    say("periodic P2M forward 2^24 particles on 256^3")
    rho = to_host(kdt.p2m(xt, mt, h, (0, 0, 0), cell, (g, g, g), order_ptr=tree.perm_ptr,
                          periodic=True))
    hh = to_host(h)
    total = float(m.astype(np.float64).sum())
    assert abs(float(rho.astype(np.float64).sum()) - total) <= 1e-5 * total
    mean = total / rho.size
    H = np.maximum(hh, np.float32(cell)).astype(np.float64)
    for lo_c in ((0, 0, 0), (248, 120, 0), (250, 250, 250), (7, 255, 100)):
        lo = np.array(lo_c) * cell
        hi = (np.array(lo_c) + 16) * cell
        gap = np.zeros_like(x, dtype=np.float64)
        for a in range(3):  # distance to the slab [lo, hi), the shorter way round
            d = np.maximum(np.maximum(lo[a] - x[:, a], x[:, a] - hi[a]), 0.0)
            d = np.minimum(d, np.maximum(np.maximum(lo[a] - (x[:, a] - 1.0), (x[:, a] - 1.0) - hi[a]), 0.0))
            d = np.minimum(d, np.maximum(np.maximum(lo[a] - (x[:, a] + 1.0), (x[:, a] + 1.0) - hi[a]), 0.0))
            gap[:, a] = d
        sel = np.nonzero(np.all(gap < H[:, None] + cell, axis=1))[0]
        say(f"oracle periodic deposit of {len(sel)} particles around cells {lo_c}")
        o = oracle.p2m(x[sel], m[sel], hh[sel], (0, 0, 0), cell, (g, g, g), periodic=True)
        cx = [np.arange(c, c + 16) % g for c in lo_c]
        og = o[np.ix_(*cx)]
        gg = rho[np.ix_(*cx)].astype(np.float64)
        assert (np.abs(gg - og) <= 1e-5 * np.maximum(np.abs(og), mean)).all()
    say("periodic P2M adjoint 2^24 particles")
    gen = torch.Generator(device=xt.device).manual_seed(13)
    up = torch.randn((g, g, g), device=xt.device, generator=gen)
    gm, gx = kdt.p2m_backward(xt, mt, h, (0, 0, 0), cell, (g, g, g), up, order_ptr=tree.perm_ptr,
                              periodic=True)
    s = workloads.sample_indices(N, 2048, seed=14)
    om, ox = oracle.p2m_backward(x[s], m[s], hh[s], (0, 0, 0), cell, (g, g, g), to_host(up),
                                 periodic=True)
    gm_s, gx_s = to_host(gm)[s].astype(np.float64), to_host(gx)[s].astype(np.float64)
    assert (np.abs(gm_s - om) <= 1e-5 * np.maximum(np.abs(om), np.abs(om).mean())).all()
    assert np.linalg.norm(gx_s - ox) <= 1e-4 * np.linalg.norm(ox)


@pytest.mark.parametrize("scheme", ("cic", "tsc"))
def test_cloud_deposit_full_size(clustered, scheme):
    """The fixed-cloud comparison of Table 3 at the full size: 2^24 particles
    on 256^3, periodic and open, total mass and sub-volumes against the
    oracle over the particles within reach."""
    x, q, xt, qt, tree, ot = clustered
    g = 256
    cell = 1.0 / g
    m = workloads.masses(N, seed=5)
    total = float(m.astype(np.float64).sum())
    mean = total / g ** 3
    for periodic in (False, True):
        say(f"{scheme} deposit of 2^24 particles on 256^3, periodic={periodic}")
        rho = to_host(kdt.p2m_cloud(xt, to_dev(m), (0, 0, 0), cell, (g, g, g), scheme,
                                    order_ptr=tree.perm_ptr, periodic=periodic))
        assert abs(float(rho.astype(np.float64).sum()) - total) <= 1e-5 * total
        # sub-volumes at a corner and across the z faces (periodic) or inside
        for lo_c in ((0, 0, 0), (100, 37, 250) if periodic else (100, 37, 240)):
            reach = 2 * cell
            cx = [np.arange(c, c + 16) % g for c in lo_c]
            lo = np.array(lo_c) * cell
            hi = (np.array(lo_c) + 16) * cell
            near = np.ones(N, bool)
            for a in range(3):
                d = np.maximum(np.maximum(lo[a] - x[:, a], x[:, a] - hi[a]), 0.0)
                if periodic:
                    d = np.minimum(d, np.maximum(lo[a] - (x[:, a] - 1.0), 0.0))
                    d = np.minimum(d, np.maximum((x[:, a] + 1.0) - hi[a], 0.0))
                near &= d < reach
            sel = np.nonzero(near)[0]
            o = oracle.p2m_cloud(x[sel], m[sel], (0, 0, 0), cell, (g, g, g), scheme,
                                 periodic=periodic)
            og, gg = o[np.ix_(*cx)], rho[np.ix_(*cx)].astype(np.float64)
            ratio = np.abs(gg - og) / (1e-5 * np.maximum(np.abs(og), mean))
            worst = np.unravel_index(np.argmax(ratio), ratio.shape)
            assert (ratio <= 1).all(), (periodic, lo_c, float(ratio.max()), worst,
                                        float(gg[worst]), float(og[worst]), len(sel))


@pytest.mark.parametrize("d", (2, 4, 8, 16))
@pytest.mark.parametrize("dist", ("uniform", "normal"))
def test_dimension_sweep_full_size_sampled(d, dist):
    """The bench's configuration: leaf size and traversal from the autotuner's
    table, every point as a query."""
    from paper_2609_18316_amd import autotune
    dev()
    n = 1 << 22
    x = workloads.uniform(n, d, 300 + d) if dist == "uniform" else workloads.normal(n, d, 400 + d)
    c = autotune.lookup(n, d, 16, f"self-{dist}")
    trav = 2 if c.queries_per_wave == 64 else 1
    say(f"dimension sweep d={d} {dist}: leaf {c.leaf_size}, traversal {trav}, kNN k=16")
    xt = to_dev(x)
    t = kdt.build(xt, leaf_size=c.leaf_size)
    idx, d2 = t.knn(None, 16, traversal=trav)
    idx, d2 = to_host(idx), to_host(d2)
    s = workloads.sample_indices(n, 1024 if d >= 8 else 1 << 14, seed=13 + d)
    say(f"oracle kNN of {len(s)} sampled points on {T} threads")
    oi, od = oracle.Tree(x, 32).knn(x[s], 16, threads=T)
    np.testing.assert_array_equal(idx[s], oi)
    np.testing.assert_array_equal(d2[s], od)


def test_batched_full_size():
    dev()
    sizes = workloads.batch_sizes(256, 3.0, 6.0, seed=4)
    say(f"batch of 256 clustered sets, {int(sizes.sum())} points")
    x, off = workloads.batched_clustered(sizes, seed_base=40000)
    lens = np.array([np.float32(0.2 * (1.0 / s) ** (1.0 / 3.0)) for s in sizes], np.float32)
    plan = kdt.BatchPlan(off, 3, 8)
    xt, lt = to_dev(x), to_dev(lens)
    a = [to_host(v) for v in plan.launch(xt, lt, use_graph=1)]
    b = [to_host(v) for v in plan.launch(xt, lt, use_graph=0)]
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    idx, d2, lab = a
    plan.close()

    def one(s):
        xs = x[off[s]:off[s + 1]]
        t = oracle.Tree(xs, 32)
        oi, od = t.knn(xs, 8)
        return s, oi, od, t.fof(float(lens[s]))

    say(f"oracle kNN and FoF of all 256 sets on {T} threads")
    done = 0
    with ThreadPoolExecutor(T) as ex:  # largest sets first
        for f in [ex.submit(one, int(s)) for s in np.argsort(-sizes, kind="stable")]:
            s, oi, od, ol = f.result()
            np.testing.assert_array_equal(idx[off[s]:off[s + 1]], oi)
            np.testing.assert_array_equal(d2[off[s]:off[s + 1]], od)
            np.testing.assert_array_equal(lab[off[s]:off[s + 1]], ol)
            done += 1
    assert done == 256
