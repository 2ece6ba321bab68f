"""Float64 coordinates on the GPU (the double-precision real kind of Sec. 2.4):
kNN and ball counts and lists bit-exact against the float64 oracle, over both
split rules, every dimension, several point kinds (including separations
float32 cannot hold and coordinates beyond the float32 range), self and
external queries, sorted and unsorted."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_18316_amd import kdt, workloads
from tests.gpu_util import dev, say, to_host

pytestmark = pytest.mark.gpu


def to_dev64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev())


def _points(kind, n, d, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "uniform":
        return rng.random((n, d))
    if kind == "normal":
        return rng.standard_normal((n, d))
    if kind == "clustered":
        x = workloads.clustered(n, seed).astype(np.float64)
        x = x if d == 3 else np.tile(x, (1, 6))[:, :d]
        return x + rng.random((n, d)) * 1e-9  # below float32 resolution
    if kind == "fine":  # a 2^-40 lattice near 1: float32 sees one point
        return 1.0 + rng.integers(0, 64, size=(n, d)) * 2.0 ** -40
    if kind == "far":  # beyond the float32 range
        return 1e300 * (1.0 + rng.random((n, d)))
    if kind == "lattice":  # exact distances, many ties
        return rng.integers(-8, 9, size=(n, d)) * 2.0 ** -4
    raise ValueError(kind)


def _queries(kind, nq, d, seed):
    if kind in ("far",):
        return _points(kind, nq, d, seed)
    if kind == "fine":
        return _points("fine", nq, d, seed)
    if kind == "lattice":
        return _points("lattice", nq, d, seed)
    return _points("uniform" if kind != "normal" else "normal", nq, d, seed)


KINDS = ("uniform", "normal", "clustered", "fine", "far", "lattice")
RULES = (kdt.SPLIT_MEDIAN, kdt.SPLIT_MIDPOINT)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("d", (2, 3, 4, 8, 16))
def test_knn_f64_equals_the_oracle(kind, d):
    dev()
    for n in (1, 33, 5000):
        x = _points(kind, n, d, 100 * n + d)
        q = _queries(kind, 300, d, 7 * n + d)
        for rule in RULES:
            for leaf in (4, 32):
                say(f"f64 kNN {kind} d={d} n={n} rule={rule} leaf={leaf}")
                t = kdt.build_f64(to_dev64(x), leaf_size=leaf, split_rule=rule)
                for k in sorted({1, 8, 33, 64, min(n + 3, 64)}):
                    oi, od = oracle.knn_brute_f64(x, q, k)
                    gi, gd = t.knn(to_dev64(q), k)
                    np.testing.assert_array_equal(to_host(gi), oi)
                    np.testing.assert_array_equal(to_host(gd), od)
                    gi, gd = t.knn(to_dev64(q), k, sort_queries=False)
                    np.testing.assert_array_equal(to_host(gi), oi)
                    np.testing.assert_array_equal(to_host(gd), od)
                k = min(16, n)
                oi, od = oracle.knn_brute_f64(x, x, k)
                gi, gd = t.knn(None, k)
                np.testing.assert_array_equal(to_host(gi), oi)
                np.testing.assert_array_equal(to_host(gd), od)
                t.close()


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("d", (2, 3, 8, 16))
def test_range_f64_equals_the_oracle(kind, d):
    dev()
    n = 5000
    x = _points(kind, n, d, 300 + d)
    q = _queries(kind, 400, d, 400 + d)
    span = np.ptp(x) if np.isfinite(np.ptp(x)) else 1.0
    for rule in RULES:
        t = kdt.build_f64(to_dev64(x), leaf_size=16, split_rule=rule)
        for frac in (0.0, 0.02, 0.1, 0.5):
            r = float(frac * span * (1.0 if d <= 4 else 2.0))
            if kind == "lattice":
                r = float(np.ceil(frac * 16) * 2.0 ** -4)  # met exactly by lattice offsets
            say(f"f64 balls {kind} d={d} rule={rule} r={r:.3g}")
            oc, ooff, oidx = oracle.range_brute_f64(x, q, r, lists=True)
            np.testing.assert_array_equal(to_host(t.range(to_dev64(q), r)), oc)
            gc, goff, gidx = t.range(to_dev64(q), r, lists=True)
            np.testing.assert_array_equal(to_host(goff), ooff)
            np.testing.assert_array_equal(to_host(gidx), oidx)
            np.testing.assert_array_equal(to_host(t.range(None, r)),
                                          oracle.range_brute_f64(x, x, r))
        t.close()


def test_f64_edge_cases():
    dev()
    x = _points("uniform", 500, 3, 1)
    t = kdt.build_f64(to_dev64(x), leaf_size=8)
    # k above the limit, periods, float32 calls on a float64 tree
    with pytest.raises(kdt.KdtError) as e:
        t.knn(to_dev64(x[:5]), 65)
    assert e.value.status == kdt.KDT_EUNSUPPORTED
    for call in (lambda: kdt.Tree.knn(t, torch.zeros((3, 3), device=dev()), 4),
                 lambda: kdt.Tree.range(t, torch.zeros((3, 3), device=dev()), 0.1),
                 lambda: kdt.Tree.fof(t, 0.01)):
        with pytest.raises(kdt.KdtError) as e:
            call()
        assert e.value.status == kdt.KDT_EUNSUPPORTED
    # empty query sets, a given order
    gi, gd = t.knn(to_dev64(np.zeros((0, 3))), 4)
    assert gi.shape == (0, 4)
    q = _points("uniform", 200, 3, 2)
    order = t.query_order(torch.from_numpy(q.astype(np.float32)).to(dev()))
    gi, gd = t.knn(to_dev64(q), 8, order=order)
    oi, od = oracle.knn_brute_f64(x, q, 8)
    np.testing.assert_array_equal(to_host(gi), oi)
    np.testing.assert_array_equal(to_host(gd), od)
    t.close()
    # NaN / Inf rejected; one point; identical points
    bad = x.copy()
    bad[17, 1] = np.nan
    with pytest.raises(kdt.KdtError) as e:
        kdt.build_f64(to_dev64(bad))
    assert e.value.status == kdt.KDT_EINVAL
    bad[17, 1] = np.inf
    with pytest.raises(kdt.KdtError):
        kdt.build_f64(to_dev64(bad))
    same = np.full((300, 2), 0.25)
    t = kdt.build_f64(to_dev64(same), leaf_size=4)
    gi, gd = t.knn(to_dev64(same[:3]), 10)
    np.testing.assert_array_equal(to_host(gi), np.tile(np.arange(10), (3, 1)))
    assert (to_host(gd) == 0).all()
    np.testing.assert_array_equal(to_host(t.range(to_dev64(same[:3]), 0.0)), [300] * 3)
    t.close()


def test_f64_full_size_sampled():
    """2^22 clustered points in float64 (the clustered mock plus offsets below
    float32 resolution), kNN k = 32 of 2^20 uniform queries: 4096 sampled rows
    against the oracle; ball counts r = 0.01 the same way."""
    dev()
    n, nq = 1 << 22, 1 << 20
    rng = np.random.Generator(np.random.PCG64(9))
    x = workloads.clustered(n, 12).astype(np.float64) + rng.random((n, 3)) * 1e-9
    q = rng.random((nq, 3))
    t = kdt.build_f64(to_dev64(x), leaf_size=0, tune_k=32)
    say(f"f64 tree over 2^22 points, leaf {t.info.leaf_size}")
    gi, gd = t.knn(to_dev64(q), 32)
    gc = t.range(to_dev64(q), 0.01)
    gi, gd, gc = to_host(gi), to_host(gd), to_host(gc)
    s = workloads.sample_indices(nq, 4096, seed=13)
    oi, od = oracle.knn_brute_f64(x, q[s], 32, threads=oracle.host_threads())
    np.testing.assert_array_equal(gi[s], oi)
    np.testing.assert_array_equal(gd[s], od)
    np.testing.assert_array_equal(gc[s[:512]], oracle.range_brute_f64(x, q[s[:512]], 0.01))
    t.close()
