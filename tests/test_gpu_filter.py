"""The matrix-core filter of the wave kNN (d = 8, 16) must never drop a
point that belongs in the answer: it marks candidates with matrix-core dot
products of split bf16 operands and a rounding margin, and the exact float32
distances decide.
These cases put the decision within a few ulps or make the norm expansion
cancel badly; results must stay bit-identical to the oracle."""
import numpy as np
import pytest

import oracle
from paper_2609_18316_amd import kdt
from tests.gpu_util import dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _shells(d, n_centres, per_shell, seed):
    """Points on thin shells around random centres (radius 0.3, relative
    spread 1e-6): many distances tie within a few ulps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.random((n_centres, d))
    pts = []
    for c in centres:
        v = rng.standard_normal((per_shell, d))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        r = 0.3 * (1.0 + 1e-6 * rng.standard_normal((per_shell, 1)))
        pts.append(c + r * v)
    return np.concatenate(pts).astype(np.float32), centres.astype(np.float32)


@pytest.mark.parametrize("d", (8, 16))
@pytest.mark.parametrize("k", (1, 16, 64))
def test_filter_keeps_near_ties(d, k):
    dev()
    x, centres = _shells(d, 40, 150, seed=31 + d)
    rng = np.random.Generator(np.random.PCG64(32 + d))
    q = (centres + 1e-7 * rng.standard_normal(centres.shape)).astype(np.float32)
    say(f"shell near-ties d={d} k={k}")
    oi, od = oracle.knn_brute(x, q, k)
    for leaf in (16, 64):
        t = kdt.build(to_dev(x), leaf_size=leaf)
        gi, gd = t.knn(to_dev(q), k, traversal=2)
        np.testing.assert_array_equal(to_host(gi), oi)
        np.testing.assert_array_equal(to_host(gd), od)
        t.close()


@pytest.mark.parametrize("d", (8, 16))
@pytest.mark.parametrize("offset", (1e3, -3e4))
def test_filter_far_from_the_origin(d, offset):
    """|q|^2 and |p|^2 dwarf the distances: the expansion cancels and the
    filter keeps almost everything, which must still give exact results."""
    dev()
    rng = np.random.Generator(np.random.PCG64(33 + d))
    x = (rng.random((6000, d)) + offset).astype(np.float32)
    q = (rng.random((500, d)) + offset).astype(np.float32)
    say(f"far from the origin d={d} offset={offset:g}")
    oi, od = oracle.knn_brute(x, q, 16)
    t = kdt.build(to_dev(x), leaf_size=64)
    gi, gd = t.knn(to_dev(q), 16, traversal=2)
    np.testing.assert_array_equal(to_host(gi), oi)
    np.testing.assert_array_equal(to_host(gd), od)
    gi, gd = t.knn(None, 16, traversal=2)
    oi, od = oracle.knn_brute(x, x, 16)
    np.testing.assert_array_equal(to_host(gi), oi)
    np.testing.assert_array_equal(to_host(gd), od)


def _large(kind, n, d, scale, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "cloud":    # far from the origin, 1 % spread: finite distances
        return (scale * (1 + 0.01 * rng.random((n, d)))).astype(np.float32)
    if kind == "spread":   # around the origin at `scale`: many distances overflow to inf
        return (scale * rng.standard_normal((n, d))).astype(np.float32)
    # mixed magnitudes 1 .. 1e19 in one set
    return (rng.standard_normal((n, d)) * 10.0 ** rng.integers(0, 20, (n, 1))).astype(np.float32)


@pytest.mark.parametrize("d", (8, 16))
@pytest.mark.parametrize("kind,scale", [(k, s) for k in ("cloud", "spread") for s in (1e18, 4e18, 1e19)]
                         + [("mixed", 1e19)])
def test_filter_large_coordinates(d, scale, kind):
    """Coordinates where |q|^2 + |p|^2 overflows float32: the filter works
    around the wave's first query and marks every pair whose norms are too
    large to trust, so results stay exact."""
    dev()
    x = _large(kind, 3000, d, scale, seed=int(71 + d + np.log10(scale)))
    q = _large(kind, 400, d, scale, seed=int(91 + d + np.log10(scale)))
    for k in (1, 16, 64):
        oi, od = oracle.knn_brute(x, q, k)
        for leaf in (16, 64):
            t = kdt.build(to_dev(x), leaf_size=leaf)
            for sort in (1, 0):
                say(f"large coordinates d={d} scale={scale:g} kind={kind} k={k} leaf={leaf} sort={sort}")
                gi, gd = t.knn(to_dev(q), k, traversal=2, sort_queries=sort)
                np.testing.assert_array_equal(to_host(gi), oi)
                np.testing.assert_array_equal(to_host(gd), od)
            t.close()
    oi, od = oracle.knn_brute(x, x, 16)
    t = kdt.build(to_dev(x), leaf_size=64)
    gi, gd = t.knn(None, 16, traversal=2)
    np.testing.assert_array_equal(to_host(gi), oi)
    np.testing.assert_array_equal(to_host(gd), od)
    t.close()


@pytest.mark.parametrize("d", (8, 16))
def test_filter_norms_overflow_dot_product_does_not(d):
    """Two points whose squared norms sum above FLT_MAX while their dot
    product stays finite, and whose distance is finite: only the guard on the
    norm sum keeps the pair.  Queries in input order put a query at the
    origin first in the wave, so the centre does not help."""
    dev()
    a = np.sqrt(1.75e38)
    cos = 3.3e38 / (2 * 1.75e38)
    rng = np.random.Generator(np.random.PCG64(5 + d))
    x = np.zeros((200, d))
    x[:100] = rng.random((100, d))
    x[100:, 0] = a * cos * (1 + 1e-3 * rng.random(100))
    x[100:, 1] = a * np.sqrt(1 - cos * cos) * (1 + 1e-3 * rng.random(100))
    x = x.astype(np.float32)
    q = np.zeros((64, d))
    q[1:, 0] = a * (1 + 1e-3 * rng.random(63))
    q = q.astype(np.float32)
    t = kdt.build(to_dev(x), leaf_size=64)
    for k in (1, 8, 64):
        say(f"norm-overflow guard d={d} k={k}")
        oi, od = oracle.knn_brute(x, q, k)
        assert np.isfinite(od[1:, 0]).all()
        gi, gd = t.knn(to_dev(q), k, traversal=2, sort_queries=0)
        np.testing.assert_array_equal(to_host(gi), oi)
        np.testing.assert_array_equal(to_host(gd), od)
    t.close()


def test_batched_forest_large_coordinates():
    """The batched forest's wave kNN uses the same filter at d = 8."""
    dev()
    sizes = [1, 40, 700, 3001, 64, 1500]
    sets = [_large(kind, n, 8, sc, seed=300 + i) for i, (n, kind, sc) in enumerate(
        zip(sizes, ("cloud", "cloud", "spread", "cloud", "mixed", "spread"),
            (1e18, 4e18, 1e19, 1e19, 1.0, 4e18)))]
    x = np.concatenate(sets)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    lens = np.zeros(len(sizes), np.float32)
    plan = kdt.BatchPlan(off, 8, 8, traversal=0)
    say("batched forest, large coordinates, d=8")
    idx, d2, lab = (to_host(a) for a in plan.launch(to_dev(x), to_dev(lens), use_graph=2))
    for s in range(len(sizes)):
        xs = sets[s]
        oi, od = oracle.knn_brute(xs, xs, 8)
        np.testing.assert_array_equal(idx[off[s]:off[s + 1]], oi)
        np.testing.assert_array_equal(d2[off[s]:off[s + 1]], od)
    plan.close()
