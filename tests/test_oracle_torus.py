"""Pins for the oracle's distances on the D-torus (periodic boundary
conditions, Sec. 2.1 and Sec. 2.4) against what the mathematics fixes:
explicit enumeration of the periodic images in integer arithmetic on a
lattice, the open metric where no way round is shorter, translation
invariance, and float64 images for general coordinates."""
import itertools

import numpy as np
import pytest

import oracle
from tests import cases

DIMS = (2, 3, 4, 8, 16)


def _image_d2(xi, qi, P):
    """Squared torus distances by enumerating the images x + m P (m in
    {-1, 0, 1} per axis, enough for coordinates in [0, P)) instead of any
    closed formula: all 3^d image vectors up to d = 4; above, per axis, since
    a sum of squares over independent per-axis images is smallest axis by axis."""
    d = xi.shape[1]
    if d <= 4:
        best = None
        for m in itertools.product((-1, 0, 1), repeat=d):
            v = ((xi + np.asarray(m) * P - qi) ** 2).sum(axis=1)
            best = v if best is None else np.minimum(best, v)
        return best
    per_axis = np.stack([(xi + m * P - qi) ** 2 for m in (-1, 0, 1)]).min(axis=0)
    return per_axis.sum(axis=1)


@pytest.mark.parametrize("d", DIMS)
def test_torus_lattice_knn_and_range_match_integer_images(d):
    """On a 1/16 lattice every float32 operation is exact, so torus kNN and
    ball counts equal the integer image enumeration, ties by index."""
    rng = np.random.Generator(np.random.PCG64(40 + d))
    per = np.array([16, 32, 8, 16] * 4)[:d]  # periods 1, 2, 0.5, 1, ... in lattice units
    xi = rng.integers(0, per, (400, d))
    qi = rng.integers(0, per, (25, d))
    x = (xi / 16.0).astype(np.float32)
    q = (qi / 16.0).astype(np.float32)
    L = (per / 16.0).astype(np.float32)
    for k in (1, 9, 70, 400, 403):
        idx, d2 = oracle.knn_brute(x, q, k, period=L)
        for s in range(q.shape[0]):
            di = _image_d2(xi, qi[s], per)
            order = np.lexsort((np.arange(len(di)), di))[:k]
            m = len(order)
            np.testing.assert_array_equal(idx[s, :m], order)
            np.testing.assert_array_equal(d2[s, :m].astype(np.float64) * 256.0, di[order])
            assert np.all(idx[s, m:] == -1)
    for r16 in (0, 3, 5.5, 12):
        cnt, off, lst = oracle.range_brute(x, q, r16 / 16.0, lists=True, period=L)
        for s in range(q.shape[0]):
            di = _image_d2(xi, qi[s], per)
            want = np.nonzero(di <= r16 * r16)[0]
            assert cnt[s] == len(want)
            np.testing.assert_array_equal(lst[off[s]:off[s + 1]], want)


@pytest.mark.parametrize("kind", cases.KINDS)
@pytest.mark.parametrize("d", DIMS)
def test_torus_equals_open_metric_inside_half_period(kind, d):
    """With every coordinate in [0, L/2) no way round is shorter, so the torus
    results equal the open-boundary ones exactly."""
    x = cases.points(kind, 500, d, seed=d)
    q = cases.points(kind, 40, d, seed=100 + d)
    lo = min(x.min(), q.min())
    span = max(x.max(), q.max()) - lo
    scale = np.float32(0.49) / np.float32(span if span > 0 else 1.0)
    xs = ((x - lo) * scale).astype(np.float32)
    qs = ((q - lo) * scale).astype(np.float32)
    for k in (1, 16, 100):
        np.testing.assert_array_equal(oracle.knn_brute(xs, qs, k, period=1.0)[0],
                                      oracle.knn_brute(xs, qs, k)[0])
        np.testing.assert_array_equal(oracle.knn_brute(xs, qs, k, period=1.0)[1],
                                      oracle.knn_brute(xs, qs, k)[1])
    for r in (0.0, 0.05, 0.2):
        np.testing.assert_array_equal(oracle.range_brute(xs, qs, r, period=1.0),
                                      oracle.range_brute(xs, qs, r))


def test_torus_translation_invariance():
    """Shifting every point and query by the same lattice vector, modulo the
    period, leaves every torus distance and so every result unchanged."""
    rng = np.random.Generator(np.random.PCG64(77))
    xi = rng.integers(0, 16, (600, 3))
    qi = rng.integers(0, 16, (30, 3))
    x, q = (xi / 16.0).astype(np.float32), (qi / 16.0).astype(np.float32)
    i0, d0 = oracle.knn_brute(x, q, 40, period=1.0)
    c0 = oracle.range_brute(x, q, 0.3, period=1.0)
    for shift in ((5, 0, 11), (15, 15, 15), (8, 8, 8)):
        xs = (((xi + shift) % 16) / 16.0).astype(np.float32)
        qs = (((qi + shift) % 16) / 16.0).astype(np.float32)
        i1, d1 = oracle.knn_brute(xs, qs, 40, period=1.0)
        np.testing.assert_array_equal(i1, i0)
        np.testing.assert_array_equal(d1, d0)
        np.testing.assert_array_equal(oracle.range_brute(xs, qs, 0.3, period=1.0), c0)


def test_torus_distances_match_float64_images():
    """General coordinates: the float32 torus d2 of each neighbour is within
    a few float32 roundings of the float64 minimum over the images."""
    rng = np.random.Generator(np.random.PCG64(5))
    x = rng.random((2000, 3), dtype=np.float32)
    q = rng.random((50, 3), dtype=np.float32)
    idx, d2 = oracle.knn_brute(x, q, 20, period=1.0)
    for s in range(q.shape[0]):
        exact = _image_d2(x[idx[s]].astype(np.float64), q[s].astype(np.float64), 1.0)
        np.testing.assert_allclose(d2[s], exact, rtol=4e-7 * 8, atol=1e-12)
        # and nothing outside the list is nearer than its last entry (beyond rounding)
        all_d = _image_d2(x.astype(np.float64), q[s].astype(np.float64), 1.0)
        assert np.sort(all_d)[19] >= exact.max() * (1 - 1e-5)


def test_torus_rejects_coordinates_outside_the_period():
    x = np.array([[0.1, 0.2], [1.0, 0.5]], np.float32)
    with pytest.raises(ValueError):
        oracle.knn_brute(x, x[:1], 1, period=1.0)
    with pytest.raises(ValueError):
        oracle.range_brute(x[:1], np.array([[-0.1, 0.2]], np.float32), 0.1, period=1.0)


def _groups_by_union(edges_ok, n):
    """Smallest-index labels of the components of a boolean adjacency matrix."""
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    ii, jj = np.nonzero(edges_ok)
    for a, b in zip(ii.tolist(), jj.tolist()):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    return np.array([find(i) for i in range(n)], np.int32)


@pytest.mark.parametrize("d", (2, 3, 8))
def test_torus_fof_lattice_matches_integer_images(d):
    """Groups on a 1/16 lattice with per-axis periods equal the components of
    the integer image-distance graph (union-find over all pairs)."""
    rng = np.random.Generator(np.random.PCG64(60 + d))
    per = np.array([16, 32, 8, 16] * 4)[:d]
    xi = rng.integers(0, per, (300, d))
    x = (xi / 16.0).astype(np.float32)
    L = (per / 16.0).astype(np.float32)
    for l16 in (0, 1, 2.5, 4):
        got = oracle.fof_brute(x, l16 / 16.0, period=L)
        d2 = np.stack([_image_d2(xi, xi[s], per) for s in range(len(xi))])
        want = _groups_by_union(d2 <= l16 * l16, len(xi))
        np.testing.assert_array_equal(got, want)


def test_torus_fof_reduces_and_translates():
    """Inside half a period FoF on the torus equals the open one; a lattice
    shift modulo the period leaves the groups unchanged."""
    x = cases.points("normal", 800, 3, seed=3)
    xs = ((x - x.min()) * (np.float32(0.49) / (x.max() - x.min()))).astype(np.float32)
    for l in (0.005, 0.02):
        np.testing.assert_array_equal(oracle.fof_brute(xs, l, period=1.0), oracle.fof_brute(xs, l))
    rng = np.random.Generator(np.random.PCG64(2))
    xi = rng.integers(0, 16, (500, 3))
    base = oracle.fof_brute((xi / 16.0).astype(np.float32), 1.5 / 16, period=1.0)
    moved = oracle.fof_brute((((xi + (7, 15, 3)) % 16) / 16.0).astype(np.float32), 1.5 / 16,
                             period=1.0)
    np.testing.assert_array_equal(moved, base)
