"""Pins for the oracle's float64-coordinate kNN and ball queries (the
double-precision real kind of Sec. 2.4).

The pins do not retype the oracle's formula: they use inputs whose float64
squared distances are exact (coordinates on a 2^-12 or 2^-40 lattice with
small integer offsets), so the right answer follows from integer arithmetic
alone -- the order of the integer squared distances with ties by index, and
the counts of integer distances within an integer radius.  A dropped axis, a
float32 intermediate, a wrong tie rule, an open instead of closed ball or a
lost padding rule each fails one of them."""
import numpy as np
import pytest

import oracle

SCALE = 2.0 ** -12


def _lattice(n, d, seed, span=40):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(-span, span + 1, size=(n, d)).astype(np.int64)


def _int_knn(pi, qi, k):
    out_i = np.full((len(qi), k), -1, np.int64)
    out_d = np.full((len(qi), k), -1, np.int64)
    for t, q in enumerate(qi):
        d2 = ((pi - q) ** 2).sum(axis=1)
        order = np.lexsort((np.arange(len(pi)), d2))[:k]
        out_i[t, :len(order)] = order
        out_d[t, :len(order)] = d2[order]
    return out_i, out_d


@pytest.mark.parametrize("d", (2, 3, 4, 8, 16))
def test_knn_on_a_lattice_equals_integer_order(d):
    pi, qi = _lattice(300, d, 10 + d), _lattice(40, d, 20 + d)
    qi[:5] = pi[:5]  # queries on data points find themselves first
    for k in (1, 7, 64, 300, 303):
        idx, d2 = oracle.knn_brute_f64(pi * SCALE, qi * SCALE, k)
        ei, ed = _int_knn(pi, qi, k)
        np.testing.assert_array_equal(idx, ei)
        pad = ei < 0
        assert np.isinf(d2[pad]).all() and (d2[pad] > 0).all()
        np.testing.assert_array_equal(d2[~pad], ed[~pad] * SCALE * SCALE)
    idx, d2 = oracle.knn_brute_f64(pi * SCALE, qi[:5] * SCALE, 1)
    assert (d2[:, 0] == 0).all()


@pytest.mark.parametrize("d", (2, 3, 8))
def test_ball_counts_and_lists_on_a_lattice(d):
    pi, qi = _lattice(400, d, 30 + d, span=12), _lattice(50, d, 40 + d, span=12)
    for R in (0, 1, 5, 13, 60):  # 5 and 13: integer radii met exactly by lattice offsets
        count, off, lst = oracle.range_brute_f64(pi * SCALE, qi * SCALE, R * SCALE, lists=True)
        for t, q in enumerate(qi):
            inside = np.nonzero(((pi - q) ** 2).sum(axis=1) <= R * R)[0]
            assert count[t] == len(inside)
            np.testing.assert_array_equal(lst[off[t]:off[t + 1]], inside)
        # the closed ball holds points exactly on the sphere
        if R == 5 and d == 3:
            on = sum(int((((pi - q) ** 2).sum(axis=1) == 25).sum()) for q in qi)
            assert on > 0


def test_separations_below_float32_resolution():
    """Points 2^-40 apart near 1: float32 would make them one point; float64
    keeps the exact order, ties by index."""
    i = np.arange(100)
    x = (1.0 + i * 2.0 ** -40)[:, None]
    q = np.array([[1.0 + 37.5 * 2.0 ** -40]])
    idx, d2 = oracle.knn_brute_f64(x, q, 10)
    key = np.abs(2 * i - 75)
    want = np.lexsort((i, key))[:10]
    np.testing.assert_array_equal(idx[0], want)
    np.testing.assert_array_equal(d2[0], (key[want] ** 2).astype(np.float64) * 2.0 ** -82)
    assert list(idx[0][:4]) == [37, 38, 36, 39]
    # ball of radius 3.5 lattice steps: |2i - 75| <= 7 -> i in 34..41
    c, off, lst = oracle.range_brute_f64(x, q, 3.5 * 2.0 ** -40, lists=True)
    np.testing.assert_array_equal(lst, np.arange(34, 42))


def test_far_coordinates_beyond_float32_range():
    """Coordinates near 1e300 with offsets that float32 cannot even hold."""
    base = 1e300
    pi = _lattice(60, 3, 7, span=20)
    x = base + pi * 2.0 ** 960  # exact: 2^960 is far above base's ulp (2^944)
    q = base + pi[:6] * 2.0 ** 960
    # squared offsets overflow float64 (2^1920): every distance is +inf except
    # the point itself; the order is then the index order among the infs
    idx, d2 = oracle.knn_brute_f64(x, q, 3)
    for t in range(6):
        same = np.nonzero((pi == pi[t]).all(axis=1))[0]
        assert idx[t, 0] == same[0] and d2[t, 0] == 0.0
    # offsets of 2^-1010 square to below the smallest subnormal: every
    # distance is 0 and the order is the index order
    small = 1e-300 + pi * 2.0 ** -1010
    idx, d2 = oracle.knn_brute_f64(small, small[:6], 4)
    assert (idx == np.arange(4)).all() and (d2 == 0).all()


def test_errors():
    with pytest.raises(ValueError):
        oracle.range_brute_f64(np.zeros((3, 2)), np.zeros((1, 2)), -1.0)
    with pytest.raises(ValueError):
        oracle.knn_brute_f64(np.zeros((3, 2)), np.zeros((1, 2)), 0)
