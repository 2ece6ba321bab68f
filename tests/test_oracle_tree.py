"""Structural invariants of the oracle's sliding-midpoint tree (Sec. 2.1,
Algorithm 1, Eq. 2)."""
import numpy as np
import pytest

import oracle
from tests import cases


def check_tree(x, leaf):
    t = oracle.Tree(x, leaf)
    e = t.export()
    n = x.shape[0]
    # the tree holds a copy of every point exactly once
    assert sorted(e["idx"].tolist()) == list(range(n))
    np.testing.assert_array_equal(e["pts"], x[e["idx"]])
    assert e["begin"][0] == 0 and e["end"][0] == n
    for v in range(t.n_nodes):
        b, en = e["begin"][v], e["end"][v]
        p = e["pts"][b:en]
        if en > b:  # tight bounding box
            np.testing.assert_array_equal(e["lo"][v], p.min(axis=0))
            np.testing.assert_array_equal(e["hi"][v], p.max(axis=0))
        l, r = e["left"][v], e["right"][v]
        if l < 0:
            coincide = en - b > 0 and (p == p[0]).all()
            assert en - b <= leaf or coincide
            continue
        # completeness (Eq. 2): the children split the parent's range
        assert e["begin"][l] == b and e["end"][l] == e["begin"][r] and e["end"][r] == en
        assert e["end"][l] > b and en > e["begin"][r]
        ax, s = e["axis"][v], e["split"][v]
        ext = e["hi"][v] - e["lo"][v]
        assert ax == int(np.argmax(ext))  # longest side, lowest axis on ties
        lv = e["pts"][b:e["end"][l], ax]
        rv = e["pts"][e["begin"][r]:en, ax]
        assert lv.max() <= rv.min()
        assert lv.max() <= s <= rv.min()
        for c in (l, r):
            assert (e["lo"][c] >= e["lo"][v]).all() and (e["hi"][c] <= e["hi"][v]).all()
    return t


@pytest.mark.parametrize("kind", cases.KINDS)
@pytest.mark.parametrize("d", (2, 3, 16))
def test_tree_invariants(kind, d):
    for n in (1, 2, 33, 500):
        for leaf in (1, 4, 16):
            check_tree(cases.points(kind, n, d, seed=n + d), leaf)


def test_midpoint_on_uniform_cube_halves_the_box():
    """The first plane of a box-filling set sits at the middle of its longest side."""
    g = np.arange(16, dtype=np.float32) / np.float32(15.0)
    x = np.stack(np.meshgrid(g, g * 0.5, indexing="ij"), -1).reshape(-1, 2).astype(np.float32)
    e = oracle.Tree(x, 4).export()
    assert e["axis"][0] == 0 and e["split"][0] == np.float32(0.5)
    assert e["end"][e["left"][0]] == 128


def test_slide_when_midpoint_rounds_onto_the_lower_face():
    """Box [1, 1 + ulp]: the midpoint rounds to 1, the lower side would be
    empty, and the plane slides so that one extreme point moves across."""
    one = np.float32(1.0)
    up = np.nextafter(one, np.float32(2))
    x = np.array([[one, 0], [up, 0], [one, 0], [up, 0], [one, 0]], np.float32)
    t = check_tree(x, 1)
    e = t.export()
    l = e["left"][0]
    assert e["end"][l] - e["begin"][l] == 1
    assert e["idx"][e["begin"][l]] == 0  # lowest index among the extreme points


def test_depth_grows_like_log_n_on_uniform():
    x = cases.points("uniform", 4096, 3, seed=1)
    t = oracle.Tree(x, 16)
    assert 8 <= t.depth <= 14
