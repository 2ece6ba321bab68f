"""Pins of the box-query oracle (rectangular ranges, Sec. 2.3) against facts
that do not come from it: a pure-Python loop over tiny inputs, boxes whose
answer is known in closed form, additivity of counts when a box is cut between
lattice planes, and nesting against the ball oracle."""
import numpy as np

import oracle
from tests import cases


def _loops(pts, lo, hi):
    out = []
    for i in range(len(lo)):
        row = []
        for j, x in enumerate(pts):
            if all(lo[i][a] <= x[a] <= hi[i][a] for a in range(len(x))):
                row.append(j)
        out.append(row)
    return out


def test_matches_a_plain_loop_on_tiny_inputs():
    rng = np.random.Generator(np.random.PCG64(90))
    for d in (2, 3, 8):
        pts = rng.random((60, d), dtype=np.float32)
        a = rng.random((40, d), dtype=np.float32)
        b = rng.random((40, d), dtype=np.float32)
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        rows = _loops(pts, lo, hi)
        c, off, idx = oracle.box_brute(pts, lo, hi, lists=True)
        assert c.tolist() == [len(r) for r in rows]
        assert idx.tolist() == [j for r in rows for j in r]
        assert off[-1] == len(idx)


def test_known_boxes():
    pts = cases.points("duplicates", 500, 3, seed=91)
    n = len(pts)
    whole = (np.full((1, 3), -1.0, np.float32), np.full((1, 3), 2.0, np.float32))
    assert oracle.box_brute(pts, *whole).tolist() == [n]
    inf = (np.full((1, 3), -np.inf, np.float32), np.full((1, 3), np.inf, np.float32))
    assert oracle.box_brute(pts, *inf).tolist() == [n]
    empty = (np.full((1, 3), 0.6, np.float32), np.full((1, 3), 0.4, np.float32))
    assert oracle.box_brute(pts, *empty).tolist() == [0]
    nan_lo = np.full((1, 3), -1.0, np.float32)
    nan_lo[0, 1] = np.nan
    assert oracle.box_brute(pts, nan_lo, whole[1]).tolist() == [0]
    # a degenerate box on a point holds exactly that point's copies
    uniq, mult = np.unique(pts, axis=0, return_counts=True)
    got = oracle.box_brute(pts, uniq[:50], uniq[:50])
    assert got.tolist() == mult[:50].tolist()


def test_additive_when_cut_between_lattice_planes():
    pts = cases.points("lattice", 2000, 3, seed=92)
    # lattice coordinates are multiples of a step; cut half-way between two planes
    step = np.min(np.diff(np.unique(pts[:, 0])))
    rng = np.random.Generator(np.random.PCG64(93))
    for _ in range(20):
        a, b = rng.random(3, dtype=np.float32), rng.random(3, dtype=np.float32)
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        axis = int(rng.integers(3))
        k = np.floor(0.5 * (lo[axis] + hi[axis]) / step)
        cut = np.float32((k + 0.5) * step)
        left_hi, right_lo = hi.copy(), lo.copy()
        left_hi[axis] = min(cut, hi[axis])
        right_lo[axis] = max(cut, lo[axis])
        whole = oracle.box_brute(pts, lo[None], hi[None])[0]
        parts = (oracle.box_brute(pts, lo[None], left_hi[None])[0] +
                 oracle.box_brute(pts, right_lo[None], hi[None])[0])
        assert whole == parts


def test_nested_between_inscribed_and_circumscribed_boxes_of_a_ball():
    rng = np.random.Generator(np.random.PCG64(94))
    pts = rng.random((3000, 3), dtype=np.float32)
    q = rng.random((100, 3), dtype=np.float32)
    r = 0.1
    ball = oracle.range_brute(pts, q, r)
    inner = r / np.sqrt(3.0) * 0.999  # strictly inside the ball
    small = oracle.box_brute(pts, (q - inner).astype(np.float32), (q + inner).astype(np.float32))
    big = oracle.box_brute(pts, (q - r * 1.001).astype(np.float32), (q + r * 1.001).astype(np.float32))
    assert (small <= ball).all() and (ball <= big).all()
    assert (small < big).any()
