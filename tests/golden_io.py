"""Readers for the hand-derived fixtures under ``tests/golden/``."""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for raw in f:
            s = raw.strip()
            if s and not s.startswith("#"):
                yield s


def knn_line():
    """Returns (points[n][2] float32, list of (query, k, idx, d2))."""
    pts, cases = [], []
    for s in _lines("knn_line.txt"):
        if "|" in s:
            q, idx, d2 = (p.split() for p in s.split("|"))
            qv = np.array([float(q[0]) / 16, float(q[1]) / 16], np.float32)
            k = int(q[2])
            iv = np.array([int(v) for v in idx], np.int32)
            dv = np.array([np.inf if v == "inf" else float(v) / 256 for v in d2], np.float32)
            cases.append((qv, k, iv, dv))
        else:
            x, y = s.split()
            pts.append((float(x) / 16, float(y) / 16))
    return np.array(pts, np.float32), cases


def range_lattice():
    """Returns list of (R2, N) pairs."""
    return [tuple(int(v) for v in s.split()) for s in _lines("range_lattice.txt")]


def fof_groups():
    """Returns (points[n][2] float32, l, expected labels int32)."""
    rows = [s.split() for s in _lines("fof_groups.txt")]
    pts = np.array([[float(r[0]), float(r[1])] for r in rows], np.float32)
    lab = np.array([int(r[2]) for r in rows], np.int32)
    return pts, 0.25, lab
