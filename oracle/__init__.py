"""CPU oracle for the k-d tree hot path -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never calls it and shares no code with it.

The arithmetic lives in ``kdt_oracle.c`` (plain single-threaded C, float32
distances with no fused multiply-add, float64 particle-to-mesh).  This module
marshals numpy arrays through ctypes; the box query, which has no arithmetic
(coordinate comparisons only), is written out here with numpy.
"""
from __future__ import annotations

import ctypes as C
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import build as _build

_lib = None

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")


class _Grid(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("cell", C.c_double), ("n", C.c_int32 * 3),
                ("periodic", C.c_int32)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build()
    lib = C.CDLL(path)
    i64, i32, f32, vp = C.c_int64, C.c_int, C.c_float, C.c_void_p
    lib.orc_sq_dist.argtypes = [_f32p, _f32p, i32]
    lib.orc_sq_dist.restype = f32
    lib.orc_knn_brute.argtypes = [_f32p, i64, i32, _f32p, i64, i32, _i32p, _f32p]
    lib.orc_range_brute.argtypes = [_f32p, i64, i32, _f32p, i64, f32, _i64p, vp, vp]
    lib.orc_knn_brute_torus.argtypes = [_f32p, i64, i32, _f32p, i64, i32, _f32p, _i32p, _f32p]
    lib.orc_range_brute_torus.argtypes = [_f32p, i64, i32, _f32p, i64, f32, _f32p, _i64p, vp, vp]
    lib.orc_knn_brute_f64.argtypes = [_f64p, i64, i32, _f64p, i64, i32, _i32p, _f64p]
    lib.orc_range_brute_f64.argtypes = [_f64p, i64, i32, _f64p, i64, C.c_double, _i64p, vp, vp]
    lib.orc_fof_brute.argtypes = [_f32p, i64, i32, f32, _i32p]
    lib.orc_fof_brute_torus.argtypes = [_f32p, i64, i32, f32, _f32p, _i32p]
    lib.orc_tree_build.argtypes = [_f32p, i64, i32, i32, C.POINTER(vp)]
    lib.orc_tree_free.argtypes = [vp]
    lib.orc_tree_free.restype = None
    lib.orc_tree_n_nodes.argtypes = [vp]
    lib.orc_tree_n_nodes.restype = i64
    lib.orc_tree_depth.argtypes = [vp]
    lib.orc_tree_depth.restype = C.c_int32
    lib.orc_tree_export.argtypes = [vp] * 11
    lib.orc_knn_tree.argtypes = [vp, _f32p, i64, i32, _i32p, _f32p]
    lib.orc_range_tree.argtypes = [vp, _f32p, i64, f32, _i64p, vp, vp, i64]
    lib.orc_fof_tree.argtypes = [vp, _f32p, f32, _i32p]
    lib.orc_m4_w.argtypes = [C.c_double]
    lib.orc_m4_w.restype = C.c_double
    lib.orc_m4_dw.argtypes = [C.c_double]
    lib.orc_m4_dw.restype = C.c_double
    for name in ("orc_p2m", "orc_p2m_brute"):
        getattr(lib, name).argtypes = [_f64p, _f64p, _f64p, i64, C.POINTER(_Grid), _f64p]
    lib.orc_p2m_backward.argtypes = [_f64p, _f64p, _f64p, i64, C.POINTER(_Grid), _f64p, vp, vp]
    lib.orc_p2m_cloud.argtypes = [_f64p, _f64p, i64, C.POINTER(_Grid), i32, _f64p, i32]
    lib.orc_cloud_shape.argtypes = [i32, C.c_double]
    lib.orc_cloud_shape.restype = C.c_double
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def host_threads() -> int:
    """Threads for slicing oracle queries: the host's cores, at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                      else (os.cpu_count() or 1)))


def _sliced(nq: int, threads: int, call):
    """Runs call(lo, hi) over contiguous query slices on `threads` host
    threads.  The C routines take their own buffers and only read the tree,
    and ctypes releases the interpreter lock while they run, so the slices
    run in parallel; each slice is the single-threaded oracle as written."""
    threads = max(1, min(int(threads), nq))
    if threads == 1:
        call(0, nq)
        return
    bounds = np.linspace(0, nq, threads + 1).astype(np.int64)
    with ThreadPoolExecutor(threads) as ex:
        for f in [ex.submit(call, int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:])]:
            f.result()


def _pts(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    if x.ndim == 1:
        x = x[:, None]
    return x


def sq_dist(p, q) -> np.float32:
    p, q = np.ascontiguousarray(p, np.float32), np.ascontiguousarray(q, np.float32)
    return np.float32(_load().orc_sq_dist(p, q, p.shape[0]))


# --------------------------------------------------------------------------
# brute force (the plain definitions)
# --------------------------------------------------------------------------

def _period(period, d: int):
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(period, np.float32), (d,)))
    return L


def knn_brute(pts, queries, k: int, period=None, threads: int = 1):
    """k smallest (d2, index) keys of every query, ascending: (idx, d2).

    ``period`` (a length or one per axis): distances on the D-torus of those
    periods (Sec. 2.1, Sec. 2.4), every coordinate in [0, period).
    ``threads``: contiguous query slices on that many host threads.
    """
    pts, queries = _pts(pts), _pts(queries)
    nq = queries.shape[0]
    idx = np.empty((nq, k), np.int32)
    d2 = np.empty((nq, k), np.float32)
    lib = _load()

    def call(a, b):
        if period is None:
            rc = lib.orc_knn_brute(pts, pts.shape[0], pts.shape[1], queries[a:b], b - a, k,
                                   idx[a:b], d2[a:b])
        else:
            rc = lib.orc_knn_brute_torus(pts, pts.shape[0], pts.shape[1], queries[a:b], b - a, k,
                                         _period(period, pts.shape[1]), idx[a:b], d2[a:b])
        _check(rc, "knn_brute")

    _sliced(nq, threads, call)
    return idx, d2


def range_brute(pts, queries, r: float, lists: bool = False, period=None):
    """Counts of points with d2 <= fl(r*r); with ``lists`` also CSR (offsets, idx).

    ``period``: distances on the D-torus, as in ``knn_brute``.
    """
    pts, queries = _pts(pts), _pts(queries)
    n, d = pts.shape
    nq = queries.shape[0]
    lib = _load()

    def call(count, offsets, idx):
        if period is None:
            return lib.orc_range_brute(pts, n, d, queries, nq, np.float32(r), count, offsets, idx)
        return lib.orc_range_brute_torus(pts, n, d, queries, nq, np.float32(r),
                                         _period(period, d), count, offsets, idx)

    count = np.empty(nq, np.int64)
    _check(call(count, None, None), "range_brute")
    if not lists:
        return count
    offsets = np.empty(nq + 1, np.int64)
    idx = np.empty(max(int(count.sum()), 1), np.int32)
    _check(call(count, offsets.ctypes.data, idx.ctypes.data), "range_brute")
    return count, offsets, idx[:int(count.sum())]


def _pts64(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    return x


def knn_brute_f64(pts, queries, k: int, threads: int = 1):
    """kNN on float64 coordinates (the double-precision real kind of
    Sec. 2.4): the k smallest (d2, index) keys with d2 in float64, ascending,
    padded with (-1, +inf): (idx int32, d2 float64)."""
    pts, queries = _pts64(pts), _pts64(queries)
    nq = queries.shape[0]
    idx = np.empty((nq, k), np.int32)
    d2 = np.empty((nq, k), np.float64)
    lib = _load()

    def call(a, b):
        _check(lib.orc_knn_brute_f64(pts, pts.shape[0], pts.shape[1], queries[a:b], b - a, k,
                                     idx[a:b], d2[a:b]), "knn_brute_f64")

    _sliced(nq, threads, call)
    return idx, d2


def range_brute_f64(pts, queries, r: float, lists: bool = False):
    """Ball counts (d2 <= fl64(r*r)) on float64 coordinates; with ``lists``
    also CSR (offsets int64, ascending indices int32)."""
    pts, queries = _pts64(pts), _pts64(queries)
    n, d = pts.shape
    nq = queries.shape[0]
    lib = _load()
    count = np.empty(nq, np.int64)
    _check(lib.orc_range_brute_f64(pts, n, d, queries, nq, float(r), count, None, None),
           "range_brute_f64")
    if not lists:
        return count
    offsets = np.empty(nq + 1, np.int64)
    idx = np.empty(max(int(count.sum()), 1), np.int32)
    _check(lib.orc_range_brute_f64(pts, n, d, queries, nq, float(r), count,
                                   offsets.ctypes.data, idx.ctypes.data), "range_brute_f64")
    return count, offsets, idx[:int(count.sum())]


def box_brute(pts, lo, hi, lists: bool = False):
    """Points inside closed axis-aligned boxes (the rectangular ranges of
    Sec. 2.3): point x is in box i when lo[i][a] <= x[a] <= hi[i][a] on every
    axis a.  A box with lo > hi on some axis, or with a NaN bound, holds no
    point.  With ``lists`` also CSR (offsets int64, ascending input indices).
    The definition written out, one box at a time; comparisons only."""
    pts, lo, hi = _pts(pts), _pts(lo), _pts(hi)
    nq = lo.shape[0]
    counts = np.empty(nq, np.int64)
    rows = []
    for i in range(nq):
        inside = np.all((pts >= lo[i]) & (pts <= hi[i]), axis=1)
        idx = np.nonzero(inside)[0].astype(np.int32)
        counts[i] = idx.size
        if lists:
            rows.append(idx)
    if not lists:
        return counts
    offsets = np.zeros(nq + 1, np.int64)
    offsets[1:] = np.cumsum(counts)
    return counts, offsets, (np.concatenate(rows) if rows else np.empty(0, np.int32))


def fof_brute(pts, l: float, period=None) -> np.ndarray:
    """Group label (smallest input index of the group) of every point;
    ``period``: friends on the D-torus, as in ``knn_brute``."""
    pts = _pts(pts)
    labels = np.empty(pts.shape[0], np.int32)
    lib = _load()
    if period is None:
        rc = lib.orc_fof_brute(pts, pts.shape[0], pts.shape[1], np.float32(l), labels)
    else:
        rc = lib.orc_fof_brute_torus(pts, pts.shape[0], pts.shape[1], np.float32(l),
                                     _period(period, pts.shape[1]), labels)
    _check(rc, "fof_brute")
    return labels


# --------------------------------------------------------------------------
# sliding-midpoint tree and the queries of Algorithms 2 and 3
# --------------------------------------------------------------------------

class Tree:
    """Sliding-midpoint k-d tree over a float32 ``[n][d]`` array."""

    def __init__(self, pts, leaf_size: int = 16):
        self.pts = _pts(pts)
        self.n, self.d = self.pts.shape
        self.leaf_size = leaf_size
        self._h = C.c_void_p()
        _check(_load().orc_tree_build(self.pts, self.n, self.d, leaf_size, C.byref(self._h)),
               "tree_build")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.orc_tree_free(h)
            self._h = None

    @property
    def n_nodes(self) -> int:
        return int(_load().orc_tree_n_nodes(self._h))

    @property
    def depth(self) -> int:
        return int(_load().orc_tree_depth(self._h))

    def export(self) -> dict:
        m, n, d = self.n_nodes, self.n, self.d
        out = dict(pts=np.empty((n, d), np.float32), idx=np.empty(n, np.int32),
                   begin=np.empty(m, np.int64), end=np.empty(m, np.int64),
                   left=np.empty(m, np.int64), right=np.empty(m, np.int64),
                   axis=np.empty(m, np.int32), split=np.empty(m, np.float32),
                   lo=np.empty((m, d), np.float32), hi=np.empty((m, d), np.float32))
        keys = ["pts", "idx", "begin", "end", "left", "right", "axis", "split", "lo", "hi"]
        _check(_load().orc_tree_export(self._h, *[out[k].ctypes.data for k in keys]), "export")
        return out

    def knn(self, queries, k: int, threads: int = 1):
        """Algorithm 2 for every query: (idx, d2) ascending by (d2, index).
        ``threads``: contiguous query slices on that many host threads."""
        q = _pts(queries)
        nq = q.shape[0]
        idx = np.empty((nq, k), np.int32)
        d2 = np.empty((nq, k), np.float32)

        def call(a, b):
            _check(_load().orc_knn_tree(self._h, q[a:b], b - a, k, idx[a:b], d2[a:b]), "knn_tree")

        _sliced(nq, threads, call)
        return idx, d2

    def range(self, queries, r: float, lists: bool = False, threads: int = 1):
        """Algorithm 3 for every query: counts, and with ``lists`` the CSR lists
        too (``threads`` applies to counts only)."""
        q = _pts(queries)
        nq = q.shape[0]
        lib = _load()
        count = np.empty(nq, np.int64)

        def call(a, b):
            _check(lib.orc_range_tree(self._h, q[a:b], b - a, np.float32(r), count[a:b], None,
                                      None, 0), "range_tree")

        _sliced(nq, threads, call)
        if not lists:
            return count
        total = int(count.sum())
        offsets = np.empty(nq + 1, np.int64)
        idx = np.empty(max(total, 1), np.int32)
        _check(lib.orc_range_tree(self._h, q, nq, np.float32(r), count, offsets.ctypes.data,
                                  idx.ctypes.data, total), "range_tree")
        return count, offsets, idx[:total]

    def fof(self, l: float) -> np.ndarray:
        labels = np.empty(self.n, np.int32)
        _check(_load().orc_fof_tree(self._h, self.pts, np.float32(l), labels), "fof_tree")
        return labels


# --------------------------------------------------------------------------
# particle-to-mesh deposit (float64)
# --------------------------------------------------------------------------

def m4_w(q: float) -> float:
    return float(_load().orc_m4_w(float(q)))


def m4_dw(q: float) -> float:
    return float(_load().orc_m4_dw(float(q)))


def _grid(lo, cell, shape, periodic=False) -> _Grid:
    g = _Grid()
    for a in range(3):
        g.lo[a] = float(lo[a])
        g.n[a] = int(shape[a])
    g.cell = float(cell)
    g.periodic = 1 if periodic else 0
    return g


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def p2m(x, m, h, lo, cell, shape, brute: bool = False, periodic: bool = False) -> np.ndarray:
    """Mass per cell, float64 ``shape`` (x slowest, z fastest).

    ``periodic``: the mesh box is a 3-torus (every H below half a period).
    ``brute``: every cell of the mesh, distances the shorter way round on a
    periodic mesh, instead of the particle's support box."""
    x, m, h = _f64(x, (-1, 3)), _f64(m), _f64(h)
    rho = np.empty(int(np.prod(shape)), np.float64)
    fn = _load().orc_p2m_brute if brute else _load().orc_p2m
    _check(fn(x, m, h, x.shape[0], C.byref(_grid(lo, cell, shape, periodic)), rho), "p2m")
    return rho.reshape(shape)


CLOUD_SCHEMES = {"ngp": 1, "cic": 2, "tsc": 3}


def p2m_cloud(x, m, lo, cell, shape, scheme: str, periodic: bool = False,
              brute: bool = False) -> np.ndarray:
    """Fixed-cloud deposit (NGP, CIC or TSC): mass per cell, float64 ``shape``.
    ``brute``: every cell of the mesh through the scheme's shape function."""
    x, m = _f64(x, (-1, 3)), _f64(m)
    rho = np.empty(int(np.prod(shape)), np.float64)
    _check(_load().orc_p2m_cloud(x, m, x.shape[0], C.byref(_grid(lo, cell, shape, periodic)),
                                 CLOUD_SCHEMES[scheme], rho, 1 if brute else 0), "p2m_cloud")
    return rho.reshape(shape)


def cloud_shape(scheme: str, v: float) -> float:
    return float(_load().orc_cloud_shape(CLOUD_SCHEMES[scheme], float(v)))


def p2m_backward(x, m, h, lo, cell, shape, g, periodic: bool = False):
    """(dL/dm, dL/dx) for L = sum(g * rho), h held fixed, float64."""
    x, m, h = _f64(x, (-1, 3)), _f64(m), _f64(h)
    g = _f64(g).reshape(-1)
    n = x.shape[0]
    dm = np.empty(n, np.float64)
    dx = np.empty((n, 3), np.float64)
    _check(_load().orc_p2m_backward(x, m, h, n, C.byref(_grid(lo, cell, shape, periodic)), g,
                                    dm.ctypes.data, dx.ctypes.data), "p2m_backward")
    return dm, dx
