"""Thin ctypes binding of ``libkdt.so`` (the C ABI declared in include/kdt.h).

Argument marshalling only: tensors must already live on the GPU, every step
runs in the library's HIP kernels on torch's current stream, and a missing or
unloadable library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkdt.so")

KDT_OK, KDT_EINVAL, KDT_EUNSUPPORTED, KDT_ENOMEM, KDT_ECAPACITY, KDT_EDEVICE = range(6)
STATUS_NAMES = {0: "KDT_OK", 1: "KDT_EINVAL", 2: "KDT_EUNSUPPORTED", 3: "KDT_ENOMEM",
                4: "KDT_ECAPACITY", 5: "KDT_EDEVICE"}
MAX_K = 64          # register lists (and the batched forest)
MAX_K_SORTED = 1 << 20  # kdt_knn above MAX_K: ball and sort
DIMS = (2, 3, 4, 8, 16)

# Every exported entry point of include/kdt.h.
EXPORTS = ("kdt_build", "kdt_free", "kdt_tree_get_info", "kdt_tree_export", "kdt_tree_nodes",
           "kdt_knn",
           "kdt_range", "kdt_box", "kdt_fof", "kdt_fof_torus", "kdt_p2m", "kdt_p2m_cloud", "kdt_p2m_backward",
           "kdt_tree_perm", "kdt_query_order",
           "kdt_batch_plan_create", "kdt_batch_launch", "kdt_batch_plan_free", "kdt_knn_noalloc",
           "kdt_stream_release", "kdt_tuning_set", "kdt_tuning_get",
           "kdt_build_f64", "kdt_knn_f64", "kdt_range_f64", "kdt_tree_check",
           "kdt_tree_gather", "kdt_tree_scatter", "kdt_p2m_tree", "kdt_p2m_tree_backward",
           "kdt_last_error")
# The test and measurement hooks of include/kdt_debug.h.
DEBUG_EXPORTS = ("kdt_debug_fail_alloc", "kdt_debug_visits", "kdt_debug_valu_probe",
                 "kdt_debug_radix_sort", "kdt_debug_exclusive_scan", "kdt_debug_sort_rows")
LIB_COUNTS_PATH = os.path.join(HERE, "libkdt_counts.so")
NOALLOC_MAX_SORTED = 1 << 22   # queries kdt_knn_noalloc can order in its static scratch


class KdtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class BuildOpts(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("check_finite", C.c_int32), ("split_rule", C.c_int32),
                ("tune_k", C.c_int32)]

SPLIT_MEDIAN, SPLIT_MIDPOINT = 0, 1


def _periods(period, d: int):
    """ctypes float[d] of the torus periods (one value or one per axis), or None."""
    if period is None:
        return None
    vals = [float(v) for v in period] if hasattr(period, "__len__") else [float(period)] * d
    if len(vals) != d:
        raise ValueError(f"period needs 1 or {d} values, got {len(vals)}")
    return (C.c_float * d)(*vals)


class QueryOpts(C.Structure):
    _fields_ = [("sort_queries", C.c_int32), ("traversal", C.c_int32), ("order", C.c_void_p),
                ("split_budget", C.c_int32), ("period", C.POINTER(C.c_float)),
                ("tree_rows", C.c_int32), ("counts_given", C.c_int32)]


class Grid(C.Structure):
    _fields_ = [("lo", C.c_float * 3), ("cell", C.c_float), ("n", C.c_int32 * 3),
                ("periodic", C.c_int32)]


class TreeInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("leaf_size", C.c_int32),
                ("levels", C.c_int32), ("stride", C.c_int32), ("n_nodes", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Loads the HIP library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2609_18316_amd.build_lib")
    lib = C.CDLL(path)
    vp, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    lib.kdt_build.argtypes = [vp, i64, i32, C.POINTER(BuildOpts), vp, C.POINTER(vp)]
    lib.kdt_free.argtypes = [vp]
    lib.kdt_tree_get_info.argtypes = [vp, C.POINTER(TreeInfo)]
    lib.kdt_tree_export.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.kdt_tree_nodes.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.kdt_knn.argtypes = [vp, vp, i64, i32, vp, vp, i32, C.POINTER(QueryOpts), vp]
    lib.kdt_knn_noalloc.argtypes = [vp, vp, i64, i32, vp, vp, i32, C.POINTER(QueryOpts), vp]
    lib.kdt_range.argtypes = [vp, vp, i64, f32, vp, vp, vp, i64, C.POINTER(C.c_int64),
                              C.POINTER(QueryOpts), vp]
    lib.kdt_box.argtypes = [vp, vp, vp, i64, vp, vp, vp, i64, C.POINTER(C.c_int64),
                            C.POINTER(QueryOpts), vp]
    lib.kdt_fof.argtypes = [vp, f32, vp, C.POINTER(C.c_int64), vp]
    lib.kdt_fof_torus.argtypes = [vp, f32, C.POINTER(C.c_float), vp, C.POINTER(C.c_int64), vp]
    lib.kdt_p2m.argtypes = [vp, vp, vp, i64, C.POINTER(Grid), vp, vp, vp]
    lib.kdt_p2m_cloud.argtypes = [vp, vp, i64, C.POINTER(Grid), i32, vp, vp, vp]
    lib.kdt_p2m_backward.argtypes = [vp, vp, vp, i64, C.POINTER(Grid), vp, vp, vp, vp, vp]
    lib.kdt_query_order.argtypes = [vp, vp, i64, C.c_int32, vp, vp]
    lib.kdt_tree_perm.argtypes = [vp]
    lib.kdt_tree_perm.restype = vp
    lib.kdt_stream_release.argtypes = [vp]
    lib.kdt_tuning_set.argtypes = [i32, i64, i32, i32, i32]
    lib.kdt_tree_check.argtypes = [vp, vp]
    lib.kdt_tree_gather.argtypes = [vp, vp, i32, vp, vp]
    lib.kdt_tree_scatter.argtypes = [vp, vp, i32, vp, vp]
    lib.kdt_p2m_tree.argtypes = [vp, vp, vp, C.POINTER(Grid), i32, vp, vp]
    lib.kdt_p2m_tree_backward.argtypes = [vp, vp, vp, C.POINTER(Grid), vp, vp, vp, vp]
    lib.kdt_build_f64.argtypes = [vp, i64, i32, C.POINTER(BuildOpts), vp, C.POINTER(vp)]
    lib.kdt_knn_f64.argtypes = [vp, vp, i64, i32, vp, vp, C.POINTER(QueryOpts), vp]
    lib.kdt_range_f64.argtypes = [vp, vp, i64, C.c_double, vp, vp, vp, i64, C.POINTER(C.c_int64),
                                  C.POINTER(QueryOpts), vp]
    lib.kdt_tuning_get.argtypes = [i32, i64, i32, vp, vp, vp]
    if hasattr(lib, "kdt_batch_plan_create"):
        lib.kdt_batch_plan_create.argtypes = [vp, i32, i32, i32, C.POINTER(BuildOpts),
                                              C.POINTER(QueryOpts), C.POINTER(vp)]
        lib.kdt_batch_launch.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp]
        lib.kdt_batch_plan_free.argtypes = [vp]
    lib.kdt_debug_fail_alloc.argtypes = [i64]
    lib.kdt_debug_visits.argtypes = [vp, i32]
    lib.kdt_debug_valu_probe.argtypes = [vp, i32, i32, vp]
    lib.kdt_debug_radix_sort.argtypes = [vp, vp, i64, i32, i32, vp]
    lib.kdt_debug_exclusive_scan.argtypes = [vp, vp, i64, i32, vp]
    lib.kdt_debug_sort_rows.argtypes = [vp, vp, vp, i64, i64, vp]
    lib.kdt_last_error.restype = C.c_char_p
    for name in EXPORTS + DEBUG_EXPORTS:
        if name not in ("kdt_last_error", "kdt_tree_perm") and hasattr(lib, name):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def tuning_set(d: int, n: int, k: int, leaf_size: int, queries_per_wave: int) -> None:
    """Installs a tuning entry (leaf size, 1 or 64 queries per traversal) for
    the shape (d, n, k) for the rest of the process (0, 0 removes it)."""
    _check(load().kdt_tuning_set(int(d), int(n), int(k), int(leaf_size), int(queries_per_wave)))


def tuning_get(d: int, n: int, k: int) -> tuple[int, int, int]:
    """(leaf size, queries per traversal, stack depth) the library uses for
    leaf_size = 0 and traversal = 0 at the shape (d, n, k)."""
    leaf, qpw, depth = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    _check(load().kdt_tuning_get(int(d), int(n), int(k), C.byref(leaf), C.byref(qpw),
                                 C.byref(depth)))
    return leaf.value, qpw.value, depth.value


def stream_release(stream=None) -> None:
    """Frees the deposit scratch the library keeps for ``stream`` (stream-ordered)."""
    _check(load().kdt_stream_release(_stream(stream)))


def radix_sort(keys: torch.Tensor, vals: torch.Tensor, begin_bit: int = 0, end_bit: int = 32,
               stream=None) -> None:
    """Test hook: the library's stable radix sort of (uint32 key as int32
    bits, int32 value) pairs in place, on key bits [begin_bit, end_bit)."""
    n = keys.numel()
    keys = _dev(keys, torch.int32, "keys", (n,))
    vals = _dev(vals, torch.int32, "vals", (n,))
    _check(load().kdt_debug_radix_sort(_ptr(keys), _ptr(vals), n, int(begin_bit), int(end_bit),
                                       _stream(stream)))


def exclusive_scan(values: torch.Tensor, out_bits: int = 64, stream=None) -> torch.Tensor:
    """Test hook: the library's exclusive running sum of int32 values;
    out_bits 64 gives n + 1 int64 sums (the last the total), 32 gives n
    int32 sums."""
    n = values.numel()
    values = _dev(values, torch.int32, "values", (n,))
    if out_bits == 64:
        out = torch.empty(n + 1, dtype=torch.int64, device=values.device)
    else:
        out = torch.empty(n, dtype=torch.int32, device=values.device)
    _check(load().kdt_debug_exclusive_scan(_ptr(values), out.data_ptr(), n, int(out_bits),
                                           _stream(stream)))
    return out


def sort_rows(values: torch.Tensor, offsets: torch.Tensor, stream=None) -> torch.Tensor:
    """Test hook: the library's per-row sort of a CSR list (int32 values,
    int64 offsets of nq + 1 entries), every row ascending."""
    total = values.numel()
    values = _dev(values, torch.int32, "values", (total,))
    offsets = _dev(offsets, torch.int64, "offsets")
    out = torch.empty(total, dtype=torch.int32, device=values.device)
    _check(load().kdt_debug_sort_rows(_ptr(values), _ptr(out), _ptr(offsets),
                                      offsets.numel() - 1, total, _stream(stream)))
    return out


def fail_alloc(after: int) -> None:
    """Test hook: the after-th next device allocation fails (<= 0 disarms)."""
    _check(load().kdt_debug_fail_alloc(int(after)))


VISIT_SLOTS = ("lane_nodes", "lane_points", "lane_inserts", "wave_nodes", "wave_points",
               "lane_node_reloads")


def visits(reset: bool = True) -> dict:
    """Work counters of the instrumented library (load it with
    ``load(LIB_COUNTS_PATH)`` first): node boxes and point records read by
    the traversals since the last reset."""
    import numpy as np
    out = np.zeros(8, np.uint64)
    _check(load().kdt_debug_visits(out.ctypes.data, 1 if reset else 0))
    return {k: int(out[i]) for i, k in enumerate(VISIT_SLOTS)}


def valu_probe(blocks: int = 8192, iters: int = 20000, stream=None) -> None:
    """Runs the VALU-only calibration kernel (see include/kdt_debug.h)."""
    out = torch.empty(blocks, dtype=torch.float32, device="cuda")
    _check(load().kdt_debug_valu_probe(_ptr(out), int(blocks), int(iters), _stream(stream)))


def _check(rc: int):
    if rc != KDT_OK:
        raise KdtError(rc, load().kdt_last_error().decode())


def _check_mode(check_finite) -> int:
    """check_finite: True (wait and reject), False (no check) or "deferred"
    (no wait; Tree.check() reports it later)."""
    if check_finite == "deferred":
        return 2
    return 1 if check_finite else 0


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _dev(t: torch.Tensor, dtype, name: str, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


@dataclass
class Info:
    n: int
    d: int
    leaf_size: int
    levels: int
    stride: int
    n_nodes: int


class Tree:
    """A device-resident k-d tree (library-owned; freed with the object)."""

    def __init__(self, points: torch.Tensor, leaf_size: int = 32, check_finite: bool = True,
                 stream=None, split_rule: int = SPLIT_MEDIAN, tune_k: int = 0):
        """split_rule: SPLIT_MEDIAN (balanced) or SPLIT_MIDPOINT (the paper's
        sliding midpoint, data-dependent depth).  leaf_size 0: the tuned
        leaf size for the shape and the kNN k ``tune_k`` (0: 32)."""
        lib = load()
        points = _dev(points, torch.float32, "points")
        if points.dim() != 2:
            raise ValueError("points must be [n][d]")
        self._h = C.c_void_p()
        opts = BuildOpts(leaf_size, _check_mode(check_finite), int(split_rule), int(tune_k))
        _check(lib.kdt_build(_ptr(points), points.shape[0], points.shape[1], C.byref(opts),
                             _stream(stream), C.byref(self._h)))
        info = TreeInfo()
        _check(lib.kdt_tree_get_info(self._h, C.byref(info)))
        self.info = Info(info.n, info.d, info.leaf_size, info.levels, info.stride, info.n_nodes)
        self.n, self.d = info.n, info.d
        self.device = points.device

    def check(self, stream=None) -> None:
        """Raises KdtError (KDT_EINVAL) if a deferred finiteness check
        (check_finite="deferred") found a NaN or infinite coordinate."""
        _check(load().kdt_tree_check(self._h, _stream(stream)))

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.kdt_free(h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def perm_ptr(self) -> int:
        """Device address of the tree order (n int32, owned by the tree)."""
        return int(load().kdt_tree_perm(self._h))

    def gather(self, values: torch.Tensor, stream=None) -> torch.Tensor:
        """Per-point values (rows of 4-byte elements, input order) in tree
        order: out[t] = values[perm[t]]."""
        return self._permute(values, "kdt_tree_gather", stream)

    def scatter(self, values: torch.Tensor, stream=None) -> torch.Tensor:
        """Per-point values in tree order back in input order:
        out[perm[t]] = values[t]."""
        return self._permute(values, "kdt_tree_scatter", stream)

    def _permute(self, values, fn, stream):
        if values.dtype not in (torch.float32, torch.int32):
            raise TypeError("values must be float32 or int32")
        if values.shape[0] != self.n:
            raise ValueError(f"values need {self.n} rows")
        values = _dev(values.contiguous(), values.dtype, "values")
        width = values.numel() // max(self.n, 1)
        out = torch.empty_like(values)
        _check(getattr(load(), fn)(self._h, _ptr(values), int(width), _ptr(out),
                                   _stream(stream)))
        return out

    def query_order(self, queries: torch.Tensor, kind: int = 0, stream=None) -> torch.Tensor:
        """Permutation of the queries along the tree (reusable through ``order=``).

        kind 0: Hilbert curve over the root box (d <= 4), the order of per-lane
        kNN and ball counts; kind 1: tree-leaf order, the order of wave-packet kNN.
        """
        nq = queries.shape[0]
        queries = _dev(queries, torch.float32, "queries", (nq, self.d))
        order = torch.empty(nq, dtype=torch.int32, device=self.device)
        _check(load().kdt_query_order(self._h, _ptr(queries), nq, int(kind), _ptr(order),
                                      _stream(stream)))
        return order

    def knn(self, queries: torch.Tensor | None, k: int, kth_only: int = 0,
            sort_queries: bool = True, traversal: int = 0, order: torch.Tensor | None = None,
            period=None, stream=None, tree_rows: bool = False):
        """k nearest neighbours, ascending by (d2, index): (idx [nq][k], d2 [nq][k]).

        ``queries=None`` queries every point of the tree (row i = input point i;
        with ``tree_rows`` row t = the tree's t-th point, input point perm[t]).
        ``kth_only=1`` returns only d2 of the k-th neighbour, ``2`` its distance.
        ``period`` (one value or one per axis): distances on the D-torus, every
        point and query in [0, period).
        """
        nq = self.n if queries is None else queries.shape[0]
        if queries is not None:
            queries = _dev(queries, torch.float32, "queries", (nq, self.d))
        per = _periods(period, self.d)
        opts = QueryOpts(1 if sort_queries else 0, int(traversal), _ptr(order), 0, per,
                         1 if tree_rows else 0)
        if kth_only:
            d2 = torch.empty(nq, dtype=torch.float32, device=self.device)
            _check(load().kdt_knn(self._h, _ptr(queries), nq, k, None, _ptr(d2), kth_only,
                                  C.byref(opts), _stream(stream)))
            return d2
        idx = torch.empty((nq, k), dtype=torch.int32, device=self.device)
        d2 = torch.empty((nq, k), dtype=torch.float32, device=self.device)
        _check(load().kdt_knn(self._h, _ptr(queries), nq, k, _ptr(idx), _ptr(d2), 0,
                              C.byref(opts), _stream(stream)))
        return idx, d2

    def knn_noalloc(self, queries: torch.Tensor | None, k: int, d2: torch.Tensor,
                    idx: torch.Tensor | None = None, kth_only: int = 0,
                    sort_queries: bool = True, traversal: int = 0,
                    order: torch.Tensor | None = None, stream=None,
                    tree_rows: bool = False) -> None:
        """kNN into caller-given outputs through ``kdt_knn_noalloc`` (no
        allocation anywhere: the library's static scratch orders the queries).

        ``d2`` is [nq][k] float32 (or [nq] with ``kth_only``), ``idx`` [nq][k]
        int32 or None.  k <= 64, open boundaries.
        """
        nq = self.n if queries is None else queries.shape[0]
        if queries is not None:
            queries = _dev(queries, torch.float32, "queries", (nq, self.d))
        d2 = _dev(d2, torch.float32, "d2", (nq,) if kth_only else (nq, k))
        if idx is not None:
            if kth_only:
                raise ValueError("idx must be None with kth_only")
            idx = _dev(idx, torch.int32, "idx", (nq, k))
        opts = QueryOpts(1 if sort_queries else 0, int(traversal), _ptr(order), 0, None,
                         1 if tree_rows else 0)
        _check(load().kdt_knn_noalloc(self._h, _ptr(queries), nq, k, _ptr(idx), _ptr(d2),
                                      kth_only, C.byref(opts), _stream(stream)))

    def range(self, queries: torch.Tensor | None, r: float, lists: bool = False,
              sort_queries: bool = True, order: torch.Tensor | None = None, traversal: int = 0,
              split_budget: int = 0, period=None, stream=None, tree_rows: bool = False):
        """Closed-ball counts; with ``lists`` also CSR (offsets int64, idx int32).

        ``split_budget`` > 0 makes every wave of the wave-shared count hand
        subtrees on to later launches after that many node visits (results are
        identical; 0 keeps the default schedule).  ``period``: balls on the
        D-torus, as in ``knn``.  ``tree_rows``: self-query rows in tree order.
        """
        nq = self.n if queries is None else queries.shape[0]
        if queries is not None:
            queries = _dev(queries, torch.float32, "queries", (nq, self.d))
        per = _periods(period, self.d)
        opts = QueryOpts(1 if sort_queries else 0, int(traversal), _ptr(order), int(split_budget),
                         per, 1 if tree_rows else 0)
        count = torch.empty(nq, dtype=torch.int32, device=self.device)
        lib = load()
        if not lists:
            _check(lib.kdt_range(self._h, _ptr(queries), nq, float(r), _ptr(count), None, None, 0,
                                 None, C.byref(opts), _stream(stream)))
            return count
        offsets = torch.empty(nq + 1, dtype=torch.int64, device=self.device)
        req = C.c_int64(0)
        _check(lib.kdt_range(self._h, _ptr(queries), nq, float(r), _ptr(count), _ptr(offsets),
                             None, 0, C.byref(req), C.byref(opts), _stream(stream)))
        idx = torch.empty(max(req.value, 1), dtype=torch.int32, device=self.device)
        opts.counts_given = 1  # the sizing call above wrote count and offsets
        _check(lib.kdt_range(self._h, _ptr(queries), nq, float(r), _ptr(count), _ptr(offsets),
                             _ptr(idx), idx.numel(), C.byref(req), C.byref(opts),
                             _stream(stream)))
        return count, offsets, idx[:req.value]

    def box(self, lo: torch.Tensor, hi: torch.Tensor, lists: bool = False,
            sort_queries: bool = True, order: torch.Tensor | None = None, traversal: int = 0,
            split_budget: int = 0, stream=None):
        """Points inside the closed boxes [lo, hi] (each [nq][d]): counts; with
        ``lists`` also CSR (offsets int64, ascending input indices int32)."""
        nq = lo.shape[0]
        lo = _dev(lo, torch.float32, "lo", (nq, self.d))
        hi = _dev(hi, torch.float32, "hi", (nq, self.d))
        opts = QueryOpts(1 if sort_queries else 0, int(traversal), _ptr(order), int(split_budget))
        count = torch.empty(nq, dtype=torch.int32, device=self.device)
        lib = load()
        if not lists:
            _check(lib.kdt_box(self._h, _ptr(lo), _ptr(hi), nq, _ptr(count), None, None, 0, None,
                               C.byref(opts), _stream(stream)))
            return count
        offsets = torch.empty(nq + 1, dtype=torch.int64, device=self.device)
        req = C.c_int64(0)
        _check(lib.kdt_box(self._h, _ptr(lo), _ptr(hi), nq, _ptr(count), _ptr(offsets), None, 0,
                           C.byref(req), C.byref(opts), _stream(stream)))
        idx = torch.empty(max(req.value, 1), dtype=torch.int32, device=self.device)
        _check(lib.kdt_box(self._h, _ptr(lo), _ptr(hi), nq, _ptr(count), _ptr(offsets), _ptr(idx),
                           idx.numel(), C.byref(req), C.byref(opts), _stream(stream)))
        return count, offsets, idx[:req.value]

    def fof(self, linking_length: float, count_groups: bool = False, period=None, stream=None):
        """Friends-of-friends labels (smallest input index of each group).

        ``period``: groups on the D-torus, as in ``knn``.
        """
        labels = torch.empty(self.n, dtype=torch.int32, device=self.device)
        ng = C.c_int64(0)
        if period is not None:
            _check(load().kdt_fof_torus(self._h, float(linking_length), _periods(period, self.d),
                                        _ptr(labels), C.byref(ng) if count_groups else None,
                                        _stream(stream)))
            return (labels, ng.value) if count_groups else labels
        _check(load().kdt_fof(self._h, float(linking_length), _ptr(labels),
                              C.byref(ng) if count_groups else None, _stream(stream)))
        return (labels, ng.value) if count_groups else labels

    def export(self, stream=None) -> dict:
        """Copies the tree to host numpy arrays (for inspection and tests)."""
        import numpy as np
        i = self.info
        out = dict(pts=np.empty((i.n, i.d), np.float32), perm=np.empty(i.n, np.int32),
                   lo=np.empty((i.n_nodes, i.d), np.float32),
                   hi=np.empty((i.n_nodes, i.d), np.float32),
                   axis=np.empty(i.n_nodes, np.int32), split=np.empty(i.n_nodes, np.float32))
        _check(load().kdt_tree_export(self._h, out["pts"].ctypes.data, out["perm"].ctypes.data,
                                      out["lo"].ctypes.data, out["hi"].ctypes.data,
                                      out["axis"].ctypes.data, out["split"].ctypes.data,
                                      _stream(stream)))
        for key in ("left", "begin", "end", "level"):
            out[key] = np.empty(i.n_nodes, np.int32)
        _check(load().kdt_tree_nodes(self._h, out["left"].ctypes.data, out["begin"].ctypes.data,
                                     out["end"].ctypes.data, out["level"].ctypes.data,
                                     _stream(stream)))
        return out


class TreeF64(Tree):
    """A tree over float64 coordinates (kdt_build_f64): its queries compute in
    float64 (``knn``, ``range``); the float32 queries are refused."""

    def __init__(self, points: torch.Tensor, leaf_size: int = 32, check_finite: bool = True,
                 stream=None, split_rule: int = SPLIT_MEDIAN, tune_k: int = 0):
        lib = load()
        points = _dev(points, torch.float64, "points")
        if points.dim() != 2:
            raise ValueError("points must be [n][d]")
        self._h = C.c_void_p()
        opts = BuildOpts(leaf_size, 1 if check_finite else 0, int(split_rule), int(tune_k))
        _check(lib.kdt_build_f64(_ptr(points), points.shape[0], points.shape[1], C.byref(opts),
                                 _stream(stream), C.byref(self._h)))
        info = TreeInfo()
        _check(lib.kdt_tree_get_info(self._h, C.byref(info)))
        self.info = Info(info.n, info.d, info.leaf_size, info.levels, info.stride, info.n_nodes)
        self.n, self.d = info.n, info.d
        self.device = points.device

    def knn(self, queries: torch.Tensor | None, k: int, sort_queries: bool = True,
            order: torch.Tensor | None = None, stream=None, tree_rows: bool = False, **unused):
        """(idx int32 [nq][k], d2 float64 [nq][k]), ascending by (d2, index)."""
        nq = self.n if queries is None else queries.shape[0]
        if queries is not None:
            queries = _dev(queries, torch.float64, "queries", (nq, self.d))
        opts = QueryOpts(1 if sort_queries else 0, 0, _ptr(order), 0, None,
                         1 if tree_rows else 0)
        idx = torch.empty((nq, k), dtype=torch.int32, device=self.device)
        d2 = torch.empty((nq, k), dtype=torch.float64, device=self.device)
        _check(load().kdt_knn_f64(self._h, _ptr(queries), nq, k, _ptr(idx), _ptr(d2),
                                  C.byref(opts), _stream(stream)))
        return idx, d2

    def range(self, queries: torch.Tensor | None, r: float, lists: bool = False,
              sort_queries: bool = True, order: torch.Tensor | None = None, stream=None,
              tree_rows: bool = False, **unused):
        """Closed-ball counts in float64; with ``lists`` also CSR."""
        nq = self.n if queries is None else queries.shape[0]
        if queries is not None:
            queries = _dev(queries, torch.float64, "queries", (nq, self.d))
        opts = QueryOpts(1 if sort_queries else 0, 0, _ptr(order), 0, None,
                         1 if tree_rows else 0)
        count = torch.empty(nq, dtype=torch.int32, device=self.device)
        lib = load()
        if not lists:
            _check(lib.kdt_range_f64(self._h, _ptr(queries), nq, float(r), _ptr(count), None,
                                     None, 0, None, C.byref(opts), _stream(stream)))
            return count
        offsets = torch.empty(nq + 1, dtype=torch.int64, device=self.device)
        req = C.c_int64(0)
        _check(lib.kdt_range_f64(self._h, _ptr(queries), nq, float(r), _ptr(count),
                                 _ptr(offsets), None, 0, C.byref(req), C.byref(opts),
                                 _stream(stream)))
        idx = torch.empty(max(req.value, 1), dtype=torch.int32, device=self.device)
        _check(lib.kdt_range_f64(self._h, _ptr(queries), nq, float(r), _ptr(count),
                                 _ptr(offsets), _ptr(idx), idx.numel(), C.byref(req),
                                 C.byref(opts), _stream(stream)))
        return count, offsets, idx[:req.value]


def build_f64(points: torch.Tensor, leaf_size: int = 32, check_finite: bool = True,
              stream=None, split_rule: int = SPLIT_MEDIAN, tune_k: int = 0) -> TreeF64:
    return TreeF64(points, leaf_size, check_finite, stream, split_rule, tune_k)


def build(points: torch.Tensor, leaf_size: int = 32, check_finite: bool = True,
          stream=None, split_rule: int = SPLIT_MEDIAN, tune_k: int = 0) -> Tree:
    return Tree(points, leaf_size, check_finite, stream, split_rule, tune_k)


def make_grid(lo, cell: float, shape, periodic: bool = False) -> Grid:
    g = Grid()
    for a in range(3):
        g.lo[a] = float(lo[a])
        g.n[a] = int(shape[a])
    g.cell = float(cell)
    g.periodic = 1 if periodic else 0
    return g


def p2m(x: torch.Tensor, m: torch.Tensor, h: torch.Tensor, lo, cell: float, shape,
        order_ptr: int | None = None, out: torch.Tensor | None = None, stream=None,
        periodic: bool = False):
    """Adaptive SPH deposit: float32 mass per cell, shape ``shape``.
    ``periodic``: the mesh box is a 3-torus (every H below half a period)."""
    n = x.shape[0]
    x = _dev(x, torch.float32, "x", (n, 3))
    m = _dev(m, torch.float32, "m", (n,))
    h = _dev(h, torch.float32, "h", (n,))
    if out is None:
        out = torch.empty(tuple(shape), dtype=torch.float32, device=x.device)
    g = make_grid(lo, cell, shape, periodic)
    _check(load().kdt_p2m(_ptr(x), _ptr(m), _ptr(h), n, C.byref(g), order_ptr, _ptr(out),
                          _stream(stream)))
    return out


CLOUD_SCHEMES = {"ngp": 1, "cic": 2, "tsc": 3}


def p2m_cloud(x: torch.Tensor, m: torch.Tensor, lo, cell: float, shape, scheme: str,
              order_ptr: int | None = None, out: torch.Tensor | None = None, stream=None,
              periodic: bool = False):
    """Fixed-cloud deposit ("ngp", "cic" or "tsc"): float32 mass per cell."""
    n = x.shape[0]
    x = _dev(x, torch.float32, "x", (n, 3))
    m = _dev(m, torch.float32, "m", (n,))
    if out is None:
        out = torch.empty(tuple(shape), dtype=torch.float32, device=x.device)
    g = make_grid(lo, cell, shape, periodic)
    _check(load().kdt_p2m_cloud(_ptr(x), _ptr(m), n, C.byref(g), CLOUD_SCHEMES[scheme],
                                order_ptr, _ptr(out), _stream(stream)))
    return out


def p2m_backward(x, m, h, lo, cell, shape, grad, order_ptr=None, need_m=True, need_x=True,
                 stream=None, periodic: bool = False):
    """(dL/dm, dL/dx) of L = sum(grad * p2m(x, m, h)), h held fixed."""
    n = x.shape[0]
    x = _dev(x, torch.float32, "x", (n, 3))
    m = _dev(m, torch.float32, "m", (n,))
    h = _dev(h, torch.float32, "h", (n,))
    grad = _dev(grad.contiguous(), torch.float32, "grad")
    gm = torch.empty(n, dtype=torch.float32, device=x.device) if need_m else None
    gx = torch.empty((n, 3), dtype=torch.float32, device=x.device) if need_x else None
    g = make_grid(lo, cell, shape, periodic)
    _check(load().kdt_p2m_backward(_ptr(x), _ptr(m), _ptr(h), n, C.byref(g), order_ptr,
                                   _ptr(grad), _ptr(gm), _ptr(gx), _stream(stream)))
    return gm, gx


def p2m_tree(tree: "Tree", m: torch.Tensor, h: torch.Tensor | None, lo, cell: float, shape,
             scheme: str = "sph", out: torch.Tensor | None = None, stream=None,
             periodic: bool = False):
    """Deposit of the tree's points (positions from its records) with m and
    h (None for the fixed clouds) in tree order: float32 mass per cell."""
    m = _dev(m, torch.float32, "m", (tree.n,))
    if h is not None:
        h = _dev(h, torch.float32, "h", (tree.n,))
    if out is None:
        out = torch.empty(tuple(shape), dtype=torch.float32, device=tree.device)
    g = make_grid(lo, cell, shape, periodic)
    code = 0 if scheme == "sph" else CLOUD_SCHEMES[scheme]
    _check(load().kdt_p2m_tree(tree._h, _ptr(m), _ptr(h), C.byref(g), code, _ptr(out),
                               _stream(stream)))
    return out


def p2m_tree_backward(tree: "Tree", m, h, lo, cell, shape, grad, need_m=True, need_x=True,
                      stream=None, periodic: bool = False):
    """(dL/dm, dL/dx) in tree order for L = sum(grad * p2m_tree(tree, m, h))."""
    m = _dev(m, torch.float32, "m", (tree.n,))
    h = _dev(h, torch.float32, "h", (tree.n,))
    grad = _dev(grad.contiguous(), torch.float32, "grad")
    gm = torch.empty(tree.n, dtype=torch.float32, device=tree.device) if need_m else None
    gx = torch.empty((tree.n, 3), dtype=torch.float32, device=tree.device) if need_x else None
    g = make_grid(lo, cell, shape, periodic)
    _check(load().kdt_p2m_tree_backward(tree._h, _ptr(m), _ptr(h), C.byref(g), _ptr(grad),
                                        _ptr(gm), _ptr(gx), _stream(stream)))
    return gm, gx


class P2M(torch.autograd.Function):
    """Differentiable deposit: gradients for masses and positions, h held fixed."""

    @staticmethod
    def forward(ctx, x, m, h, grid):
        """grid: (lo, cell, shape, order_ptr) or (lo, cell, shape, order_ptr, periodic)."""
        lo, cell, shape, order_ptr = grid[:4]
        periodic = bool(grid[4]) if len(grid) > 4 else False
        ctx.save_for_backward(x, m, h)
        ctx.grid = (lo, cell, shape, order_ptr, periodic)
        return p2m(x.detach(), m.detach(), h.detach(), lo, cell, shape, order_ptr,
                   periodic=periodic)

    @staticmethod
    def backward(ctx, g):
        x, m, h = ctx.saved_tensors
        lo, cell, shape, order_ptr, periodic = ctx.grid
        gm, gx = p2m_backward(x.detach(), m.detach(), h.detach(), lo, cell, shape, g,
                              order_ptr, need_m=ctx.needs_input_grad[1],
                              need_x=ctx.needs_input_grad[0], periodic=periodic)
        return gx, gm, None, None


class BatchPlan:
    """Many point sets of uneven size: fixed shapes, one launch per batch."""

    def __init__(self, offsets, d: int, k: int, leaf_size: int = 32, traversal: int = 0):
        """traversal: 0 measured default, 1 one query per lane, 2 wave packets.
        leaf_size 0: each set takes the tuned leaf size of its own size."""
        import numpy as np
        lib = load()
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        self.offsets = off
        self.n_sets = len(off) - 1
        self.total = int(off[-1])
        self.d, self.k = d, k
        self._h = C.c_void_p()
        bo = BuildOpts(leaf_size, 0)
        qo = QueryOpts(1, int(traversal), None)
        _check(lib.kdt_batch_plan_create(off.ctypes.data, self.n_sets, d, k, C.byref(bo),
                                         C.byref(qo), C.byref(self._h)))

    def launch(self, points: torch.Tensor, linking: torch.Tensor, use_graph: int = 1,
               out=None, stream=None):
        """Builds every set and runs kNN (k from the plan) and friends-of-friends.

        use_graph: 1 batched kernels replayed from a hipGraph, 2 the same kernels
        launched eagerly, 0 the per-set baseline (single-tree calls per set).
        """
        points = _dev(points, torch.float32, "points", (self.total, self.d))
        linking = _dev(linking, torch.float32, "linking", (self.n_sets,))
        if out is None:
            dev = points.device
            out = (torch.empty((self.total, self.k), dtype=torch.int32, device=dev),
                   torch.empty((self.total, self.k), dtype=torch.float32, device=dev),
                   torch.empty(self.total, dtype=torch.int32, device=dev))
        idx, d2, labels = out
        _check(load().kdt_batch_launch(self._h, _ptr(points), _ptr(linking), _ptr(idx), _ptr(d2),
                                       _ptr(labels), int(use_graph), _stream(stream)))
        return idx, d2, labels

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.kdt_batch_plan_free(h)
            self._h = None

    def __del__(self):
        self.close()
