"""The candidate filter of the wave kNN in d = 8 and 16 (matrix-core dot
products of bf16 hi/lo splits, a rounding margin) emulated on the host: no
point whose exact float32 squared distance is within a query's current k-th
distance may go unmarked, at any magnitude of the coordinates.

The emulation follows the kernel's arithmetic step by step (centre = the
wave's first active query, recentred float32 operands, norms, each operand
split into v_hi = bf16(v) and v_lo = bf16(v - v_hi) by round to nearest
even, the three products q_hi.p_hi + q_hi.p_lo + q_lo.p_hi accumulated in
float32, the margin test and the overflow guard).  The accumulation of a
matrix core has no fixed order, so three orders are tried: left to right in
float32, pairs within blocks of four, and exact then rounded once.  Marks
only grow with the threshold, so testing every pair at worst = its own exact
distance covers every list state.  Copies of the filter without the centre,
without the guard, and without the low halves (one bf16 product) are checked
to fail on the same inputs, so the test can tell them apart.
"""
import numpy as np
import pytest

F = np.float32
MARGIN_LO = F(1.0 - 2.0 ** -13)
MARGIN_HI = F(1.0 + 2.0 ** -16)
ABS = F(2.0 ** -100)
GUARD = F(2.0 ** 125)


def exact_d2(q, p):
    """float32 squared distances [nq][np], axes summed left to right, every
    operation rounded on its own (the library's and the oracle's metric)."""
    acc = np.zeros((q.shape[0], p.shape[0]), F)
    with np.errstate(over="ignore", invalid="ignore"):
        for a in range(q.shape[1]):
            t = (p[None, :, a] - q[:, None, a]).astype(F)
            acc = (acc + (t * t).astype(F)).astype(F)
    return acc


def _norms(v):
    n = np.zeros(v.shape[0], F)
    with np.errstate(over="ignore", invalid="ignore"):
        for a in range(v.shape[1]):
            n = (n + (v[:, a] * v[:, a]).astype(F)).astype(F)
    return n


def bf16(v):
    """float32 -> the float32 value of its bf16 rounding (nearest even; NaN
    to a quiet NaN, past the range to infinity), as the kernel rounds."""
    v = np.asarray(v, F)
    u = v.view(np.uint32).astype(np.uint64)
    h = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    h = np.where(nan, np.uint32(0x7FC00000), h)
    return h.view(F)


def split(v):
    with np.errstate(over="ignore", invalid="ignore"):
        hi = bf16(v)
        lo = bf16((v - hi).astype(F))
    return hi, lo


def _dots(qc, pc, order, halves=True):
    """q'.p' [nq][np] from the bf16 splits, accumulated in float32 with the
    given order (halves False: the high halves alone)."""
    qh, ql = split(qc)
    ph, pl = split(pc)
    with np.errstate(over="ignore", invalid="ignore"):
        terms = [(qh[:, None, :].astype(np.float64) * ph[None, :, :]).astype(F)]
        if halves:  # products of bf16 values are exact in float32
            terms = [(qh[:, None, :].astype(np.float64) * pl[None, :, :]).astype(F),
                     (ql[:, None, :].astype(np.float64) * ph[None, :, :]).astype(F)] + terms
        prod = np.concatenate(terms, axis=2)
        if order == "seq":
            acc = np.zeros(prod.shape[:2], F)
            for a in range(prod.shape[2]):
                acc = (acc + prod[:, :, a]).astype(F)
            return acc
        if order == "pairs":
            acc = np.zeros(prod.shape[:2], F)
            for b in range(0, prod.shape[2], 4):
                s01 = (prod[:, :, b] + prod[:, :, b + 1]).astype(F)
                s23 = (prod[:, :, b + 2] + prod[:, :, b + 3]).astype(F)
                acc = (acc + (s01 + s23).astype(F)).astype(F)
            return acc
        if order == "exact":
            return prod.astype(np.float64).sum(axis=2).astype(F)
    raise ValueError(order)


def marks(q, p, worst, order, centre=True, guard=True, halves=True):
    """The filter's decision for every (query, point) pair at threshold
    worst [nq][np] (centre / guard / halves False: the filter without that
    part)."""
    with np.errstate(over="ignore", invalid="ignore"):
        if centre:
            c = q[0]
            qc = (q - c[None, :]).astype(F)
            pc = (p - c[None, :]).astype(F)
        else:
            qc, pc = q, p
        ns = (_norms(qc)[:, None] + _norms(pc)[None, :]).astype(F)
        acc = _dots(qc, pc, order, halves)
        lhs = ((ns * MARGIN_LO).astype(F) - (F(2.0) * acc).astype(F)).astype(F)
        thr = ((worst * MARGIN_HI).astype(F) + ABS).astype(F)
        if guard:
            return ~(lhs > thr) | ~(ns < GUARD)
        if centre:
            return ~(lhs > thr)
        return lhs <= thr


def _cases(d):
    rng = np.random.Generator(np.random.PCG64(1700 + d))
    out = []
    for scale in (1.0, 1e3, 1e9, 1e15, 1e18, 4e18, 1e19):
        # a cloud at `scale` with a spread of 1 % (distances stay finite), and
        # a cloud of the same size next to the origin
        out.append((f"cloud@{scale:g}", (scale * (1 + 0.01 * rng.random((96, d)))).astype(F)))
        out.append((f"spread@{scale:g}", (scale * rng.standard_normal((96, d))).astype(F)))
    # mixed scales: small and huge coordinates in one wave and one leaf
    mix = rng.standard_normal((96, d)) * 10.0 ** rng.integers(0, 20, (96, 1))
    out.append(("mixed", mix.astype(F)))
    # two points whose norms overflow float32 while their dot product does
    # not: only the guard on s keeps the pair (see the kernel's comment)
    a = np.sqrt(1.75e38)
    cos = 3.3e38 / (2 * 1.75e38)
    adv = np.zeros((4, d))
    adv[1, 0] = a
    adv[2, 0], adv[2, 1] = a * cos, a * np.sqrt(1 - cos * cos)
    adv[3, 0] = 1.0
    out.append(("guard", adv.astype(F)))
    return out


@pytest.mark.parametrize("d", (8, 16))
@pytest.mark.parametrize("order", ("seq", "pairs", "exact"))
def test_filter_never_drops_a_candidate(d, order):
    for name, pts in _cases(d):
        q = pts[: len(pts) // 2] if len(pts) > 8 else pts
        p = pts[len(pts) // 2:] if len(pts) > 8 else pts
        ex = exact_d2(q, p)
        m = marks(q, p, ex, order)
        bad = np.argwhere(~m)
        assert bad.size == 0, f"{name}: {len(bad)} candidates dropped, first {bad[:3]}"
        # a point outside every list is still allowed to be dropped: the
        # filter does prune (except where the centre cannot help)
        if name.startswith("cloud"):
            worst = np.full_like(ex, F(0.0))
            pruned = ~marks(q, p, worst, order)
            assert pruned.mean() > 0.5, f"{name}: the filter prunes nothing"


@pytest.mark.parametrize("d", (8, 16))
def test_filter_without_centre_or_guard_fails_these_inputs(d):
    """Without the centre and the guard, large coordinates overflow |q|^2 +
    |p|^2 and the filter drops true neighbours; with the centre alone, the
    pairs whose norms overflow while their dot product does not are still
    dropped.  The emulation must see both."""
    old, no_guard = {}, {}
    for name, pts in _cases(d):
        q = pts[: len(pts) // 2] if len(pts) > 8 else pts
        p = pts[len(pts) // 2:] if len(pts) > 8 else pts
        ex = exact_d2(q, p)
        old[name] = int((~marks(q, p, ex, "seq", centre=False, guard=False)).sum())
        no_guard[name] = int((~marks(q, p, ex, "seq", guard=False)).sum())
    assert old["cloud@1"] == 0 and no_guard["cloud@1"] == 0
    assert old["cloud@1e+19"] > 0 and no_guard["cloud@1e+19"] == 0
    assert old["guard"] > 0 and no_guard["guard"] > 0


@pytest.mark.parametrize("d", (8, 16))
def test_filter_needs_the_low_halves(d):
    """One bf16 product (the high halves alone, 2^-8 per operand) is far
    outside the margin: the same inputs lose true neighbours without the
    low halves, and lose none with them."""
    lost = 0
    for name, pts in _cases(d):
        q = pts[: len(pts) // 2] if len(pts) > 8 else pts
        p = pts[len(pts) // 2:] if len(pts) > 8 else pts
        ex = exact_d2(q, p)
        lost += int((~marks(q, p, ex, "seq", halves=False)).sum())
        assert not (~marks(q, p, ex, "seq")).any()
    assert lost > 0
