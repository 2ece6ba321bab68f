"""The library's radix sort (it orders the queries along the tree and the
deposit's particles): bit-identical to numpy's stable sort on the same key
bits, for sizes spanning several tiles and a ragged tail, full and partial
bit ranges, heavy ties, and every digit value.  Its exclusive scan (the CSR
offsets of the ball lists, the sliding midpoint build's ranks): equal to
numpy's cumulative sum, with totals past 2^31 in the 64-bit form."""
import numpy as np
import pytest
import torch

from paper_2609_18316_amd import kdt
from tests.gpu_util import dev, say, to_host

pytestmark = pytest.mark.gpu


def _reference(keys, vals, lo, hi):
    sel = (keys.astype(np.uint64) >> lo) & ((1 << (hi - lo)) - 1)
    order = np.argsort(sel, kind="stable")
    return keys[order], vals[order]


@pytest.mark.parametrize("n", (0, 1, 2, 7, 4095, 4096, 4097, 100003, 1 << 20))
def test_sort_equals_stable_numpy_sort(n):
    dev()
    rng = np.random.Generator(np.random.PCG64(n + 3))
    cases = {
        "full": rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32),
        "ties": rng.integers(0, 5, size=n, dtype=np.uint64).astype(np.uint32) * 0x01010101,
        "sorted": np.arange(n, dtype=np.uint32),
        "reversed": np.arange(n, dtype=np.uint32)[::-1].copy(),
    }
    for name, keys in cases.items():
        for lo, hi in ((0, 32), (0, 30), (0, 13), (8, 24), (5, 6), (0, 0)):
            vals = np.arange(n, dtype=np.int32)
            say(f"radix sort n={n} {name} bits [{lo}, {hi})")
            kt = torch.from_numpy(keys.view(np.int32).copy()).to(dev())
            vt = torch.from_numpy(vals).to(dev())
            kdt.radix_sort(kt, vt, lo, hi)
            ek, ev = _reference(keys, vals, lo, hi)
            np.testing.assert_array_equal(to_host(kt).view(np.uint32), ek)
            np.testing.assert_array_equal(to_host(vt), ev)


def test_sort_rejects_bad_bits():
    dev()
    k = torch.zeros(4, dtype=torch.int32, device=dev())
    v = torch.zeros(4, dtype=torch.int32, device=dev())
    for lo, hi in ((3, 2), (-1, 4), (0, 33)):
        with pytest.raises(kdt.KdtError):
            kdt.radix_sort(k, v, lo, hi)


@pytest.mark.parametrize("n", (0, 1, 2, 255, 256, 4095, 4096, 4097, 1 << 20, 4096 * 300 + 17))
def test_scan_equals_cumulative_sum(n):
    dev()
    rng = np.random.Generator(np.random.PCG64(n + 11))
    cases = {
        "small": rng.integers(0, 8, size=n).astype(np.int32),
        "zeros": np.zeros(n, np.int32),
        "wide": rng.integers(0, 1 << 30, size=n).astype(np.int32),  # totals past 2^31
    }
    for name, v in cases.items():
        say(f"exclusive scan n={n} {name}")
        want = np.concatenate([[0], np.cumsum(v.astype(np.int64))])
        got = to_host(kdt.exclusive_scan(torch.from_numpy(v).to(dev()), 64))
        np.testing.assert_array_equal(got, want)
        if want[-1] < 2 ** 31:
            got = to_host(kdt.exclusive_scan(torch.from_numpy(v).to(dev()), 32))
            np.testing.assert_array_equal(got, want[:-1].astype(np.int32))


def test_scan_rejects_bad_width():
    dev()
    with pytest.raises(kdt.KdtError):
        kdt.exclusive_scan(torch.zeros(4, dtype=torch.int32, device=dev()), 16)


def _rows_case(lengths, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    vals = np.empty(int(off[-1]), np.int32)
    for r, L in enumerate(lengths):  # distinct indices per row, shuffled
        vals[off[r]:off[r + 1]] = rng.permutation(rng.choice(1 << 24, size=L, replace=False))
    return vals, off


@pytest.mark.parametrize("case", ("every_size", "random_mix", "all_small", "long_rows"))
def test_row_sort_equals_numpy(case):
    """Every row of a CSR list ascending: the lengths span the register path
    (<= 64), both LDS paths (<= 1024, <= 16384) and the long-row fallback,
    with empty rows and rows of one entry in between."""
    dev()
    rng = np.random.Generator(np.random.PCG64(len(case)))
    if case == "every_size":
        lengths = [0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 1023, 1024, 1025, 4096, 16383, 16384,
                   16385, 40000, 0, 1]
    elif case == "random_mix":
        lengths = list(rng.geometric(1 / 60, size=20000) - 1) + [3000, 20000, 0, 900]
    elif case == "all_small":
        lengths = list(rng.integers(0, 65, size=100003))
    else:
        lengths = [70000, 5, 17000, 0, 33000]
    vals, off = _rows_case(lengths, 5)
    say(f"row sort {case}: {len(lengths)} rows, {len(vals)} entries")
    got = to_host(kdt.sort_rows(torch.from_numpy(vals).to(dev()), torch.from_numpy(off).to(dev())))
    want = vals.copy()
    for r in range(len(lengths)):
        want[off[r]:off[r + 1]].sort()
    np.testing.assert_array_equal(got, want)


def test_row_sort_empty_and_errors():
    dev()
    got = kdt.sort_rows(torch.zeros(0, dtype=torch.int32, device=dev()),
                        torch.zeros(4, dtype=torch.int64, device=dev()))
    assert got.numel() == 0
    with pytest.raises(kdt.KdtError):  # in place
        v = torch.zeros(4, dtype=torch.int32, device=dev())
        o = torch.tensor([0, 4], dtype=torch.int64, device=dev())
        kdt._check(kdt.load().kdt_debug_sort_rows(kdt._ptr(v), kdt._ptr(v), kdt._ptr(o), 1, 4,
                                                  kdt._stream()))
