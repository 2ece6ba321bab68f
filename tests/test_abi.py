"""The C ABI library loads on the CPU and exports every entry point that
include/kdt.h declares (no compute calls: there is no GPU here)."""
import os
import re

import pytest

from paper_2609_18316_amd import kdt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "kdt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kdt_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_binding_surface():
    names = declared_symbols()
    assert set(names) == set(kdt.EXPORTS), names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(kdt.LIB_PATH):
        pytest.fail("libkdt.so is not built (run __graft_entry__.build())")
    lib = kdt.load()
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing
