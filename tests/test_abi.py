"""The C ABI library loads on the CPU and exports every entry point that
include/kdt.h declares (no compute calls: there is no GPU here)."""
import os
import re

import pytest

from paper_2609_18316_amd import kdt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols(header="kdt.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kdt_[a-z_0-9]+)\s*\(", src)))


def all_declared_symbols():
    headers = sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    return sorted(set(sum((declared_symbols(h) for h in headers), [])))


def test_header_declares_the_binding_surface():
    names = declared_symbols()
    assert set(names) == set(kdt.EXPORTS), names
    assert set(declared_symbols("kdt_debug.h")) == set(kdt.DEBUG_EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(kdt.LIB_PATH):
        pytest.fail("libkdt.so is not built (run __graft_entry__.build())")
    lib = kdt.load()
    missing = [n for n in all_declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


# ctypes mirrors of the header's structs: (C type, binding class)
STRUCTS = (("kdt_build_opts", kdt.BuildOpts), ("kdt_query_opts", kdt.QueryOpts),
           ("kdt_grid", kdt.Grid), ("kdt_tree_info", kdt.TreeInfo))


def test_struct_layouts_match_the_header(tmp_path):
    """Size and every field offset of each ctypes mirror equal what a C
    compiler makes of include/kdt.h."""
    import shutil
    import subprocess
    hip_inc = "/opt/rocm/include"
    if shutil.which("gcc") is None or not os.path.isdir(hip_inc):
        pytest.skip("gcc or the HIP headers are not available")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "kdt.h"', "int main(void) {"]
    for cname, cls in STRUCTS:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I",
                    hip_inc, str(src), "-o", str(exe)], check=True, capture_output=True)
    got = dict((" ".join(l.split()[:2]), int(l.split()[2]))
               for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                       text=True).stdout.splitlines())
    for cname, cls in STRUCTS:
        assert got[f"{cname} size"] == kdt.C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[f"{cname} {fname}"] == getattr(cls, fname).offset, (cname, fname)


def test_period_marshalling():
    """Torus periods: one value for every axis or one per axis, host floats."""
    assert kdt._periods(None, 3) is None
    p = kdt._periods(0.5, 3)
    assert list(p) == [0.5, 0.5, 0.5]
    p = kdt._periods([1.0, 2.0, 0.25], 3)
    assert list(p) == [1.0, 2.0, 0.25]
    with pytest.raises(ValueError):
        kdt._periods([1.0, 2.0], 3)
    opts = kdt.QueryOpts(1, 0, None, 0, kdt._periods(2.0, 2))
    assert opts.period[0] == 2.0 and opts.period[1] == 2.0
    assert not kdt.QueryOpts(1, 0, None).period
