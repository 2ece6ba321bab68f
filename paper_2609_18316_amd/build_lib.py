"""Compiles the HIP sources under ``csrc/`` into ``libkdt.so`` for gfx950.

Flags that matter for results:
  -ffp-contract=off   every float32 multiply and add of a squared distance is
                      rounded on its own (no fused multiply-add), which makes
                      kNN, ball and grouping results bit-exact;
  -munsafe-fp-atomics float64 atomic adds use the hardware instructions;
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      keeps the compiler from emitting packed float32 ops.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libkdt.so")
# The instrumented variant (KDT_COUNT_VISITS): the same kernels counting the
# node boxes and point records their traversals read, for the algorithmic
# bytes of the roofline.  Measurement only; the product path loads LIB.
BUILD_COUNTS = os.path.join(HERE, "_build_counts")
LIB_COUNTS = os.path.join(HERE, "libkdt_counts.so")
ARCH = os.environ.get("KDT_OFFLOAD_ARCH", "gfx950")

SOURCES = ["kdt_api.hip", "kdt_build.hip", "kdt_query.hip", "kdt_fof.hip", "kdt_p2m.hip",
           "kdt_batch.hip", "kdt_packet.hip", "kdt_box.hip", "kdt_bigk.hip",
           "kdt_torus.hip", "kdt_noalloc.hip", "kdt_midpoint.hip", "kdt_tuning.hip",
           "kdt_f64.hip", "kdt_sort.hip", "kdt_rowsort.hip"]

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def _compile(src: str, counts: bool = False) -> str:
    obj = os.path.join(BUILD_COUNTS if counts else BUILD, os.path.splitext(src)[0] + ".o")
    extra = ["-DKDT_COUNT_VISITS=1"] if counts else []
    cmd = [_hipcc(), *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(jobs: int = 8, counts: bool = False) -> str:
    """Compiles every source (always) and links ``libkdt.so`` (with
    ``counts``: the instrumented ``libkdt_counts.so``); returns its path."""
    os.makedirs(BUILD_COUNTS if counts else BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(lambda s: _compile(s, counts), srcs))
    lib = LIB_COUNTS if counts else LIB
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "-shared", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else 8))
