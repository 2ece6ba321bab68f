"""Compiles the C oracle into ``oracle/libkdt_oracle.so`` with gcc.

The oracle is test infrastructure (see ``kdt_oracle.c``).  It is built with
``-ffp-contract=off`` so that every float32 multiply and add in the distance
sums is rounded on its own, and without any fast-math or flush-to-zero flag.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kdt_oracle.c")
LIB = os.path.join(HERE, "libkdt_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = True, extra: list[str] | None = None, out: str | None = None) -> str:
    """Compile the oracle; returns the path of the shared library."""
    out = out or LIB
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, *(extra or []), SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
