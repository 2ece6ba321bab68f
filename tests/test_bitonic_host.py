"""Host check of the workgroup bitonic sort that the large-k rows and the
CSR list rows share: its per-thread phases are host-and-device functions, so
the header compiles for the host as it is, and a harness runs every phase
over every thread in turn (inside a phase the threads touch disjoint keys,
so this is exactly what a workgroup does between its barriers).  Every
size 32..16384 with 128..1024 threads, random, heavily tied and reversed
keys, 64- and 32-bit, must come out equal to std::sort; the same harness
with the strided phase left out must not."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2609_18316_amd", "csrc")

HARNESS = r"""
#define __host__
#define __device__
#define __forceinline__ inline
static inline void __syncthreads() {}
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>
#include "kdt_bitonic.h"
using namespace kdt;

template <class K>
static bool one(int pn, int T, std::mt19937_64& g, int kind) {
  std::vector<K> s(pn + pn / 16, (K)0), ref(pn);
  for (int i = 0; i < pn; ++i) {
    const K v = kind == 0 ? (K)(g() >> 1) : kind == 1 ? (K)(g() % 7) : (K)(pn - i);
    s[pad16(i)] = v;
    ref[i] = v;
  }
  const bool strided = pn >= 256;
  for (int t = 0; t < T; ++t) if (t * 16 < pn) bitonic_first_runs(s.data(), t);
  for (int k = 32; k <= pn; k <<= 1) {
    for (int j = k >> 1; j >= (strided ? 256 : 16); j >>= 1)
      for (int t = 0; t < T; ++t) bitonic_lds_step(s.data(), pn, k, j, t, T);
#ifndef LEAVE_OUT_STRIDED
    if (strided)
      for (int t = 0; t < T; ++t) if (t * 16 < pn) bitonic_strided_steps(s.data(), k, t);
#endif
    for (int t = 0; t < T; ++t) if (t * 16 < pn) bitonic_run_steps(s.data(), k, t);
  }
  std::sort(ref.begin(), ref.end());
  for (int i = 0; i < pn; ++i)
    if (s[pad16(i)] != ref[i]) {
      std::printf("unsorted: pn=%d T=%d kind=%d at %d\n", pn, T, kind, i);
      return false;
    }
  return true;
}

int main() {
  std::mt19937_64 g(2609);
  int cases = 0;
  for (int pn = 32; pn <= 16384; pn <<= 1)
    for (int T : {pn / 16, 128, 256, 1024})
      if (T * 16 >= pn)
        for (int kind = 0; kind < 3; ++kind) {
          if (!one<uint64_t>(pn, T, g, kind) || !one<int32_t>(pn, T, g, kind)) return 1;
          cases += 2;
        }
  std::printf("sorted %d cases\n", cases);
  return 0;
}
"""


def _build(tmp_path, name, extra):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not available")
    inc = tmp_path / "inc" / "hip"
    inc.mkdir(parents=True, exist_ok=True)
    (inc / "hip_runtime.h").write_text("")  # the attributes are defined away above
    src = tmp_path / f"{name}.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / name
    subprocess.run(["g++", "-O2", "-std=c++17", *extra, "-I", str(tmp_path / "inc"), "-I", CSRC,
                    str(src), "-o", str(exe)], check=True, capture_output=True, text=True)
    return exe


def test_workgroup_bitonic_sort_phases_sort(tmp_path):
    exe = _build(tmp_path, "bitonic", [])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("sorted ")


def test_the_check_fails_without_the_strided_phase(tmp_path):
    exe = _build(tmp_path, "bitonic_no_strided", ["-DLEAVE_OUT_STRIDED"])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 1 and r.stdout.startswith("unsorted: pn=256"), r.stdout
