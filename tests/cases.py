"""Small structured inputs used by both the oracle pins and the GPU parity tests.

Random numbers only: no distance, tree or query arithmetic lives here.
"""
from __future__ import annotations

import numpy as np

KINDS = ("uniform", "duplicates", "identical", "collinear", "lattice", "normal")


def points(kind: str, n: int, d: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "uniform":
        return rng.random((n, d), dtype=np.float32)
    if kind == "normal":
        return rng.standard_normal((n, d), dtype=np.float32)
    if kind == "duplicates":
        base = rng.random((max(1, n // 4), d), dtype=np.float32)
        return np.ascontiguousarray(base[rng.integers(0, base.shape[0], n)])
    if kind == "identical":
        return np.repeat(rng.random((1, d), dtype=np.float32), n, axis=0)
    if kind == "collinear":
        t = rng.random(n, dtype=np.float32)
        direction = np.zeros(d, np.float32)
        direction[0] = 1.0
        direction[d - 1] = 1.0
        return np.ascontiguousarray((t[:, None] * direction[None, :]).astype(np.float32))
    if kind == "lattice":
        # coordinates on a 1/16 grid: many exactly equal squared distances
        return (rng.integers(0, 8, (n, d)).astype(np.float32) / np.float32(16.0))
    raise ValueError(kind)
