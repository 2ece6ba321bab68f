"""Helpers for the GPU tests: device handle and host/device conversions."""
from __future__ import annotations

import numpy as np
import pytest
import torch


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def to_host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(msg: str):
    print(msg, flush=True)
