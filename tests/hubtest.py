"""Test helpers: load (or build once) the HIP library and the oracle, and
move seeded inputs to the GPU.  Nothing here computes the method."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1007_3432_amd import hub  # noqa: E402


def ensure_built() -> None:
    if not os.path.exists(hub.LIB_PATH):
        from paper_1007_3432_amd import build
        build.build()
    hub.load()


def to_dev(a: np.ndarray, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def empty(n: int, hdtype: int):
    import torch
    return torch.empty(n, dtype=hub._torch_dtype(hdtype), device="cuda:0")


def rel_err(a: np.ndarray, b: np.ndarray) -> float:
    """Norm-wise relative difference |a - b| / |b|."""
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def log_case(msg: str) -> None:
    print(f"[case] {msg}", flush=True)
