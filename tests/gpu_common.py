"""Shared helpers of the GPU parity tests (imported by test_gpu_*.py)."""

import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_07295_amd  # noqa: F401  (fails loudly if the library is missing)
    return torch


def to_dev(torch, arr):
    return torch.as_tensor(np.ascontiguousarray(arr), device="cuda")


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))
