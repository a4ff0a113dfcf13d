"""Helpers for the GPU parity tests (device tensors, printing the case first)."""
from __future__ import annotations

import sys

import numpy as np


def announce(*parts):
    """Print what the next GPU step runs, flushed, so a crash names its case."""
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def to_dev(a, dtype):
    torch = torch_dev()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
