"""Shared helpers for the GPU parity tests (no method arithmetic here)."""
import numpy as np
import pytest


def device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def to_dev(x, dev):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)
