"""Helpers for the GPU parity tests (tensor marshalling only)."""
import numpy as np
import pytest


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(a, dtype=None):
    torch = torch_cuda()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t):
    return t.detach().cpu().numpy()


def announce(*parts):
    print("[case]", *parts, flush=True)
