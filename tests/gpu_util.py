"""Helpers for the GPU parity tests (device transfer, error measures)."""
import numpy as np


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    return torch


def to_dev(a, dtype):
    torch = torch_cuda()
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def true_rel_res(A, x, b):
    return float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
