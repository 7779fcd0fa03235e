"""Shared helpers of the GPU tests: tensor conversion and error measures."""
import numpy as np


def rel(a, b):
    """Normwise relative error ||a - b|| / ||b||."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dweighted(psi, ref, D):
    """D-weighted object error ||D (psi - ref)|| / ||D ref||."""
    return float(np.linalg.norm(D * (psi - ref)) / np.linalg.norm(D * ref))


def c64(x):
    return np.ascontiguousarray(np.asarray(x), dtype=np.complex64)


def to_dev(x, dtype=None):
    import torch
    arr = np.ascontiguousarray(x if dtype is None else np.asarray(x, dtype=dtype))
    return torch.from_numpy(arr).to("cuda")


def to_host(t):
    return t.detach().cpu().numpy()
