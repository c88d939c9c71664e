"""Shared helpers of the test suite (no method arithmetic here)."""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def to_dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    return t if dtype is None else t.to(dtype).contiguous()


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def projector_distance(X, Y):
    """||X X^T - Y Y^T||_F via the p x p identity (no n x n matrices)."""
    a = np.linalg.norm(X.T @ X) ** 2 + np.linalg.norm(Y.T @ Y) ** 2 - 2 * np.linalg.norm(X.T @ Y) ** 2
    return float(np.sqrt(max(a, 0.0)))
