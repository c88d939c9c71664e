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


def green_1d_extended(rho):
    """phi = T^{-1} rho for T = tridiag(-1,2,-1) by the textbook Green's function
    min(i,j)(n+1-max(i,j))/(n+1), evaluated with prefix / suffix sums in x87
    extended precision (64-bit mantissa) and returned as float64."""
    r = np.asarray(rho, dtype=np.longdouble)
    n = r.shape[0]
    j = np.arange(1, n + 1, dtype=np.longdouble)
    A = np.cumsum(j * r)                          # sum_{j <= i} j rho_j
    t = (n + 1 - j) * r
    B = np.cumsum(t[::-1])[::-1] - t              # sum_{j > i} (n+1-j) rho_j
    phi = ((n + 1 - j) * A + j * B) / (n + 1)
    return phi.astype(np.float64)


def assert_converged(rc, kkt_rel, tol, slack=1.01):
    """The status contract of a converged solve: STF_OK (0) exactly when the
    float64 check of the returned point meets tol; a point just above it after
    the orthonormalization post-process is STF_TOL_UNMET (2)."""
    assert rc in (0, 2), rc
    assert (rc == 0) == (kkt_rel <= tol), (rc, kkt_rel, tol)
    assert kkt_rel <= slack * tol, (kkt_rel, tol)


def maxrel(a, b):
    """Elementwise bound: max |a - b| / max |b| (a relative Frobenius norm can
    hide a localized error, e.g. one wrong boundary plane)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = float(np.max(np.abs(b))) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0)) if b.size else 0.0
