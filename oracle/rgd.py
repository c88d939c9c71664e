"""An independent feasible solver used only to pin the oracle's converged objective.

Test infrastructure only (see the package docstring).

Riemannian gradient descent on the Stiefel manifold with the QR retraction
(the projection-like retraction that the paper's MOptQR comparator uses,
Table 1), a Barzilai-Borwein trial step and Armijo backtracking on f:
    R(X)   = grad f(X) - X Psi(X^T grad f(X))      (the KKT residual of (kkt2))
    X_new  = qf(X - tau R(X)),  qf = Q factor with diag(R) > 0.
It shares nothing with the PLAM / PCAL loop beyond the problem's f and grad f.
"""
from __future__ import annotations

import numpy as np


def _qf(Y):
    q, r = np.linalg.qr(Y)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def _rgrad(op, X):
    G = op.grad(X)
    return G - X @ (0.5 * (X.T @ G + G.T @ X))


def solve(op, X0, tol=1e-9, max_iter=20000, tau0=None):
    X = _qf(np.array(X0, dtype=np.float64))
    R = _rgrad(op, X)
    r0 = np.linalg.norm(R)
    f = op.f(X)
    tau = tau0 if tau0 is not None else 1.0 / max(op.s_bound, 1.0)
    X_prev = R_prev = None
    it = 0
    for it in range(max_iter):
        nr = np.linalg.norm(R)
        if nr <= tol * r0:
            break
        if X_prev is not None:
            s = (X - X_prev).ravel()
            y = (R - R_prev).ravel()
            sy = abs(float(s @ y))
            if sy > 0:
                tau = float(s @ s) / sy
        t = tau
        while True:
            Xn = _qf(X - t * R)
            fn = op.f(Xn)
            if fn <= f - 1e-4 * t * nr * nr or t < 1e-12:
                break
            t *= 0.5
        X_prev, R_prev = X, R
        X, f = Xn, fn
        R = _rgrad(op, X)
    return X, f, float(np.linalg.norm(R) / r0), it
