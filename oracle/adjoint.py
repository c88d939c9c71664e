"""Implicit-differentiation reference for d loss(X*) / dV (oracle).

Test infrastructure only (see the package docstring).

X* is a stationary point of min f(X) s.t. X^T X = I with the potential V
entering f through 1/2 tr(X^T Diag(V) X).  First-order optimality (the KKT
system (kkt) of Section 2.1) reads grad f(X) = X Lam with Lam = X^T grad f(X)
symmetric.  f and the losses used here are invariant under X -> X Q for
orthogonal Q, so the solution is a point of the quotient and perturbations are
taken in the horizontal space {xi : X^T xi = 0}.  Differentiating the
stationarity condition along a change dV of the potential gives

    Hess[dX] = -P(Diag(dV) X),
    Hess[xi] = P(grad^2 f(X)[xi] - xi Lam),   P = I - X X^T,

whose bilinear form is the second-order expression of (son).  For a loss l(X*)
with Euclidean gradient g, the adjoint zeta solves Hess[zeta] = P(g), and

    dl/dV_j = -sum_i zeta_ji X_ji     (rowdot(zeta, X)).

Two routes are provided: a dense solve in an orthonormal basis of the
horizontal space (small problems; the reference), and conjugate gradients on
the same operator (larger problems).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def weighted_gram_loss(X, w):
    """l(X) = ||X^T Diag(w) X||_F^2 (invariant under X -> X Q)."""
    M = X.T @ (w[:, None] * X)
    return float(np.sum(M * M))


def weighted_gram_loss_grad(X, w):
    """Euclidean gradient 4 Diag(w) X (X^T Diag(w) X)."""
    M = X.T @ (w[:, None] * X)
    return 4.0 * (w[:, None] * X) @ M


def project(X, Z):
    return Z - X @ (X.T @ Z)


def hess_apply(op, X, Lam, xi):
    return project(X, op.hess_vec(X, xi) - xi @ Lam)


def adjoint_dense(op, X, Lam, g):
    """zeta and dl/dV by a dense solve in an orthonormal basis of the horizontal space."""
    n, p = X.shape
    Qfull, _ = np.linalg.qr(np.concatenate([X, np.eye(n)], axis=1))
    Xp = Qfull[:, p:n]                      # orthonormal complement of span(X)
    m = (n - p) * p
    H = np.empty((m, m))
    for c in range(m):
        K = np.zeros((n - p, p))
        K.flat[c] = 1.0
        H[:, c] = (Xp.T @ hess_apply(op, X, Lam, Xp @ K)).ravel()
    H = 0.5 * (H + H.T)
    rhs = (Xp.T @ project(X, g)).ravel()
    K = sla.solve(H, rhs, assume_a="sym")
    zeta = Xp @ K.reshape(n - p, p)
    return zeta, -np.einsum("ij,ij->i", zeta, X)


def adjoint_cg(op, X, Lam, g, tol=1e-12, maxit=5000):
    """The same solve by conjugate gradients on the horizontal space."""
    b = project(X, g)
    z = np.zeros_like(b)
    r = b.copy()
    d = r.copy()
    rr = float(np.sum(r * r))
    b2 = rr
    it = 0
    for it in range(1, maxit + 1):
        Hd = hess_apply(op, X, Lam, d)
        a = rr / float(np.sum(d * Hd))
        z += a * d
        r -= a * Hd
        rr_new = float(np.sum(r * r))
        if rr_new <= tol * tol * b2:
            rr = rr_new
            break
        d = r + (rr_new / rr) * d
        rr = rr_new
    return z, -np.einsum("ij,ij->i", z, X), it, float(np.sqrt(rr / b2))
