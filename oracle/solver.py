"""PLAM (Algorithm 2) and PCAL (Algorithm 3) in plain float64 (oracle).

Test infrastructure only (see the package docstring).

Notation follows the paper: Psi(A) = (A + A^T)/2 and Phi(A) = Diag(diag(A))
(Section 1.3); the augmented Lagrangian L_beta and its gradient
    grad_X L_beta(X, Lam) = grad f(X) - X Lam + beta X (X^T X - I)
(Section 2.2, the gradient formula in the proof of Lemma 1).

One iteration k, in the paper's order:
  1. G = grad f(X^k); the multiplier Lam^k = Psi(G^T X^k)       (Alg. 2, step 3)
     and, for PCAL with the heuristic rule, Lam^k += Phi(X^T grad_X L_beta(X, Psi))
                                                                 (Alg. 3, step 3)
  2. the stop test on ||G - X Psi(G^T X)||_F relative to its value at X^0
     (Section 5.1; Section 3.3 explains the use of X Psi instead of X G^T X)
  3. eta^k by one of the rules of Section 5.1
  4. PLAM: X^{k+1} = X^k - grad_X L_beta(X^k, Lam^k) / eta^k   (Section 3.1)
     PCAL: the same point, then every column scaled to unit 2-norm, all
     columns from the same X^k (the closed-form solution in Section 3.2)
After the loop an orthonormalization post-process is applied (Section 5.3,
Table 2); here it is CholeskyQR2 in float64.

Readings where the paper is silent or ambiguous (each is a switch here):
  * BB pair: ``bb_index="standard"`` uses S = X^k - X^{k-1},
    Y = gradL^k - gradL^{k-1} for eta^k (the usual Barzilai-Borwein pair);
    ``"lagged"`` uses S^{k-1}, Y^{k-1} exactly as printed in Section 5.1 for
    the BB quotients.  The differential rule eta_D is printed with the newest
    pair, so it uses (X^k - X^{k-1}, gradL^k - gradL^{k-1}) under both.
  * eta^0 is an input; k counts from 0, so ABB takes BB1 at odd k.
  * A rule whose quotient is not finite or not positive keeps eta^{k-1}.
  * PCAL updates all columns from X^k (one Jacobi sweep per iteration).
  * The stop test is evaluated on X^k before the update; X^k is returned.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.linalg as sla

STATUS_CONVERGED = 0
STATUS_MAX_ITER = 1
STATUS_DIVERGED = -2


def Psi(A: np.ndarray) -> np.ndarray:
    """Average of a square matrix and its transpose (Section 1.3)."""
    return 0.5 * (A + A.T)


def Phi(A: np.ndarray) -> np.ndarray:
    """Diagonal matrix holding the diagonal of A (Section 1.3)."""
    return np.diag(np.diag(A))


@dataclass
class Options:
    variant: str = "pcal"          # "pcal" | "plam"
    beta: float = 1.0
    eta_rule: str = "abb"          # "const" | "diff" | "bb1" | "bb2" | "abb"
    eta0: float = 1.0
    eta_const: float = 1.0         # gamma of the constant rule
    tol: float = 1e-8
    max_iter: int = 3000
    mult: str = "psi_phi"          # "psi" (eq. Lambda1) | "psi_phi" (eq. lambda2, PCAL only)
                                   # | "dual" (dual ascent, eq. (Lambda-alm): PLAM-DA / PCAL-DA)
    bb_index: str = "standard"     # "standard" | "lagged"
    orth_final: bool = True
    feas_blowup: float = 1e3
    record_history: bool = False
    record_iterates: Sequence[int] = ()


@dataclass
class Result:
    status: int
    iters: int
    X: np.ndarray                  # the last iterate (before orthonormalization)
    Q: Optional[np.ndarray]        # after CholeskyQR2 (if requested)
    kkt0: float
    kkt_abs: float                 # ||G - X Psi(G^T X)||_F at the returned point
    kkt_rel: float
    feas: float                    # ||X^T X - I||_F at the returned point
    f: float
    eta_last: float
    Lam: Optional[np.ndarray] = None
    history: Dict[str, List[float]] = field(default_factory=dict)
    iterates: Dict[int, np.ndarray] = field(default_factory=dict)
    # for k in record_iterates (k < iters): the gradL^k the update of iteration k
    # stepped with, and the multiplier Lambda^k it was formed with
    grads: Dict[int, np.ndarray] = field(default_factory=dict)
    mults: Dict[int, np.ndarray] = field(default_factory=dict)


def kkt_residual(op, X: np.ndarray, G: Optional[np.ndarray] = None) -> float:
    """||grad f(X) - X Psi(grad f(X)^T X)||_F (Section 3.3 / Section 5.1)."""
    if G is None:
        G = op.grad(X)
    return float(np.linalg.norm(G - X @ Psi(G.T @ X)))


def feasibility(X: np.ndarray) -> float:
    p = X.shape[1]
    return float(np.linalg.norm(X.T @ X - np.eye(p)))


def cholqr2(X: np.ndarray) -> np.ndarray:
    """CholeskyQR applied twice, float64.

    R1 = chol(X^T X) (upper), Q1 = X R1^{-1}; R2 = chol(Q1^T Q1), Q = Q1 R2^{-1}.
    """
    Q = X
    for _ in range(2):
        R = np.linalg.cholesky(Q.T @ Q).T          # upper triangular, Q^T Q = R^T R
        Q = sla.solve_triangular(R, Q.T, trans="T", lower=False).T
    return Q


def grad_lagrangian(X, G, Lam, beta):
    """grad_X L_beta(X, Lam) = G - X Lam + beta X (X^T X - I)."""
    p = X.shape[1]
    return G - X @ Lam + beta * X @ (X.T @ X - np.eye(p))


def _bb_quotient(rule: str, k: int, s_s: float, s_y: float, y_y: float) -> float:
    """eta from the inner products <S,S>, <S,Y>, <Y,Y> (Section 5.1)."""
    if rule == "diff":
        return np.sqrt(y_y) / np.sqrt(s_s) if s_s > 0 else np.nan
    if rule == "bb1" or (rule == "abb" and k % 2 == 1):
        return abs(s_y) / s_s if s_s > 0 else np.nan
    if rule == "bb2" or rule == "abb":
        return y_y / abs(s_y) if s_y != 0 else np.nan
    raise ValueError(rule)


def solve(op, X0: np.ndarray, opt: Options) -> Result:
    """Run PLAM or PCAL from X0 (float64) and return the iterate and report."""
    if opt.variant not in ("pcal", "plam"):
        raise ValueError(opt.variant)
    if opt.mult == "psi_phi" and opt.variant != "pcal":
        raise ValueError("the Phi-corrected multiplier belongs to PCAL")
    if opt.mult not in ("psi", "psi_phi", "dual"):
        raise ValueError(opt.mult)
    X = np.array(X0, dtype=np.float64, copy=True)
    n, p = X.shape
    I = np.eye(p)
    hist: Dict[str, List[float]] = {"kkt_rel": [], "feas": [], "eta": [], "f": []}
    iterates: Dict[int, np.ndarray] = {}
    grads: Dict[int, np.ndarray] = {}
    mults: Dict[int, np.ndarray] = {}
    rec = set(int(k) for k in opt.record_iterates)

    X_prev = None          # X^{k-1}
    X_prev2 = None         # X^{k-2}
    gL_prev = None         # grad L^{k-1}
    gL_prev2 = None        # grad L^{k-2}
    eta = float(opt.eta0)
    kkt0 = None
    status = STATUS_MAX_ITER
    k = 0
    Lam = None
    Lam_da = None          # the dual-ascent multiplier Lambda^{k-1}
    while True:
        if not np.all(np.isfinite(X)):
            status = STATUS_DIVERGED
            break
        if k in rec:
            iterates[k] = X.copy()
        # step 3: gradient and the closed-form multiplier
        G = op.grad(X)
        W = X.T @ G                      # X^T grad f   (its transpose is G^T X)
        S = X.T @ X
        C = S - I
        Lam_psi = Psi(W)                 # Psi(grad f^T X), eq. (Lambda1)
        kkt = float(np.linalg.norm(G - X @ Lam_psi))
        if kkt0 is None:
            kkt0 = kkt
        feas = float(np.linalg.norm(C))
        if opt.record_history:
            hist["kkt_rel"].append(kkt / kkt0 if kkt0 > 0 else 0.0)
            hist["feas"].append(feas)
            hist["f"].append(op.f(X))
        if not np.isfinite(kkt) or feas > opt.feas_blowup:
            status = STATUS_DIVERGED
            break
        if kkt0 == 0.0 or kkt / kkt0 <= opt.tol:
            status = STATUS_CONVERGED
            break
        if k >= opt.max_iter:
            status = STATUS_MAX_ITER
            break
        # grad_X L_beta(X^k, Psi), then the PCAL diagonal correction, eq. (lambda2)
        R = G - X @ Lam_psi + opt.beta * (X @ C)
        if opt.variant == "pcal" and opt.mult == "psi_phi":
            D = Phi(X.T @ R)
            Lam = Lam_psi + D
            gL = R - X @ D
        elif opt.mult == "dual":
            # PLAM-DA / PCAL-DA (Section 5.3): Step 3 replaced by the dual
            # ascent of the augmented Lagrangian method, eq. (Lambda-alm),
            # Lambda^k = Lambda^{k-1} - beta (X^k^T X^k - I), started from the
            # closed form Psi(G^T X) at X^0
            Lam = Lam_psi if k == 0 else Lam_da - opt.beta * C
            Lam_da = Lam
            gL = G - X @ Lam + opt.beta * (X @ C)
        else:
            Lam = Lam_psi
            gL = R
        # eta^k (Section 5.1)
        if opt.eta_rule == "const":
            eta_k = float(opt.eta_const)
        elif k == 0:
            eta_k = float(opt.eta0)
        else:
            # eta_D is defined with the newest pair under both readings; only the
            # BB quotients are printed with the lagged pair
            if opt.bb_index == "standard" or opt.eta_rule == "diff":
                Sd = X - X_prev
                Yd = gL - gL_prev
            else:
                if k == 1:
                    Sd = None
                else:
                    Sd = X_prev - X_prev2
                    Yd = gL_prev - gL_prev2
            if Sd is None:
                eta_k = float(opt.eta0)
            else:
                q = _bb_quotient(opt.eta_rule, k, float(np.sum(Sd * Sd)),
                                 float(np.sum(Sd * Yd)), float(np.sum(Yd * Yd)))
                eta_k = q if (np.isfinite(q) and q > 0.0) else eta
        eta = eta_k
        if opt.record_history:
            hist["eta"].append(eta)
        if k in rec:
            grads[k] = gL.copy()
            mults[k] = Lam.copy()
        # step 4: the proximal linearized update
        Y = X - gL / eta
        if opt.variant == "pcal":
            Xn = Y / np.linalg.norm(Y, axis=0)[None, :]
        else:
            Xn = Y
        X_prev2, X_prev = X_prev, X
        gL_prev2, gL_prev = gL_prev, gL
        X = Xn
        k += 1

    if status == STATUS_DIVERGED:
        return Result(status=status, iters=k, X=X, Q=None, kkt0=kkt0 or np.nan,
                      kkt_abs=np.nan, kkt_rel=np.nan, feas=np.nan, f=np.nan,
                      eta_last=eta, history=hist, iterates=iterates,
                      grads=grads, mults=mults)
    Q = cholqr2(X) if opt.orth_final else None
    if Q is not None:
        Gq = op.grad(Q)
        kkt_q = float(np.linalg.norm(Gq - Q @ Psi(Gq.T @ Q)))
        return Result(status=status, iters=k, X=X, Q=Q, kkt0=kkt0, kkt_abs=kkt_q,
                      kkt_rel=kkt_q / kkt0, feas=feasibility(Q), f=op.f(Q),
                      eta_last=eta, Lam=Psi(Gq.T @ Q), history=hist, iterates=iterates,
                      grads=grads, mults=mults)
    return Result(status=status, iters=k, X=X, Q=None, kkt0=kkt0, kkt_abs=kkt,
                  kkt_rel=kkt / kkt0, feas=feas, f=op.f(X), eta_last=eta,
                  Lam=Lam_psi, history=hist, iterates=iterates, grads=grads, mults=mults)


def merit(op, X: np.ndarray, beta: float) -> float:
    """The merit function h of Section 4.1:
    h(X) = f(X) - 1/2 <Psi(grad f^T X), X^T X - I> + beta/4 ||X^T X - I||_F^2."""
    p = X.shape[1]
    G = op.grad(X)
    C = X.T @ X - np.eye(p)
    return op.f(X) - 0.5 * float(np.sum(Psi(G.T @ X) * C)) + 0.25 * beta * float(np.sum(C * C))


def moptqr(op, X0: np.ndarray, opt: Options) -> Result:
    """The retraction-based comparator MOptQR with the Cholesky-QR retraction
    (Table 1; Section 5.5 computes its QR with a Cholesky factorization):

        D = grad f(X) - X grad f(X)^T X,   V = X - D / eta,
        V^T V = R^T R (R upper),            X <- V R^{-1}.

    eta (the reciprocal step size) follows the rules of Section 5.1 with the
    pair S = X^k - X^{k-1}, Y = D^k - D^{k-1} (``bb_index`` as for PLAM/PCAL);
    the stop test is the one of Section 5.1.  ``opt.variant``, ``beta`` and
    ``mult`` are not used.  X0 is expected orthonormal.
    """
    X = np.array(X0, dtype=np.float64, copy=True)
    n, p = X.shape
    hist: Dict[str, List[float]] = {"kkt_rel": [], "feas": [], "eta": [], "f": []}
    iterates: Dict[int, np.ndarray] = {}
    grads: Dict[int, np.ndarray] = {}
    rec = set(int(k) for k in opt.record_iterates)
    X_prev = X_prev2 = D_prev = D_prev2 = None
    eta = float(opt.eta0)
    kkt0 = None
    status = STATUS_MAX_ITER
    k = 0
    while True:
        if not np.all(np.isfinite(X)):
            status = STATUS_DIVERGED
            break
        if k in rec:
            iterates[k] = X.copy()
        G = op.grad(X)
        W = X.T @ G
        kkt = float(np.linalg.norm(G - X @ Psi(W)))
        if kkt0 is None:
            kkt0 = kkt
        feas = feasibility(X)
        if opt.record_history:
            hist["kkt_rel"].append(kkt / kkt0 if kkt0 > 0 else 0.0)
            hist["feas"].append(feas)
            hist["f"].append(op.f(X))
        if not np.isfinite(kkt):
            status = STATUS_DIVERGED
            break
        if kkt0 == 0.0 or kkt / kkt0 <= opt.tol:
            status = STATUS_CONVERGED
            break
        if k >= opt.max_iter:
            status = STATUS_MAX_ITER
            break
        D = G - X @ W.T                      # grad f - X grad f^T X
        if opt.eta_rule == "const":
            eta_k = float(opt.eta_const)
        elif k == 0:
            eta_k = float(opt.eta0)
        else:
            if opt.bb_index == "standard" or opt.eta_rule == "diff":
                Sd, Yd = X - X_prev, D - D_prev
            elif k == 1:
                Sd = None
            else:
                Sd, Yd = X_prev - X_prev2, D_prev - D_prev2
            if Sd is None:
                eta_k = float(opt.eta0)
            else:
                q = _bb_quotient(opt.eta_rule, k, float(np.sum(Sd * Sd)),
                                 float(np.sum(Sd * Yd)), float(np.sum(Yd * Yd)))
                eta_k = q if (np.isfinite(q) and q > 0.0) else eta
        eta = eta_k
        if opt.record_history:
            hist["eta"].append(eta)
        if k in rec:
            grads[k] = D.copy()
        V = X - D / eta
        try:
            R = np.linalg.cholesky(V.T @ V).T
        except np.linalg.LinAlgError:
            status = STATUS_DIVERGED
            break
        Xn = sla.solve_triangular(R, V.T, trans="T", lower=False).T
        X_prev2, X_prev = X_prev, X
        D_prev2, D_prev = D_prev, D
        X = Xn
        k += 1
    if status == STATUS_DIVERGED:
        return Result(status=status, iters=k, X=X, Q=None, kkt0=kkt0 or np.nan,
                      kkt_abs=np.nan, kkt_rel=np.nan, feas=np.nan, f=np.nan,
                      eta_last=eta, history=hist, iterates=iterates, grads=grads)
    Q = cholqr2(X) if opt.orth_final else X
    Gq = op.grad(Q)
    kkt_q = float(np.linalg.norm(Gq - Q @ Psi(Gq.T @ Q)))
    return Result(status=status, iters=k, X=X, Q=Q if opt.orth_final else None, kkt0=kkt0,
                  kkt_abs=kkt_q, kkt_rel=kkt_q / kkt0, feas=feasibility(Q), f=op.f(Q),
                  eta_last=eta, Lam=Psi(Gq.T @ Q), history=hist, iterates=iterates,
                  grads=grads)
