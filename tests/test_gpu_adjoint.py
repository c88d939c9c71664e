"""GPU adjoint (pcal_adjoint_v and the autograd.Function) against the oracle.

The loss is l(X*) = ||X*^T Diag(w) X*||_F^2 (invariant under X* -> X* Q).
* the C-ABI adjoint at the GPU's own X* matches the oracle's dense
  horizontal-space solve evaluated at that same point (1e-8 relative);
* torch.autograd through PCALSolve gives the same dl/dV;
* central finite differences of l through re-converged GPU solves agree
  (1e-5 relative: the solves stop at a KKT of ~1e-11).
"""
import copy

import numpy as np
import pytest
import torch

import workloads as W
from oracle.problems import OracleProblem
from oracle import adjoint as A
from paper_1810_03930_amd import stiefel as S
from paper_1810_03930_amd.autograd import PCALSolve
from tests.helpers import rel, to_dev, to_np

pytestmark = pytest.mark.gpu

BETA = 4.0


def _opts(prob, tol=1e-12, max_iter=20000):
    return S.SolveOptions(variant="pcal", precision="fp64", beta=BETA, eta0=BETA + prob.s_bound,
                          tol=tol, max_iter=max_iter, check_every=50)


def _solve(prob, x0, tol=1e-12):
    dp = S.DeviceProblem.from_host(prob)
    X = to_dev(x0, torch.float64)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        res, x64, lam = S.solve(dp, X, _opts(prob, tol), want_x64=True, want_lambda=True, stream=s)
    torch.cuda.synchronize()
    assert res["rc"] == 0
    return dp, res, x64, lam


def _loss_grad(X, w):
    M = X.T @ (w[:, None] * X)
    return 4.0 * (w[:, None] * X) @ M


@pytest.mark.parametrize("grid,p", [((5, 4, 4), 3), ((7, 6, 5), 5)])
def test_adjoint_matches_dense_reference(grid, p):
    prob, x0, w = W.ks3d(grid=grid, p=p, alpha=1.0)
    dp, res, x64, lam = _solve(prob, x0)
    wd = to_dev(w)
    g = _loss_grad(x64, wd).contiguous()
    gV, its, rr = S.adjoint_v(dp, x64, lam, g, cg_tol=1e-12, cg_maxit=5000)
    torch.cuda.synchronize()
    op = OracleProblem(prob)
    X, Lam = to_np(x64), to_np(lam)
    _, gV_ref = A.adjoint_dense(op, X, Lam, A.weighted_gram_loss_grad(X, w))
    print(f"{grid} p={p}: cg iterations {its}, relres {rr:.2e}, "
          f"rel err {rel(to_np(gV), gV_ref):.2e}")
    assert rr <= 1e-12
    assert rel(to_np(gV), gV_ref) <= 1e-8


def test_autograd_function_and_finite_differences():
    prob, x0, w = W.ks3d(grid=(5, 4, 4), p=3, alpha=1.0)
    dp = S.DeviceProblem.from_host(prob)
    V = to_dev(prob.v).clone().requires_grad_(True)
    X0 = to_dev(x0, torch.float64)
    wd = to_dev(w)
    Xs = PCALSolve.apply(V, dp, X0, _opts(prob), 1e-12, 5000)
    loss = torch.sum((Xs.T @ (wd[:, None] * Xs)) ** 2)
    loss.backward()
    gV = to_np(V.grad)
    op = OracleProblem(prob)
    X = to_np(Xs.detach())
    lam = O_lam(op, X)
    _, gV_ref = A.adjoint_dense(op, X, lam, A.weighted_gram_loss_grad(X, w))
    assert rel(gV, gV_ref) <= 1e-8
    # central differences through warm-started, re-converged GPU solves
    h = 1e-4 * float(np.max(np.abs(prob.v)))
    for sidx in range(2):
        dv = W.random_matrix(31, prob.n, salt=sidx)
        dv /= np.linalg.norm(dv)
        vals = []
        for sgn in (+1.0, -1.0):
            pp = copy.deepcopy(prob)
            pp.v = prob.v + sgn * h * dv
            _, r, xp, _ = _solve(pp, X, tol=1e-8)
            assert r["kkt_abs"] <= 1e-10
            vals.append(A.weighted_gram_loss(to_np(xp), w))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gV @ dv) <= 1e-5 * max(abs(fd), 1e-3 * np.linalg.norm(gV))


def O_lam(op, X):
    G = op.grad(X)
    return 0.5 * (G.T @ X + X.T @ G)
