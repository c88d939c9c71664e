"""Pins of the adjoint reference (oracle/adjoint.py): the dense horizontal-space
solve and conjugate gradients agree, and both match central finite differences
of the loss through fully re-converged solves."""
import copy

import numpy as np

import workloads as W
from oracle.problems import OracleProblem
from oracle import solver as O
from oracle import adjoint as A


def _solve(prob, x0, tol=1e-12):
    """PCAL to a relative KKT of tol (beta = 4 exceeds the p-th eigenvalue of
    these small grids; smaller beta lets two columns collapse)."""
    op = OracleProblem(prob)
    res = O.solve(op, x0, O.Options(variant="pcal", beta=4.0, eta0=4.0 + prob.s_bound, tol=tol,
                                    max_iter=20000))
    assert res.status == 0
    return op, res


def test_adjoint_dense_cg_and_finite_differences():
    prob, x0, w = W.ks3d(grid=(5, 4, 4), p=3, alpha=1.0)
    op, res = _solve(prob, x0)
    X, Lam = res.Q, res.Lam
    g = A.weighted_gram_loss_grad(X, w)
    zd, gv_dense = A.adjoint_dense(op, X, Lam, g)
    zc, gv_cg, its, rr = A.adjoint_cg(op, X, Lam, g, tol=1e-13)
    assert np.linalg.norm(gv_cg - gv_dense) <= 1e-9 * np.linalg.norm(gv_dense)
    assert np.linalg.norm(X.T @ zd) <= 1e-12 * np.linalg.norm(zd)       # horizontal
    h = 1e-4 * float(np.max(np.abs(prob.v)))
    for s in range(3):
        dv = W.random_matrix(21, prob.n, salt=s)
        dv /= np.linalg.norm(dv)
        vals = []
        for sgn in (+1.0, -1.0):
            pp = copy.deepcopy(prob)
            pp.v = prob.v + sgn * h * dv
            # warm start from X*: the starting KKT is already O(h), so the
            # relative tolerance 1e-8 means an absolute KKT of ~1e-12
            _, r = _solve(pp, X, tol=1e-8)
            assert r.kkt_abs <= 1e-11
            vals.append(A.weighted_gram_loss(r.Q, w))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gv_dense @ dv) <= 1e-6 * max(abs(fd), 1e-3 * np.linalg.norm(gv_dense))
