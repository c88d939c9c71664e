"""Pins of the oracle's further problem terms and solvers against what the
paper and the mathematics fix: the block-diagonal operator of Section 5.5,
the exchange term of Problem 6, the linear term of Problem 2, the right
factor of Problem 4, the dual-ascent multiplier of PLAM-DA / PCAL-DA
(Section 5.3) and the MOptQR comparator of Table 1."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linear_sum_assignment

import workloads as W
from oracle.problems import OracleProblem, laplacian_1d, laplacian_eigenvalues_1d
from oracle import solver as O
from oracle import rgd


# ----------------------------------------------------- block operator (5.5) --
def test_block_laplacian_structure_spectrum_and_green_function():
    """Diag(L_1..L_s), L_i = tridiag(-1,2,-1) of order 5 (the last block of
    order n mod 5): the spectrum is the union of the blocks' closed forms and
    L^{-1} is block-diagonal with the textbook Green's function per block."""
    n, b = 23, 5
    L = laplacian_1d(n, b).toarray()
    ev = np.sort(np.concatenate([laplacian_eigenvalues_1d(b)] * 4 + [laplacian_eigenvalues_1d(3)]))
    assert np.allclose(np.linalg.eigvalsh(L), ev, atol=1e-13)
    assert L[4, 5] == 0 and L[5, 4] == 0 and L[3, 4] == -1 and L[20, 19] == 0
    prob, _ = W.ks1d_block(n=n, p=2, block=b)
    op = OracleProblem(prob)
    rho = W.random_uniform(3, n)
    green = np.zeros((n, n))
    for s0 in range(0, n, b):
        m = min(b, n - s0)
        i = np.arange(1, m + 1)[:, None]
        j = np.arange(1, m + 1)[None, :]
        green[s0:s0 + m, s0:s0 + m] = np.minimum(i, j) * (m + 1 - np.maximum(i, j)) / (m + 1)
    assert np.allclose(op.hartree(rho), green @ rho, rtol=1e-14, atol=0)


# ------------------------------------------------------- gradients by FD --
def _problems():
    out = []
    prob, x0 = W.ks_exchange(n=40, p=3, block=5)
    out.append(("exchange", prob, x0))
    prob, x0 = W.ocqp_tridiag(n=40, p=3)
    out.append(("ocqp_tridiag", prob, x0))
    prob, x0 = W.ocqp_dense(n=30, p=3)
    out.append(("ocqp_dense", prob, x0))
    prob, x0 = W.qap_dense(n=30, p=3)
    out.append(("qap", prob, x0))
    return out


@pytest.mark.parametrize("name,prob,x0", _problems(), ids=lambda v: v if isinstance(v, str) else "")
def test_new_terms_gradient_and_hessian_by_finite_differences(name, prob, x0):
    """grad f against Richardson-extrapolated central differences of f, and the
    Hessian-vector product against differences of grad f."""
    op = OracleProblem(prob)
    X = x0 + 0.05 * W.random_matrix(14, x0.shape)
    xi = W.random_matrix(15, x0.shape)

    def cd(h):
        return (op.f(X + h * xi) - op.f(X - h * xi)) / (2 * h)
    fd = (4.0 * cd(5e-5) - cd(1e-4)) / 3.0
    g = op.grad(X)
    assert abs(float(np.sum(g * xi)) - fd) <= 1e-9 * max(abs(fd), 1.0), name
    h = 1e-6
    hv = (op.grad(X + h * xi) - op.grad(X - h * xi)) / (2 * h)
    assert np.linalg.norm(op.hess_vec(X, xi) - hv) <= 1e-7 * np.linalg.norm(hv), name


def test_exchange_energy_on_unit_vectors():
    """X = distinct unit vectors e_j: rho is the indicator of the p rows, so the
    exchange energy is -3/4 gamma p and adds to the Hartree-only energy."""
    n, p = 30, 4
    prob, _ = W.ks_exchange(n=n, p=p, block=5)
    rows = [1, 7, 12, 26]
    X = np.zeros((n, p))
    X[rows, range(p)] = 1.0
    op = OracleProblem(prob)
    prob0, _ = W.ks_exchange(n=n, p=p, block=5)
    prob0.gamma = 0.0
    f0 = OracleProblem(prob0).f(X)
    assert abs(op.f(X) - (f0 - 0.75 * W.EXCHANGE_GAMMA * p)) <= 1e-13 * abs(f0)
    # ... and rho^{1/3} = rho there, so the exchange gradient is -2 gamma X
    assert np.allclose(op.grad(X) - OracleProblem(prob0).grad(X), -2.0 * W.EXCHANGE_GAMMA * X,
                       atol=1e-14)


# ------------------------------------------------ converged values (pins) --
def test_problem4_optimum_is_an_assignment_problem():
    """f = 1/2 tr(X^T A X B) = 1/2 sum_ij lambda_i(A) mu_j(B) (U^T X V)_ij^2, and
    the squares form a column-stochastic, row-substochastic matrix, so the
    minimum over the Stiefel manifold is half the optimal assignment of the
    p eigenvalues of B to distinct eigenvalues of A (scipy's assignment
    solver).  PLAM, PCAL and MOptQR all reach it."""
    prob, x0 = W.qap_dense(n=60, p=5)
    op = OracleProblem(prob)
    cost = np.outer(np.linalg.eigvalsh(prob.B), np.linalg.eigvalsh(prob.A))
    r, c = linear_sum_assignment(cost)
    fstar = 0.5 * cost[r, c].sum()
    b = prob.s_bound + 0.1
    for variant, mult, beta in [("pcal", "psi_phi", 1.0), ("plam", "psi", b)]:
        res = O.solve(op, x0, O.Options(variant=variant, mult=mult, beta=beta,
                                        eta0=beta + prob.s_bound, tol=1e-10, max_iter=20000))
        assert res.status == 0, variant
        assert abs(res.f - fstar) <= 1e-10 * abs(fstar), variant
    res = O.moptqr(op, x0, O.Options(eta0=prob.s_bound, tol=1e-10, max_iter=20000))
    assert res.status == 0 and abs(res.f - fstar) <= 1e-10 * abs(fstar)


@pytest.mark.parametrize("which", ["ocqp_dense", "ocqp_tridiag"])
def test_nonsymmetric_problems_reach_independent_solver(which):
    """Problem 2 (X^T G not symmetric during the iteration): PCAL, PLAM and
    MOptQR reach the objective of the independent Riemannian solver, and at
    the solution Lambda = grad f^T X is symmetric (eq. (closed-multi))."""
    if which == "ocqp_dense":
        prob, x0 = W.ocqp_dense(n=200, p=8)
    else:
        prob, x0 = W.ocqp_tridiag(n=150, p=6)
    op = OracleProblem(prob)
    Xr, fr, kr, _ = rgd.solve(op, x0, tol=1e-11, max_iter=40000)
    assert kr <= 1e-11
    b = prob.s_bound + 0.1
    G0 = op.grad(x0)
    asym = np.linalg.norm(x0.T @ G0 - G0.T @ x0) / np.linalg.norm(x0.T @ G0)
    assert asym >= 1e-3
    for variant, mult, beta in [("pcal", "psi_phi", max(1.0, b)), ("plam", "psi", 2 * b)]:
        res = O.solve(op, x0, O.Options(variant=variant, mult=mult, beta=beta,
                                        eta0=beta + prob.s_bound, tol=1e-10, max_iter=40000))
        assert res.status == 0, (which, variant)
        assert abs(res.f - fr) <= 1e-9 * abs(fr), (which, variant, res.f, fr)
        G = op.grad(res.Q)
        XtG = res.Q.T @ G
        assert np.linalg.norm(XtG - XtG.T) <= 1e-8 * np.linalg.norm(XtG)
    res = O.moptqr(op, x0, O.Options(eta0=prob.s_bound, tol=1e-10, max_iter=40000))
    assert res.status == 0 and abs(res.f - fr) <= 1e-9 * abs(fr)


def test_exchange_problem_minimizers_satisfy_first_and_second_order_conditions():
    """Problem 6 is nonconvex (it has several local minimizers): every solver's
    limit is checked on its own.  The exchange gradient H(X) X keeps X^T G
    symmetric; at each limit Lambda = G^T X is symmetric and stationary, and
    the second-order form of (son) is positive on horizontal directions.
    PCAL with a larger beta and MOptQR land on the Riemannian solver's point."""
    prob, x0 = W.ks_exchange(n=150, p=6, block=5)
    op = OracleProblem(prob)
    G0 = op.grad(x0)
    assert np.linalg.norm(x0.T @ G0 - G0.T @ x0) <= 1e-14 * np.linalg.norm(G0)
    Xr, fr, kr, _ = rgd.solve(op, x0, tol=1e-11, max_iter=40000)
    runs = [O.solve(op, x0, O.Options(variant="pcal", beta=beta, eta0=beta + prob.s_bound,
                                      tol=1e-10, max_iter=40000)) for beta in (1.0, 20.0)]
    runs.append(O.moptqr(op, x0, O.Options(eta0=prob.s_bound, tol=1e-10, max_iter=40000)))
    for res in runs:
        assert res.status == 0
        X, Lam = res.Q, res.Lam
        G = op.grad(X)
        assert np.linalg.norm(G - X @ Lam) <= 1e-9 * np.linalg.norm(G)
        for s in range(4):
            Z = W.random_matrix(17, X.shape, salt=s)
            Y = Z - X @ (X.T @ Z)
            assert float(np.sum(Y * op.hess_vec(X, Y)) - np.trace(Lam @ (Y.T @ Y))) > 0
    assert abs(runs[1].f - fr) <= 1e-9 * abs(fr) and abs(runs[2].f - fr) <= 1e-9 * abs(fr)


# ------------------------------------------------------------ dual ascent --
def test_dual_ascent_multiplier_step_and_convergence():
    """PCAL-DA (Section 5.3): the step is the gradient of L_beta(., Lambda^k) at
    X^k (eq. (Lag), checked by differences of L_beta), Lambda^0 is the closed
    form at X^0, and the iteration reaches the Ky Fan optimum of a quadratic
    (more slowly than PCAL, the point of Fig. 4)."""
    prob, x0 = W.quad_tridiag(n=300, p=8)
    op = OracleProblem(prob)
    beta = 1.0
    ks = [0, 3, 8]
    opt = O.Options(variant="pcal", mult="dual", beta=beta, eta0=beta + prob.s_bound,
                    tol=0.0, max_iter=10, record_history=True, record_iterates=ks)
    res = O.solve(op, x0, opt)
    for k in ks:
        X, gL, Lam = res.iterates[k], res.grads[k], res.mults[k]
        C = X.T @ X - np.eye(8)

        def Lb(Y):
            Cy = Y.T @ Y - np.eye(8)
            return op.f(Y) - 0.5 * float(np.sum(Lam * Cy)) + 0.25 * beta * float(np.sum(Cy * Cy))
        xi = W.random_matrix(16, X.shape, salt=k)
        fd = (4.0 * (Lb(X + 5e-5 * xi) - Lb(X - 5e-5 * xi)) / 1e-4
              - (Lb(X + 1e-4 * xi) - Lb(X - 1e-4 * xi)) / 2e-4) / 3.0
        assert abs(float(np.sum(gL * xi)) - fd) <= 1e-9 * abs(fd), k
        assert np.allclose(Lam, Lam.T, atol=1e-13)
    G0 = op.grad(x0)
    assert np.allclose(res.mults[0], O.Psi(G0.T @ x0), atol=1e-14)
    fstar = 0.5 * np.sum(np.linalg.eigvalsh(op.H0.toarray())[:8])
    full = O.solve(op, x0, O.Options(variant="pcal", mult="dual", beta=beta,
                                     eta0=beta + prob.s_bound, tol=1e-9, max_iter=40000))
    ref = O.solve(op, x0, O.Options(variant="pcal", beta=beta, eta0=beta + prob.s_bound,
                                    tol=1e-9, max_iter=40000))
    assert full.status == 0 and ref.status == 0
    assert abs(full.f - fstar) <= 1e-9 * fstar
    assert full.iters > ref.iters


# ---------------------------------------------------------------- MOptQR --
def test_moptqr_retraction_is_qr_and_iterates_feasible():
    """MOptQR (Table 1): D = grad f - X grad f^T X is a tangent vector at a
    feasible X (X^T D antisymmetric), every iterate is orthonormal, and
    X^{k+1} is the Q factor with positive diagonal R of V = X^k - D/eta^k
    (numpy's Householder QR)."""
    prob, x0, _ = W.ks3d(grid=(6, 5, 4), p=4)
    op = OracleProblem(prob)
    ks = [0, 1, 5]
    opt = O.Options(eta0=prob.s_bound, tol=0.0, max_iter=6, record_history=True,
                    record_iterates=ks + [k + 1 for k in ks], orth_final=False)
    res = O.moptqr(op, x0, opt)
    for k in ks:
        X, D, eta = res.iterates[k], res.grads[k], res.history["eta"][k]
        assert np.linalg.norm(X.T @ X - np.eye(4)) <= 1e-14 * 4
        XtD = X.T @ D
        assert np.linalg.norm(XtD + XtD.T) <= 1e-12 * np.linalg.norm(D)
        q, r = np.linalg.qr(X - D / eta)
        q = q * np.sign(np.diag(r))[None, :]
        assert np.max(np.abs(q - res.iterates[k + 1])) <= 1e-12, k
