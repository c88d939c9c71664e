"""Pins of the float64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a closed form, a
textbook routine on a special case, an invariant the paper states, brute force
on tiny inputs, or an independent solver.  A dropped term, a wrong sign or
factor, a transposed operand or an off-by-one in the step-size bookkeeping
fails at least one of them.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle.problems import (OracleProblem, laplacian_1d, laplacian_3d,
                             laplacian_eigenvalues_1d, laplacian_eigenvalues_3d)
from oracle import solver as O
from oracle import rgd


# ---------------------------------------------------------------- operators --
def test_laplacian_1d_spectrum_closed_form():
    """tridiag(-1,2,-1) has eigenvalues 4 sin^2(k pi / (2(n+1)))."""
    n = 37
    ev = np.linalg.eigvalsh(laplacian_1d(n).toarray())
    assert np.allclose(ev, np.sort(laplacian_eigenvalues_1d(n)), atol=1e-13)


def test_laplacian_3d_spectrum_and_stencil():
    grid = (5, 4, 3)
    L = laplacian_3d(grid).toarray()
    ev = np.linalg.eigvalsh(L)
    assert np.allclose(ev, np.sort(laplacian_eigenvalues_3d(grid).ravel()), atol=1e-12)
    assert np.allclose(np.diag(L), 6.0)
    # interior point (x=2, y=1, z=1) has exactly its 6 neighbours at -1
    nx, ny, _ = grid
    r = 2 + nx * (1 + ny * 1)
    nbrs = sorted([r - 1, r + 1, r - nx, r + nx, r - nx * ny, r + nx * ny])
    off = np.nonzero(L[r])[0].tolist()
    off.remove(r)
    assert off == nbrs and np.allclose(L[r, nbrs], -1.0)


def test_hartree_1d_green_function():
    """L^{-1} of tridiag(-1,2,-1) is min(i,j)(n+1-max(i,j))/(n+1) (1-based)."""
    n = 50
    prob, _ = W.ks1d(n=n, p=2)
    op = OracleProblem(prob)
    i = np.arange(1, n + 1)[:, None]
    j = np.arange(1, n + 1)[None, :]
    green = np.minimum(i, j) * (n + 1 - np.maximum(i, j)) / (n + 1)
    rho = W.random_uniform(1, n)
    assert np.allclose(op.hartree(rho), green @ rho, rtol=1e-13, atol=0)


def test_hartree_1d_large_n_extended_precision():
    """At n = 20000 (condition number ~ 1.6e8) the refined solve stays at the
    unit-roundoff level of an extended-precision Green's-function evaluation."""
    from tests.helpers import green_1d_extended
    n = 20000
    prob, _ = W.ks1d(n=n, p=2)
    rho = W.random_uniform(2, n)
    phi = OracleProblem(prob).hartree(rho)
    ex = green_1d_extended(rho)
    assert np.linalg.norm(phi - ex) <= 1e-15 * np.linalg.norm(ex)


def test_hartree_3d_residual_and_sine_mode():
    grid = (9, 7, 6)
    prob, _, _ = W.ks3d(grid=grid, p=2)
    op = OracleProblem(prob)
    rho = W.random_uniform(2, prob.n)
    phi = op.hartree(rho)
    assert np.linalg.norm(op.L @ phi - rho) <= 1e-12 * np.linalg.norm(rho)
    # a single sine mode is an eigenvector: L^{-1} s = s / lambda_abc
    nx, ny, nz = grid
    a, b, c = 2, 3, 1
    sx = np.sin(np.pi * a * np.arange(1, nx + 1) / (nx + 1))
    sy = np.sin(np.pi * b * np.arange(1, ny + 1) / (ny + 1))
    sz = np.sin(np.pi * c * np.arange(1, nz + 1) / (nz + 1))
    mode = (sz[:, None, None] * sy[None, :, None] * sx[None, None, :]).ravel()
    lam = 4 * (np.sin(a * np.pi / (2 * (nx + 1))) ** 2 + np.sin(b * np.pi / (2 * (ny + 1))) ** 2
               + np.sin(c * np.pi / (2 * (nz + 1))) ** 2)
    assert np.allclose(op.hartree(mode), mode / lam, atol=1e-13)


# ------------------------------------------------------------ f and grad f --
def _central_fd(op, X, E, h=1e-5):
    return (op.f(X + h * E) - op.f(X - h * E)) / (2 * h)


@pytest.mark.parametrize("which", ["quad", "ks1d", "ks1d_v", "ks3d", "dense"])
def test_gradient_matches_finite_differences(which):
    if which == "quad":
        prob, x0 = W.quad_tridiag(n=40, p=3)
    elif which == "ks1d":
        prob, x0 = W.ks1d(n=30, p=4, alpha=1.3)
    elif which == "ks1d_v":
        prob, x0 = W.ks1d(n=30, p=4, alpha=0.7, with_potential=True)
    elif which == "ks3d":
        prob, x0, _ = W.ks3d(grid=(4, 3, 5), p=3, alpha=1.0)
    else:
        prob, x0 = W.dense_quadratic(n=24, p=3, dtype=np.float64, power_iters=3)
    op = OracleProblem(prob)
    X = x0 + 0.1 * W.random_matrix(3, x0.shape)
    G = op.grad(X)
    for s in range(3):
        E = W.random_matrix(4, x0.shape, salt=s)
        fd = _central_fd(op, X, E)
        assert abs(fd - np.sum(G * E)) <= 1e-7 * max(1.0, abs(fd))


def test_hartree_energy_closed_form_on_unit_vectors():
    """X = [e_i, e_j]: rho is the indicator of {i, j}, so
    f = 1/2 (T_ii + T_jj) + alpha/4 (g_ii + 2 g_ij + g_jj) with the Green's function g."""
    n, alpha = 25, 1.7
    prob, _ = W.ks1d(n=n, p=2, alpha=alpha)
    op = OracleProblem(prob)
    i, j = 4, 17  # 0-based
    X = np.zeros((n, 2))
    X[i, 0] = 1.0
    X[j, 1] = 1.0
    g = lambda a, b: min(a + 1, b + 1) * (n + 1 - max(a + 1, b + 1)) / (n + 1)
    expect = 0.5 * (2 + 2) + alpha / 4 * (g(i, i) + 2 * g(i, j) + g(j, j))
    assert abs(op.f(X) - expect) <= 1e-12 * expect


def test_hessian_vector_matches_finite_differences():
    prob, x0, _ = W.ks3d(grid=(4, 4, 3), p=3, alpha=1.0)
    op = OracleProblem(prob)
    X = x0 + 0.05 * W.random_matrix(5, x0.shape)
    xi = W.random_matrix(6, x0.shape)
    h = 1e-6
    fd = (op.grad(X + h * xi) - op.grad(X - h * xi)) / (2 * h)
    assert np.linalg.norm(op.hess_vec(X, xi) - fd) <= 1e-7 * np.linalg.norm(fd)


# ------------------------------------------------------------ CholeskyQR2 --
def test_cholqr2_equals_householder_qr_up_to_signs():
    X = W.random_matrix(8, (300, 17)) + 0.3
    Q = O.cholqr2(X)
    q, r = np.linalg.qr(X)
    q = q * np.sign(np.diag(r))[None, :]
    assert np.linalg.norm(Q.T @ Q - np.eye(17)) <= 1e-14 * 17
    assert np.max(np.abs(Q - q)) <= 1e-12
    R = Q.T @ X
    assert np.allclose(np.tril(R, -1), 0.0, atol=1e-12)
    assert np.allclose(Q @ R, X, atol=1e-12)


def test_cholqr2_second_pass_on_ill_conditioned_input():
    """CholeskyQR loses orthogonality as kappa(X)^2 u; the second pass restores
    it to the unit roundoff (Fukaya et al.; the post-process of Section 5.3).
    At kappa = 3e6 one pass leaves ||Q^T Q - I|| ~ 1e-4, two leave ~1e-15."""
    n, p = 400, 20
    U, _ = np.linalg.qr(W.random_matrix(12, (n, p)))
    V, _ = np.linalg.qr(W.random_matrix(13, (p, p)))
    sig = np.logspace(0.0, -6.5, p)
    X = (U * sig[None, :]) @ V.T
    Q = O.cholqr2(X)
    assert np.linalg.norm(Q.T @ Q - np.eye(p)) <= 1e-14 * p
    # Q spans range(X) and X = Q R with R upper triangular
    R = Q.T @ X
    assert np.linalg.norm(np.tril(R, -1)) <= 1e-12 * np.linalg.norm(R)
    assert np.linalg.norm(Q @ R - X) <= 1e-13 * np.linalg.norm(X)
    # the test discriminates: a single CholeskyQR pass misses the bound by far
    c = np.linalg.cholesky(X.T @ X)
    Q1 = np.linalg.solve(c, X.T).T
    assert np.linalg.norm(Q1.T @ Q1 - np.eye(p)) >= 1e-8


# ------------------------------------------------------------- iteration --
def _aug_lagrangian(op, X, Lam, beta):
    """L_beta(X, Lam) = f(X) - 1/2 <Lam, X^T X - I> + beta/4 ||X^T X - I||_F^2, eq. (Lag)."""
    C = X.T @ X - np.eye(X.shape[1])
    return op.f(X) - 0.5 * float(np.sum(Lam * C)) + 0.25 * beta * float(np.sum(C * C))


@pytest.mark.parametrize("mult", ["psi_phi", "psi"])
def test_pcal_step_is_gradient_of_lagrangian_and_tangent(mult):
    """The step PCAL takes (Alg. 3, closed form after (PLLagSph)):

    * gradL^k is the Euclidean gradient of L_beta(., Lam^k) at X^k, eq. (Lag),
      checked by central differences of L_beta itself (pins the sign of X Lam,
      the factor of the beta term);
    * with the Phi-corrected multiplier eq. (lambda2) and unit columns,
      X_i^T gradL_i = 0 for every column i (the correction removes exactly the
      radial part; a dropped, sign-flipped or wrongly built correction leaves
      it nonzero), while eq. (Lambda1) leaves it nonzero;
    * X^{k+1}_i = (X^k_i - gradL^k_i/eta^k) / ||.||, so under eq. (lambda2)
      the normalizer is sqrt(1 + ||gradL_i||^2 / eta^2);
    * the iterates keep unit columns.
    """
    prob, x0 = W.ks1d(n=160, p=6, alpha=1.0, config=2, with_potential=True)
    op = OracleProblem(prob)
    beta = 30.0
    ks = [0, 1, 4, 9]
    opt = O.Options(variant="pcal", mult=mult, beta=beta, eta0=beta + prob.s_bound, tol=0.0,
                    max_iter=10, record_history=True, record_iterates=ks + [k + 1 for k in ks])
    res = O.solve(op, x0, opt)
    for k in ks:
        X, gL, Lam, eta = res.iterates[k], res.grads[k], res.mults[k], res.history["eta"][k]
        assert np.allclose(np.linalg.norm(X, axis=0), 1.0, atol=1e-14)
        xi = W.random_matrix(11, X.shape, salt=k)

        def cd(h):
            return (_aug_lagrangian(op, X + h * xi, Lam, beta)
                    - _aug_lagrangian(op, X - h * xi, Lam, beta)) / (2 * h)
        fd = (4.0 * cd(5e-5) - cd(1e-4)) / 3.0      # Richardson: O(h^4) error
        assert abs(float(np.sum(gL * xi)) - fd) <= 1e-9 * abs(fd), (k, mult)
        radial = np.abs(np.einsum("ij,ij->j", X, gL))
        if mult == "psi_phi":
            assert radial.max() <= 1e-13 * np.linalg.norm(gL), k
            nrm = np.sqrt(1.0 + np.sum(gL * gL, axis=0) / eta ** 2)
        else:
            # at the orthonormal X^0 both multipliers coincide (W symmetric, S = I)
            assert k == 0 or radial.max() >= 1e-6 * np.linalg.norm(gL), k
            nrm = np.linalg.norm(X - gL / eta, axis=0)
        Xn = (X - gL / eta) / nrm[None, :]
        assert np.max(np.abs(Xn - res.iterates[k + 1])) <= 1e-13, k


def test_ky_fan_quadratic_small():
    """min 1/2 tr(X^T A X) over the Stiefel manifold = 1/2 (sum of the p smallest eigenvalues)."""
    prob, x0 = W.quad_tridiag(n=300, p=8)
    op = OracleProblem(prob)
    fstar = 0.5 * np.sum(np.linalg.eigvalsh(op.H0.toarray())[:8])
    for variant, beta, mult in [("pcal", 1.0, "psi_phi"), ("pcal", 1.0, "psi"),
                                ("plam", prob.s_bound + 0.1, "psi")]:
        res = O.solve(op, x0, O.Options(variant=variant, beta=beta, mult=mult,
                                        eta0=beta + prob.s_bound, tol=1e-10, max_iter=5000))
        assert res.status == 0, variant
        assert abs(res.f - fstar) <= 1e-9 * abs(fstar), variant
        assert res.feas <= 1e-14 * 8


def test_ky_fan_laplacian_closed_form():
    """alpha = 0, v = 0: the optimum is half the sum of the p smallest 4 sin^2(k pi/(2(n+1)))."""
    prob, x0 = W.ks1d(n=120, p=5, alpha=0.0)
    op = OracleProblem(prob)
    fstar = 0.5 * np.sum(laplacian_eigenvalues_1d(120)[:5])
    res = O.solve(op, x0, O.Options(variant="pcal", beta=1.0, eta0=5.0, tol=1e-11,
                                    max_iter=20000))
    assert res.status == 0
    assert abs(res.f - fstar) <= 1e-9 * fstar


def test_multiplier_symmetric_and_stationary_at_convergence():
    """At a stationary point Lambda = grad f^T X is symmetric (eq. (closed-multi))."""
    prob, x0, _ = W.ks3d(grid=(6, 5, 5), p=5)
    op = OracleProblem(prob)
    res = O.solve(op, x0, O.Options(variant="pcal", beta=4.0, eta0=4.0 + prob.s_bound,
                                    tol=1e-10, max_iter=5000))
    assert res.status == 0
    G = op.grad(res.Q)
    XtG = res.Q.T @ G
    assert np.linalg.norm(XtG - res.Lam) <= 1e-8 * np.linalg.norm(res.Lam)
    assert np.linalg.norm(XtG - XtG.T) <= 1e-8 * np.linalg.norm(XtG)


def test_ks_plam_pcal_and_independent_solver_agree():
    """Table 2 pattern: PLAM and PCAL reach the same objective after the
    orthonormalization; a feasible Riemannian solver reaches it too."""
    prob, x0 = W.ks1d(n=400, p=6, alpha=1.0)
    op = OracleProblem(prob)
    r1 = O.solve(op, x0, O.Options(variant="pcal", beta=100.0, eta0=104.0, tol=1e-10,
                                   max_iter=20000))
    r2 = O.solve(op, x0, O.Options(variant="plam", mult="psi", beta=2000.0, eta0=2004.0,
                                   tol=1e-10, max_iter=20000))
    Xr, fr, kr, _ = rgd.solve(op, x0, tol=1e-10)
    assert r1.status == 0 and r2.status == 0
    assert abs(r1.f - r2.f) <= 1e-10 * abs(r1.f)
    assert abs(r1.f - fr) <= 1e-9 * abs(r1.f)
    # the orthonormalization changes the KKT measure only slightly (Table 2)
    assert r1.feas <= 1e-14 * 6


def test_second_order_condition_at_ks_minimizer():
    """(son): tr(Y^T Hess f[Y] - Lam Y^T Y) >= 0 on the tangent space."""
    prob, x0, _ = W.ks3d(grid=(6, 5, 4), p=4)
    op = OracleProblem(prob)
    res = O.solve(op, x0, O.Options(variant="pcal", beta=4.0, eta0=4.0 + prob.s_bound,
                                    tol=1e-10, max_iter=5000))
    X, Lam = res.Q, res.Lam
    for s in range(5):
        Z = W.random_matrix(9, X.shape, salt=s)
        Y = Z - X @ (X.T @ Z)                     # horizontal tangent vector
        q = float(np.sum(Y * op.hess_vec(X, Y)) - np.trace(Lam @ (Y.T @ Y)))
        assert q > 0


def test_merit_function_decreases_for_constant_large_eta():
    """Lemma 5 (sufficient decrease of h) with a constant, large eta."""
    prob, x0 = W.quad_tridiag(n=150, p=4)
    op = OracleProblem(prob)
    beta = prob.s_bound + 0.1
    X0 = x0 * 0.98                                # infeasible start with sigma_min > 0
    opt = O.Options(variant="plam", mult="psi", beta=beta, eta_rule="const",
                    eta_const=20.0 * (beta + prob.s_bound), eta0=1.0, tol=0.0, max_iter=60,
                    record_iterates=list(range(61)))
    res = O.solve(op, X0, opt)
    h = [O.merit(op, res.iterates[k], beta) for k in range(61)]
    assert all(h[k + 1] <= h[k] + 1e-13 for k in range(60))
    assert h[-1] < h[0]


def test_bb_indexing_standard_and_lagged():
    """The recorded eta^k is the BB quotient of the pair the option names."""
    prob, x0 = W.quad_tridiag(n=120, p=4)
    op = OracleProblem(prob)
    K = 12
    for bb in ["standard", "lagged"]:
        for rule in ["bb1", "bb2", "abb", "diff"]:
            opt = O.Options(variant="plam", mult="psi", beta=prob.s_bound + 0.1,
                            eta_rule=rule, bb_index=bb, eta0=9.0, tol=0.0, max_iter=K,
                            record_history=True, record_iterates=list(range(K + 1)))
            res = O.solve(op, x0, opt)
            Xs = res.iterates
            # PLAM: gradL^k = eta^k (X^k - X^{k+1}); lagged BB1 may blow up early,
            # then the recorded iterations are checked
            eta = res.history["eta"]
            Ke = min(len(eta), max(Xs) )
            assert Ke >= 4
            gL = {k: eta[k] * (Xs[k] - Xs[k + 1]) for k in range(Ke)}
            for k in range(2, Ke):
                if bb == "standard" or rule == "diff":
                    # eta_D is printed with the newest pair (Section 5.1)
                    Sd, Yd = Xs[k] - Xs[k - 1], gL[k] - gL[k - 1]
                else:
                    Sd, Yd = Xs[k - 1] - Xs[k - 2], gL[k - 1] - gL[k - 2]
                ss, sy, yy = np.sum(Sd * Sd), np.sum(Sd * Yd), np.sum(Yd * Yd)
                if rule == "bb1" or (rule == "abb" and k % 2 == 1):
                    q = abs(sy) / ss
                elif rule == "diff":
                    q = np.sqrt(yy / ss)
                else:
                    q = yy / abs(sy)
                assert abs(eta[k] - q) <= 1e-6 * q, (bb, rule, k)


def test_orthonormalization_post_process_table2_pattern():
    """Table 2: the post-process keeps the KKT violation and fixes feasibility."""
    prob, x0 = W.ks1d(n=500, p=6, alpha=1.0)
    op = OracleProblem(prob)
    res = O.solve(op, x0, O.Options(variant="pcal", beta=100.0, eta0=104.0, tol=1e-5,
                                    max_iter=5000, orth_final=False))
    kkt_stop = res.kkt_abs
    Q = O.cholqr2(res.X)
    kkt_orth = O.kkt_residual(op, Q)
    assert O.feasibility(Q) <= 1e-14 * 6
    assert O.feasibility(res.X) > O.feasibility(Q)
    assert abs(kkt_orth - kkt_stop) <= 0.05 * kkt_stop


# ---------------------------------------------------------- failure paths --
def test_failure_paths():
    with pytest.raises(ValueError):
        W.Problem(name="bad", kind="stencil1d", n=10, p=6)
    prob, x0 = W.quad_tridiag(n=2000, p=20)
    op = OracleProblem(prob)
    # PLAM with beta = 1 < s on config 1 diverges (Section 5.3 warns small beta may diverge)
    r = O.solve(op, x0, O.Options(variant="plam", mult="psi", beta=1.0, eta0=1.0 + prob.s_bound,
                                  tol=0.0, max_iter=500))
    assert r.status == O.STATUS_DIVERGED
    bad = x0.copy()
    bad[3, 2] = np.nan
    r = O.solve(op, bad, O.Options(max_iter=5))
    assert r.status == O.STATUS_DIVERGED
    r = O.solve(op, x0, O.Options(beta=1.0, eta0=6.0, tol=1e-14, max_iter=3, orth_final=False))
    assert r.status == O.STATUS_MAX_ITER and r.iters == 3
