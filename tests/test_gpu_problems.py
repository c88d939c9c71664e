"""GPU parity of the further test problems, multiplier rules and the MOptQR
comparator against the float64 oracle (through the C ABI):

* Problem 2 (linear term tr(G^T X)), Problem 4 (right factor B), Problem 6
  (exchange term) and the block-diagonal operator of the parallel experiments
  of Section 5.5: gradient and (f, KKT, feasibility) at 1e-13, iterates after
  k steps at 1e-10 (relative Frobenius and elementwise) for PLAM and PCAL;
  X^T G is not symmetric for Problems 2 and 4, so these runs take the whole
  Gram W;
* PLAM-DA / PCAL-DA (dual-ascent multiplier, Section 5.3): iterates at 1e-10;
* MOptQR with the Cholesky-QR retraction (Table 1, Section 5.5): iterates at
  1e-10 and the converged objective;
* the blocked Cholesky of CholeskyQR2 at ragged and wide p, and an iteration
  with p above 1024.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.problems import OracleProblem
from oracle import solver as O
from paper_1810_03930_amd import stiefel as S
from tests.helpers import maxrel, rel, to_dev, to_np

pytestmark = pytest.mark.gpu


def _prob(which):
    if which == "exchange":
        return W.ks_exchange(n=3000, p=40, block=5)
    if which == "exchange_small":
        return W.ks_exchange(n=150, p=6, block=5)
    if which == "block":
        return W.ks1d_block(n=2000, p=70, block=5)
    if which == "ocqp_tridiag":
        return W.ocqp_tridiag(n=2000, p=30)
    if which == "ocqp_wide":
        return W.ocqp_tridiag(n=1200, p=130)
    if which == "ocqp_dense":
        return W.ocqp_dense(n=600, p=20)
    if which == "qap":
        return W.qap_dense(n=500, p=12)
    if which == "quad":
        return W.quad_tridiag(n=800, p=16)
    if which == "quad_small":
        return W.quad_tridiag(n=300, p=8)
    if which == "ks3d":
        prob, x0, _ = W.ks3d(grid=(12, 10, 9), p=10)
        return prob, x0
    raise ValueError(which)


def _beta(which, variant):
    prob, _ = _prob(which)
    b = prob.s_bound + 0.1
    if which in ("ocqp_tridiag", "ocqp_wide", "ocqp_dense"):
        return max(1.0, b) if variant == "pcal" else 2 * b
    if which in ("exchange", "exchange_small", "block"):
        # PLAM with a large beta takes a tiny first step and a huge BB step after
        # it (the oracle diverges from these starts for beta >= 50)
        return 20.0 if variant == "pcal" else 10.0
    if which == "ks3d":
        return 4.0
    return 1.0 if variant == "pcal" else b


def _run(prob, x0, variant, mult, beta, k, eta_rule="abb", tol=0.0, orth=False,
         check_every=16):
    eta0 = (beta if variant != "moptqr" else 0.0) + prob.s_bound
    o = O.Options(variant="pcal" if variant == "moptqr" else variant, mult=mult, beta=beta,
                  eta_rule=eta_rule, eta0=eta0, eta_const=2 * eta0, tol=tol, max_iter=k,
                  orth_final=orth, record_iterates=[k] if tol == 0.0 else [])
    op = OracleProblem(prob)
    ref = O.moptqr(op, x0, o) if variant == "moptqr" else O.solve(op, x0, o)
    g = S.SolveOptions(variant=variant, mult=mult, eta_rule=eta_rule, precision="fp64",
                       max_iter=k, orth_final=orth, check_every=check_every, beta=beta,
                       eta0=eta0, eta_const=2 * eta0, tol=tol)
    dp = S.DeviceProblem.from_host(prob)
    X = to_dev(x0, torch.float64)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        res, x64, lam = S.solve(dp, X, g, want_x64=True, want_lambda=True, stream=s)
    torch.cuda.synchronize()
    return ref, res, to_np(X), op, dp


@pytest.mark.parametrize("which", ["exchange", "block", "ocqp_tridiag", "ocqp_dense", "qap"])
def test_gradient_and_evaluation(which):
    prob, x0 = _prob(which)
    op = OracleProblem(prob)
    X = x0 + 0.02 * W.random_matrix(21, x0.shape)
    dp = S.DeviceProblem.from_host(prob)
    Xd = to_dev(X, torch.float64)
    G = to_np(S.gradient(dp, Xd))
    Gr = op.grad(X)
    assert rel(G, Gr) <= 1e-13 and maxrel(G, Gr) <= 1e-13, which
    f, kkt, feas = S.evaluate(dp, Xd)
    assert abs(f - op.f(X)) <= 1e-12 * abs(op.f(X)), which
    assert abs(kkt - O.kkt_residual(op, X)) <= 1e-12 * O.kkt_residual(op, X), which
    assert abs(feas - O.feasibility(X)) <= 1e-12 * max(O.feasibility(X), 1e-3), which


def test_block_hartree():
    prob, _ = W.ks1d_block(n=2003, p=4, block=5)
    op = OracleProblem(prob)
    rho = W.random_uniform(31, prob.n)
    dp = S.DeviceProblem.from_host(prob)
    phi = to_np(S.hartree(dp, to_dev(rho)))
    ref = op.hartree(rho)
    assert maxrel(phi, ref) <= 1e-14
    long_prob, _ = W.ks1d_block(n=5000, p=4, block=1200)   # one workgroup per block
    rho2 = W.random_uniform(32, 5000)
    phi2 = to_np(S.hartree(S.DeviceProblem.from_host(long_prob), to_dev(rho2)))
    assert maxrel(phi2, OracleProblem(long_prob).hartree(rho2)) <= 1e-13


@pytest.mark.parametrize("which", ["exchange", "block", "ocqp_tridiag", "ocqp_wide",
                                   "ocqp_dense", "qap"])
@pytest.mark.parametrize("variant", ["pcal", "plam"])
@pytest.mark.parametrize("k", [1, 5, 20])
def test_problem_iterates(which, variant, k):
    prob, x0 = _prob(which)
    mult = "psi_phi" if variant == "pcal" else "psi"
    ref, res, X, _, _ = _run(prob, x0, variant, mult, _beta(which, variant), k)
    assert ref.status == O.STATUS_MAX_ITER, (which, variant, ref.status)
    assert res["rc"] == 1 and res["iters"] == k
    assert rel(X, ref.iterates[k]) <= 1e-10 and maxrel(X, ref.iterates[k]) <= 1e-10


@pytest.mark.parametrize("which", ["quad", "ks3d", "ocqp_tridiag"])
@pytest.mark.parametrize("variant", ["pcal", "plam"])
@pytest.mark.parametrize("k", [1, 5, 20])
def test_dual_ascent_iterates(which, variant, k):
    """PLAM-DA / PCAL-DA: Step 3 is the dual ascent Lam^k = Lam^{k-1} - beta C."""
    prob, x0 = _prob(which)
    ref, res, X, _, _ = _run(prob, x0, variant, "dual", _beta(which, variant), k)
    assert ref.status == O.STATUS_MAX_ITER and res["iters"] == k
    assert rel(X, ref.iterates[k]) <= 1e-10 and maxrel(X, ref.iterates[k]) <= 1e-10


@pytest.mark.parametrize("which", ["quad", "ks3d", "ocqp_tridiag", "qap", "exchange",
                                   "ocqp_wide"])
@pytest.mark.parametrize("k", [1, 5, 20])
def test_moptqr_iterates(which, k):
    prob, x0 = _prob(which)
    ref, res, X, _, _ = _run(prob, x0, "moptqr", "psi", 0.0, k)
    assert ref.status == O.STATUS_MAX_ITER and res["iters"] == k
    assert rel(X, ref.iterates[k]) <= 1e-10 and maxrel(X, ref.iterates[k]) <= 1e-10
    assert np.linalg.norm(X.T @ X - np.eye(prob.p)) <= 1e-13 * prob.p


@pytest.mark.parametrize("which,variant,mult", [
    ("exchange_small", "pcal", "psi_phi"), ("ocqp_tridiag", "pcal", "psi_phi"),
    ("qap", "pcal", "psi_phi"), ("ocqp_tridiag", "moptqr", "psi"), ("quad_small", "pcal", "dual"),
    ("ocqp_dense", "plam", "psi")])
def test_converged_solves(which, variant, mult):
    """Runs to tol: the GPU's float64 report equals the oracle's evaluation of
    the returned point, and the objective the oracle's converged one (the
    converged objective does not depend on the chaotic trajectory)."""
    prob, x0 = _prob(which)
    tol = 1e-9
    beta = _beta(which, variant) if variant != "moptqr" else 0.0
    ref, res, X, op, dp = _run(prob, x0, variant, mult, beta, 40000, tol=tol, orth=True,
                               check_every=50)
    assert ref.status == 0 and res["rc"] in (0, 2), (which, variant, res)
    # the status contract: STF_OK exactly when the float64 check meets tol
    assert (res["rc"] == 0) == (res["kkt_rel"] <= tol)
    # the orthonormalization post-process moves the KKT value (Table 2 shows it
    # unchanged to two digits for its problem).  Dual ascent stops where the
    # closed-form stop test is met but its own multiplier is not yet the closed
    # form, at a less feasible point whose distance from the manifold depends
    # on where the chaotic trajectory ends (measured: 1e-9 oracle, 3e-8 GPU
    # after 7500 iterations), so it gets a looser bound
    slack = 100.0 if mult == "dual" else 1.1
    assert res["kkt_rel"] <= max(slack * tol, 3.0 * ref.kkt_rel), (res["kkt_rel"], ref.kkt_rel)
    f_own = op.f(X)
    assert abs(res["fval"] - f_own) <= 1e-9 * abs(f_own)
    assert abs(res["kkt_abs"] - O.kkt_residual(op, X)) <= 1e-8 * res["kkt_abs"] + 1e-14
    assert res["feas"] <= 1e-13 * prob.p
    assert abs(res["fval"] - ref.f) <= 1e-8 * abs(ref.f), (res["fval"], ref.f)


@pytest.mark.parametrize("n,p,cond", [(3000, 256, 1.0), (2000, 300, 1.0), (3000, 512, 1.0),
                                      (1500, 200, 1e6), (2100, 1030, 1.0)])
def test_cholqr2_blocked(n, p, cond):
    """CholeskyQR2 with the blocked Cholesky and triangular inverse (64 x 64
    blocks, ragged last block) against the oracle's, on well- and
    ill-conditioned inputs."""
    Z = W.random_matrix(41, (n, p))
    if cond != 1.0:
        q, _ = np.linalg.qr(Z)
        Z = q * np.logspace(0, -np.log10(cond), p)[None, :]
    prob = W.Problem(name="cq", kind="stencil1d", n=n, p=p, alpha=0.0)
    dp = S.DeviceProblem.from_host(prob)
    Q = to_np(S.cholqr2(dp, to_dev(Z)))
    ref = O.cholqr2(Z)
    assert rel(Q, ref) <= 1e-11 and maxrel(Q, ref) <= 1e-10
    assert np.linalg.norm(Q.T @ Q - np.eye(p)) <= 1e-14 * p


def test_wide_iterates_above_1024_columns():
    """p = 1100 (the parallel experiments of Section 5.5 go to p = 2500):
    PCAL iterates after 3 steps on Problem 2 with the tridiagonal A."""
    prob, x0 = W.ocqp_tridiag(n=2300, p=1100)
    ref, res, X, _, _ = _run(prob, x0, "pcal", "psi_phi", 4.1, 3)
    assert res["iters"] == 3
    assert rel(X, ref.iterates[3]) <= 1e-10 and maxrel(X, ref.iterates[3]) <= 1e-10
