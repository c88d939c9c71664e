"""GPU parity of the whole PLAM / PCAL iteration against the float64 oracle.

* Iterates after k steps (k in {1, 5, 20, 50}) must match the oracle's to
  1e-10 relative in the FP64 form.
* Every eta rule, both BB indexings and both multiplier rules are covered.
* Long runs: the Barzilai-Borwein iteration is chaotic -- the oracle itself,
  started from X0 perturbed by 1e-15, drifts by 1e-7 after 150 iterations and
  ends 500 iterations with a 10x different KKT value -- so trajectories are
  compared only for the first 50 steps.  Runs to a tolerance are compared on
  the converged objective (1e-8 relative), on the oracle's float64
  re-evaluation of the GPU's returned point (KKT norm, feasibility, multiplier
  to 1e-8 relative) and on both reaching the tolerance.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.problems import OracleProblem
from oracle import solver as O
from paper_1810_03930_amd import stiefel as S
from tests.helpers import assert_converged, maxrel, rel, to_dev, to_np, projector_distance

pytestmark = pytest.mark.gpu


def _pair(prob, variant="pcal", beta=1.0, eta_rule="abb", bb_index="standard", mult=None,
          tol=0.0, max_iter=50, orth=False, eta_const=None, precision="fp64", kkt_every=1,
          use_graph=True, check_every=16):
    if mult is None:
        mult = "psi_phi" if variant == "pcal" else "psi"
    eta0 = beta + prob.s_bound
    gam = eta_const if eta_const is not None else 2.0 * eta0
    o = O.Options(variant=variant, beta=beta, eta_rule=eta_rule, eta0=eta0, eta_const=gam,
                  tol=tol, max_iter=max_iter, mult=mult, bb_index=bb_index, orth_final=orth)
    g = S.SolveOptions(variant=variant, mult=mult, eta_rule=eta_rule, bb_index=bb_index,
                       precision=precision, max_iter=max_iter, kkt_every=kkt_every,
                       orth_final=orth, check_every=check_every, use_graph=use_graph,
                       beta=beta, eta0=eta0, eta_const=gam, tol=tol)
    return o, g


def _gpu_solve(prob, x0, gopt, stream=None):
    dp = S.DeviceProblem.from_host(prob)
    X = to_dev(x0, S.storage_dtype(gopt.precision))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        res, x64, lam = S.solve(dp, X, gopt, want_x64=True, want_lambda=True, stream=s)
    torch.cuda.synchronize()
    return res, to_np(X), to_np(x64), to_np(lam)


def _problem(which):
    if which == "quad":
        return W.quad_tridiag()
    if which == "quad_small":
        return W.quad_tridiag(n=333, p=7)
    if which == "ks1d":
        return W.ks1d(n=1500, p=12)
    if which == "ks3d":
        prob, x0, _ = W.ks3d(grid=(12, 10, 9), p=10)
        return prob, x0
    raise ValueError(which)


BETA = {"quad": 1.0, "quad_small": 1.0, "ks1d": 100.0, "ks3d": 4.0}


@pytest.mark.parametrize("which", ["quad", "ks1d", "ks3d"])
@pytest.mark.parametrize("k", [1, 5, 20, 50])
def test_pcal_iterates(which, k):
    prob, x0 = _problem(which)
    o, g = _pair(prob, beta=BETA[which], max_iter=k)
    o.record_iterates = [k]
    ref = O.solve(OracleProblem(prob), x0, o)
    res, X, _, _ = _gpu_solve(prob, x0, g)
    assert res["rc"] == 1 and res["iters"] == k
    assert rel(X, ref.iterates[k]) <= 1e-10 and maxrel(X, ref.iterates[k]) <= 1e-10


@pytest.mark.parametrize("which", ["quad", "ks3d"])
@pytest.mark.parametrize("eta_rule", ["const", "diff", "bb1", "bb2", "abb"])
@pytest.mark.parametrize("bb_index", ["standard", "lagged"])
def test_eta_rules(which, eta_rule, bb_index):
    prob, x0 = _problem(which)
    k = 20
    o, g = _pair(prob, beta=BETA[which], eta_rule=eta_rule, bb_index=bb_index, max_iter=k)
    o.record_iterates = [k]
    ref = O.solve(OracleProblem(prob), x0, o)
    res, X, _, _ = _gpu_solve(prob, x0, g)
    assert res["iters"] == k
    assert rel(X, ref.iterates[k]) <= 1e-10 and maxrel(X, ref.iterates[k]) <= 1e-10


@pytest.mark.parametrize("variant,mult,beta", [("plam", "psi", None), ("pcal", "psi", None),
                                               ("plam", "psi", 100.0)])
@pytest.mark.parametrize("which", ["quad", "ks1d"])
def test_variants(variant, mult, beta, which):
    """PLAM (Algorithm 2) and PCAL with the plain multiplier; PLAM with a beta far
    below the Hartree curvature of the 1D problem diverges on both sides at the
    same iteration (Section 5.3 warns that PLAM with small beta may diverge)."""
    prob, x0 = _problem(which)
    if beta is None:
        beta = prob.s_bound + 0.1 if (variant == "plam" and which == "quad") else BETA[which]
        if variant == "plam" and which == "ks1d":
            beta = 2e4
    k = 20
    o, g = _pair(prob, variant=variant, mult=mult, beta=beta, max_iter=k)
    o.record_iterates = [k]
    ref = O.solve(OracleProblem(prob), x0, o)
    res, X, _, _ = _gpu_solve(prob, x0, g)
    assert res["rc"] == (1 if ref.status == O.STATUS_MAX_ITER else ref.status)
    assert res["iters"] == ref.iters
    if ref.status == O.STATUS_MAX_ITER:
        assert rel(X, ref.iterates[k]) <= 1e-10 and maxrel(X, ref.iterates[k]) <= 1e-10


def _check_returned_point(op, res, X64, lam):
    """The GPU's float64 report of its returned point equals the oracle's
    evaluation of that same point."""
    G = op.grad(X64)
    kkt = O.kkt_residual(op, X64, G)
    assert abs(res["kkt_abs"] - kkt) <= 1e-8 * kkt + 1e-14
    assert abs(res["fval"] - op.f(X64)) <= 1e-12 * abs(op.f(X64))
    # feasibility after CholeskyQR2 is rounding noise (~1e-15): compared absolutely
    p = X64.shape[1]
    assert abs(res["feas"] - O.feasibility(X64)) <= 1e-8 * O.feasibility(X64) + 1e-14 * p
    assert rel(lam, O.Psi(G.T @ X64)) <= 1e-12


@pytest.mark.parametrize("variant,beta", [("pcal", 1.0), ("plam", None)])
def test_quadratic_500_iterations_ky_fan(variant, beta):
    """Config 1: tridiag(-1,2,-1) + Diag(u), n = 2000, p = 20, 500 iterations;
    objective vs the oracle and vs the Ky Fan sum of the 20 smallest eigenvalues."""
    prob, x0 = W.quad_tridiag()
    op = OracleProblem(prob)
    if beta is None:
        beta = prob.s_bound + 0.1      # PLAM at beta = 1 < s diverges (oracle pin)
    o, g = _pair(prob, variant=variant, beta=beta, max_iter=500, orth=True)
    ref = O.solve(op, x0, o)
    res, X, X64, lam = _gpu_solve(prob, x0, g)
    assert res["rc"] == 1 and res["iters"] == 500
    assert res["feas"] <= 1e-13
    _check_returned_point(op, res, X64, lam)
    # 500 fixed iterations stop short of convergence (relative KKT ~1e-6), so
    # both sides sit ~1e-8 above the optimum at different points of chaotic
    # trajectories: f is compared with the Ky Fan value at that level
    fstar = 0.5 * np.linalg.eigvalsh(op.H0.toarray())[:prob.p].sum()
    print(f"{variant}: f-f* gpu {res['fval'] - fstar:.3e}, oracle {ref.f - fstar:.3e}, "
          f"kkt_rel gpu {res['kkt_rel']:.2e} oracle {ref.kkt_rel:.2e}")
    assert 0.0 <= res["fval"] - fstar <= 1e-7 * abs(fstar)
    assert 0.0 <= ref.f - fstar <= 1e-7 * abs(fstar)


@pytest.mark.parametrize("which", ["quad_small", "ks1d", "ks3d"])
def test_converged_parity(which):
    prob, x0 = _problem(which)
    op = OracleProblem(prob)
    o, g = _pair(prob, beta=BETA[which], max_iter=3000, tol=1e-7, orth=True)
    ref = O.solve(op, x0, o)
    res, X, X64, lam = _gpu_solve(prob, x0, g)
    assert ref.status == 0
    assert_converged(res["rc"], res["kkt_rel"], 1e-7)
    print(f"{which}: iterations to tol: gpu {res['iters']}, oracle {ref.iters}")
    assert ref.kkt_rel <= 1.01e-7
    assert abs(res["fval"] - ref.f) <= 1e-8 * abs(ref.f)
    assert res["feas"] <= 1e-13 * prob.p
    # the multiplier at the returned point is Psi(grad f^T X) (eq. (closed-multi))
    _check_returned_point(op, res, X64, lam)


@pytest.mark.parametrize("use_graph", [False, True])
def test_graph_and_checkpoints_agree(use_graph):
    prob, x0 = _problem("ks3d")
    _, g = _pair(prob, beta=4.0, max_iter=37, use_graph=use_graph, check_every=6)
    res, X, _, _ = _gpu_solve(prob, x0, g)
    _, g2 = _pair(prob, beta=4.0, max_iter=37, use_graph=False, check_every=1)
    res2, X2, _, _ = _gpu_solve(prob, x0, g2)
    assert res["iters"] == res2["iters"] == 37
    assert np.array_equal(X, X2)


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
@pytest.mark.parametrize("k", [1, 5, 50])
def test_reduced_precision_iterates(precision, k):
    """float32 storage forms vs the float64 oracle after k steps (error stated)."""
    prob, x0 = _problem("ks3d")
    o, g = _pair(prob, beta=4.0, max_iter=k, precision=precision)
    o.record_iterates = [k]
    ref = O.solve(OracleProblem(prob), x0, o)
    res, X, _, _ = _gpu_solve(prob, x0, g)
    err = rel(X, ref.iterates[k])
    print(f"{precision} form: relative iterate error after {k} steps = {err:.3e}")
    assert res["iters"] == k
    assert err <= 1e-5 * k


def test_fp32_form_error_stated():
    """FP32 storage / float32 MFMA form vs the float64 oracle after 50 steps."""
    prob, x0 = _problem("ks3d")
    o, g = _pair(prob, beta=4.0, max_iter=50, precision="fp32")
    o.record_iterates = [50]
    ref = O.solve(OracleProblem(prob), x0, o)
    res, X, _, _ = _gpu_solve(prob, x0, g)
    err = rel(X, ref.iterates[50])
    print(f"fp32 form: relative iterate error after 50 steps = {err:.3e}")
    assert err <= 1e-4


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_switch_at_start_is_the_fp64_form(precision):
    """switch_tol >= 1 hands over at k = 0: the solve is then the float64 form
    started from the float32-rounded X0, bit for bit, and so matches the oracle."""
    prob, x0 = _problem("ks3d")
    x0r = x0.astype(np.float32).astype(np.float64)
    o, g = _pair(prob, beta=4.0, max_iter=40, precision=precision)
    g.switch_tol = 2.0
    res, _, X64, _ = _gpu_solve(prob, x0r, g)
    _, g64 = _pair(prob, beta=4.0, max_iter=40)
    res64, _, X64b, _ = _gpu_solve(prob, x0r, g64)
    assert res["switch_iter"] == 0 and res64["switch_iter"] == -1
    assert res["iters"] == res64["iters"] == 40
    assert np.array_equal(X64, X64b)
    o.record_iterates = [40]
    ref = O.solve(OracleProblem(prob), x0r, o)
    assert rel(X64, ref.iterates[40]) <= 1e-10 and maxrel(X64, ref.iterates[40]) <= 1e-10


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_switch_reaches_fp64_tolerance(precision):
    """A reduced-precision solve handed over to float64 at 1e-4 reaches a
    tolerance below what float32 arithmetic can resolve, at the oracle's minimum."""
    prob, x0 = _problem("ks3d")
    op = OracleProblem(prob)
    o, g = _pair(prob, beta=4.0, max_iter=3000, tol=1e-9, orth=True, precision=precision)
    g.switch_tol = 1e-4
    ref = O.solve(op, x0, o)
    res, _, X64, lam = _gpu_solve(prob, x0, g)
    print(f"{precision}: switched to float64 at k={res['switch_iter']}, "
          f"converged at {res['iters']} (oracle {ref.iters}), kkt_rel {res['kkt_rel']:.2e}")
    assert ref.status == 0
    assert_converged(res["rc"], res["kkt_rel"], 1e-9)
    assert 0 < res["switch_iter"] < res["iters"]
    assert abs(res["fval"] - ref.f) <= 1e-8 * abs(ref.f)
    _check_returned_point(op, res, X64, lam)


def test_switch_on_stall():
    """With a switch_tol it cannot reach, a MIXED solve hands over once its
    stop-test value has not improved for 100 iterations (its split-bf16 Grams
    put a floor far above 1e-10 under its own stop test), and the float64
    phase then reaches 1e-10.  (FP32 on this small grid drives its own stop
    test below 1e-10 -- it measures the float32-rounded G -- so it is not
    a stall case.)"""
    precision = "mixed"
    prob, x0 = _problem("ks3d")
    op = OracleProblem(prob)
    o, g = _pair(prob, beta=4.0, max_iter=6000, tol=1e-10, orth=True, precision=precision)
    g.switch_tol = 1e-30
    res, _, X64, lam = _gpu_solve(prob, x0, g)
    print(f"{precision}: hand-over on stall at k={res['switch_iter']}, converged at "
          f"{res['iters']}, kkt_rel {res['kkt_rel']:.2e}")
    assert_converged(res["rc"], res["kkt_rel"], 1e-10)
    assert 100 <= res["switch_iter"] < res["iters"]
    _check_returned_point(op, res, X64, lam)



@pytest.mark.parametrize("precision,fused", [("fp32", False), ("mixed", False),
                                             ("mixed32", False), ("mixed32", True)])
def test_stall_above_start_restarts_from_x0(precision, fused):
    """A reduced-precision descent that stalls at a stop-test value above the
    one at X^0 is discarded, and float64 restarts from X^0.  Constant steps
    50 times too long (eta = eta0 / 50) keep the stop test at least 1.5 times
    its X^0 value for 160 iterations in the float64 oracle, so the float32
    phase hands over on stall at k = 100 with restarted = 1, and the solve is
    then the float64 form from the float32-rounded X^0, bit for bit (in the
    two-pass and the single-pass forms)."""
    prob, x0, _ = W.ks3d(grid=(20, 18, 16), p=100)
    x0r = x0.astype(np.float32).astype(np.float64)
    m = 130
    eta0 = 4.0 + prob.s_bound
    _, g = _pair(prob, beta=4.0, eta_rule="const", eta_const=eta0 / 50, max_iter=m,
                 precision=precision)
    g.switch_tol = 1e-4
    g.fused = fused
    g.bb_index = "lagged" if fused else "standard"
    g.tol = 1e-14
    res, _, X64, _ = _gpu_solve(prob, x0r, g)
    _, g64 = _pair(prob, beta=4.0, eta_rule="const", eta_const=eta0 / 50, max_iter=m)
    g64.fused = fused
    g64.bb_index = g.bb_index
    g64.tol = 1e-14
    res64, X64b, _, _ = _gpu_solve(prob, x0r, g64)
    print(f"{precision} fused={fused}: hand-over at {res['switch_iter']}, "
          f"restarted {res['restarted']}, {res['iters']} float64 iterations")
    assert res["switch_iter"] == 100 and res["restarted"] == 1
    assert res["iters"] == res64["iters"] == m and res64["restarted"] == 0
    assert np.array_equal(X64, X64b)
    assert res["kkt_abs"] == res64["kkt_abs"] and res["kkt_abs"] > res["kkt0"]


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
@pytest.mark.parametrize("grid,p", [((20, 18, 16), 100), ((16, 16, 12), 300)])
def test_reduced_precision_iterates_wide(precision, grid, p):
    """Column blocks beyond one tile and ragged p (100: two 64-column blocks,
    the second partly empty; 300: K padded to 320) in the float32 forms."""
    prob, x0, _ = W.ks3d(grid=grid, p=p)
    k = 5
    o, g = _pair(prob, beta=4.0, max_iter=k, precision=precision)
    o.record_iterates = [k]
    ref = O.solve(OracleProblem(prob), x0, o)
    res, X, _, _ = _gpu_solve(prob, x0, g)
    err = rel(X, ref.iterates[k])
    print(f"{precision} form {grid} p={p}: relative iterate error after {k} steps = {err:.3e}")
    assert res["iters"] == k
    assert err <= 1e-5 * k


@pytest.mark.parametrize("grid,p", [((20, 18, 16), 100), ((16, 16, 12), 300), ((9, 8, 7), 37)])
@pytest.mark.parametrize("k", [1, 10])
def test_fp64_iterates_ragged_tiles(grid, p, k):
    """FP64 form with p off the tile grids: 64-column residual blocks (100:
    the second half empty; 300: five blocks, the last 44 wide; 37: one partly
    filled block), 128 x 128 Gram tiles with ragged edges, 16-deep K chunks
    with a short last chunk; iterates to 1e-10 of the oracle."""
    prob, x0, _ = W.ks3d(grid=grid, p=p)
    o, g = _pair(prob, beta=4.0, max_iter=k)
    o.record_iterates = [k]
    ref = O.solve(OracleProblem(prob), x0, o)
    res, X, _, _ = _gpu_solve(prob, x0, g)
    err = rel(X, ref.iterates[k])
    print(f"fp64 {grid} p={p}: relative iterate error after {k} steps = {err:.2e}")
    assert res["iters"] == k
    assert err <= 1e-10


def test_reduced_precision_status_contract():
    """An FP32 solve without hand-over whose in-loop stop test (float64 p x p
    identity over float32-rounded G and gradL) reaches tol is reported as
    converged only when the float64 check of the returned point agrees."""
    prob, x0 = _problem("ks3d")
    _, g = _pair(prob, beta=4.0, max_iter=3000, tol=1e-10, orth=True, precision="fp32")
    g.switch_tol = 0.0
    res, _, _, _ = _gpu_solve(prob, x0, g)
    print(f"fp32 without hand-over: rc {res['rc']}, kkt_rel {res['kkt_rel']:.2e}, "
          f"iters {res['iters']}")
    assert res["rc"] in (0, 1, 2)
    if res["rc"] == 0:
        assert res["kkt_rel"] <= 1e-10
    if res["rc"] == 2:
        assert res["kkt_rel"] > 1e-10
