"""Parity at the full 3D Kohn-Sham workload (64^3 grid, n = 262144, p = 256,
alpha = 1, beta = 4, ABB) in the launch configuration the benchmark times:
the same problem and options give the same plans (85 Gram chunks x 6 upper
tiles, 128 x 64 residual tiles over 256 row-block workgroups, four column-dot
groups, the 1024-thread Hartree passes).

* FP64: whole iterates after 1 and 3 steps against the float64 oracle, 1e-10
  relative (the oracle runs the same iterations on the host; about a second
  each on 16 cores).
* MIXED: iterates after 3 steps, 1e-5 * k as for the small grids.
* the Gram step at full size against the float64 product of the same inputs.
* the single-pass form (options.fused, lagged Barzilai-Borwein pair) in FP64
  and MIXED32 after 3 steps against the oracle run with the lagged pair, at
  the same bounds.
"""
import pytest
import torch

import workloads as W
from oracle.problems import OracleProblem
from oracle import solver as O
from paper_1810_03930_amd import stiefel as S
from tests.helpers import maxrel, rel, to_dev, to_np

pytestmark = pytest.mark.gpu

BETA = 4.0


@pytest.fixture(scope="module")
def c5():
    prob, x0, _ = W.ks3d(grid=(64, 64, 64), p=256, alpha=1.0)
    return prob, x0, OracleProblem(prob)


def _opts(prob, k, precision, fused=False):
    eta0 = BETA + prob.s_bound
    bb = "lagged" if fused else "standard"
    o = O.Options(variant="pcal", beta=BETA, eta_rule="abb", eta0=eta0, eta_const=2 * eta0,
                  tol=0.0, max_iter=k, mult="psi_phi", bb_index=bb, orth_final=False,
                  record_iterates=list(range(1, k + 1)))
    g = S.SolveOptions(variant="pcal", mult="psi_phi", eta_rule="abb", precision=precision,
                       beta=BETA, eta0=eta0, tol=0.0, max_iter=k, orth_final=False,
                       check_every=k, use_graph=True, bb_index=bb, fused=fused)
    return o, g


def _gpu(prob, x0, gopt):
    dp = S.DeviceProblem.from_host(prob)
    X = to_dev(x0, S.storage_dtype(gopt.precision))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        res, x64, _ = S.solve(dp, X, gopt, want_x64=True, stream=s)
    torch.cuda.synchronize()
    out = to_np(x64)
    del X, x64, dp
    torch.cuda.empty_cache()
    return res, out


@pytest.fixture(scope="module")
def oracle_iterates(c5):
    prob, x0, op = c5
    o, _ = _opts(prob, 3, "fp64")
    ref = O.solve(op, x0, o)
    return ref.iterates


@pytest.mark.parametrize("k", [1, 3])
def test_fullsize_fp64_iterates(c5, oracle_iterates, k):
    prob, x0, _ = c5
    _, g = _opts(prob, k, "fp64")
    res, X = _gpu(prob, x0, g)
    err = rel(X, oracle_iterates[k])
    emax = maxrel(X, oracle_iterates[k])
    print(f"64^3 p=256 FP64: relative iterate error after {k} steps = {err:.2e} "
          f"(elementwise {emax:.2e})")
    assert res["iters"] == k
    assert err <= 1e-10 and emax <= 1e-10


@pytest.mark.parametrize("precision", ["mixed", "mixed32"])
def test_fullsize_mixed_iterates(c5, oracle_iterates, precision):
    """The split-bf16 forms after 3 steps: the relative Frobenius error and the
    largest elementwise error, max|dX| / max|X| (a localized error such as one
    wrong boundary plane would show in the second, not the first)."""
    prob, x0, _ = c5
    k = 3
    _, g = _opts(prob, k, precision)
    res, X = _gpu(prob, x0, g)
    err = rel(X, oracle_iterates[k])
    emax = maxrel(X, oracle_iterates[k])
    print(f"64^3 p=256 {precision}: relative iterate error after {k} steps = {err:.2e} "
          f"(elementwise {emax:.2e})")
    assert res["iters"] == k
    assert err <= 1e-5 * k and emax <= 1e-5 * k


def test_fullsize_gram(c5):
    prob, x0, _ = c5
    G = W.random_matrix(13, x0.shape)
    dp = S.DeviceProblem.from_host(prob)
    Sg, Wg = S.gram(dp, to_dev(x0), to_dev(G), "fp64")
    errS = rel(to_np(Sg), x0.T @ x0)
    errW = rel(to_np(Wg), x0.T @ G)
    print(f"64^3 p=256 Gram: rel err S {errS:.2e} W {errW:.2e}")
    assert errS <= 1e-13 and errW <= 1e-13


@pytest.fixture(scope="module")
def oracle_iterates_lagged(c5):
    prob, x0, op = c5
    o, _ = _opts(prob, 3, "fp64", fused=True)
    return O.solve(op, x0, o).iterates


@pytest.mark.parametrize("precision", ["fp64", "mixed32"])
def test_fullsize_fused_iterates(c5, oracle_iterates_lagged, precision):
    prob, x0, _ = c5
    k = 3
    _, g = _opts(prob, k, precision, fused=True)
    res, X = _gpu(prob, x0, g)
    ref = oracle_iterates_lagged[k]
    err, emax = rel(X, ref), maxrel(X, ref)
    print(f"64^3 p=256 fused {precision}: relative iterate error after {k} steps = {err:.2e} "
          f"(elementwise {emax:.2e})")
    assert res["iters"] == k
    bound = 1e-10 if precision == "fp64" else 1e-5 * k
    assert err <= bound and emax <= bound
