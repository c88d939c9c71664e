"""GPU parity of the individual steps against the float64 oracle.

Each step of the iteration is called through the C ABI (via the ctypes
binding) on seeded inputs and compared element by element with the oracle.
Sizes span several tiles and end in a ragged tail (n, p not multiples of the
tile sizes 16 / 32 / 64 / 128).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.problems import OracleProblem
from oracle import solver as O
from paper_1810_03930_amd import stiefel as S
from tests.helpers import maxrel, rel, to_dev, to_np, green_1d_extended

pytestmark = pytest.mark.gpu

CASES_1D = [
    # n, p, alpha, with potential
    (130, 20, 0.0, True),
    (1000, 37, 1.0, False),
    (5003, 100, 1.0, True),
]
CASES_3D = [
    ((6, 7, 5), 9, 1.0),
    ((16, 16, 16), 70, 1.0),
    ((20, 18, 17), 130, 0.5),
    ((9, 7, 5), 64, 1.0),
]


@pytest.mark.parametrize("n,p,alpha,pot", CASES_1D)
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_gradient_1d(n, p, alpha, pot, dt):
    prob, x0 = W.ks1d(n=n, p=p, alpha=alpha, with_potential=pot)
    op = OracleProblem(prob)
    x = to_dev(x0, dt)
    g_ref = op.grad(to_np(x))
    dp = S.DeviceProblem.from_host(prob)
    g = S.gradient(dp, x)
    tol = 1e-13 if dt == torch.float64 else 2e-6
    assert rel(to_np(g), g_ref) <= tol
    assert maxrel(to_np(g), g_ref) <= (tol if dt == torch.float64 else 1e-5)


@pytest.mark.parametrize("grid,p,alpha", CASES_3D)
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_gradient_3d(grid, p, alpha, dt):
    prob, x0, _ = W.ks3d(grid=grid, p=p, alpha=alpha)
    op = OracleProblem(prob)
    x = to_dev(x0, dt)
    g_ref = op.grad(to_np(x))
    dp = S.DeviceProblem.from_host(prob)
    g = S.gradient(dp, x)
    tol = 1e-13 if dt == torch.float64 else 2e-6
    assert rel(to_np(g), g_ref) <= tol
    assert maxrel(to_np(g), g_ref) <= (tol if dt == torch.float64 else 1e-5)


def test_gradient_3d_grid_stride():
    """More 64-row runs than one launch of the line-walking gradient holds
    (65536 workgroups x 4 waves): its grid-stride loop, float32 G, alpha = 0."""
    prob, x0, _ = W.ks3d(grid=(256, 256, 260), p=4, alpha=0.0)
    op = OracleProblem(prob)
    x = to_dev(x0, torch.float32)
    g_ref = op.grad(to_np(x))
    dp = S.DeviceProblem.from_host(prob)
    g = S.gradient(dp, x)
    assert rel(to_np(g), g_ref) <= 2e-6


@pytest.mark.parametrize("n,p", [(300, 37), (520, 130), (257, 64)])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_gradient_dense(n, p, dt):
    prob, x0 = W.dense_quadratic(n=n, p=p, dtype=np.float32 if dt == torch.float32 else np.float64,
                                 power_iters=5)
    op = OracleProblem(prob)
    x = to_dev(x0, dt)
    g_ref = op.grad(to_np(x))
    dp = S.DeviceProblem.from_host(prob, A_dtype=dt)
    g = S.gradient(dp, x)
    tol = 1e-13 if dt == torch.float64 else 2e-6
    assert rel(to_np(g), g_ref) <= tol
    assert maxrel(to_np(g), g_ref) <= (tol if dt == torch.float64 else 1e-5)


@pytest.mark.parametrize("n,p", [(520, 130), (1000, 200), (2051, 77)])
def test_gradient_dense_float32_operator_float64_arithmetic(n, p):
    """A stored in float32, X and G in float64: the float64 product widens A
    exactly, so it matches the float64 product of the rounded A to 1e-13
    (ragged n and p, several 128 x 128 tiles and 16-deep K steps)."""
    prob, x0 = W.dense_quadratic(n=n, p=p, dtype=np.float32, power_iters=5)
    op = OracleProblem(prob)
    g_ref = op.grad(x0)
    dp = S.DeviceProblem.from_host(prob, A_dtype=torch.float32)
    g = to_np(S.gradient(dp, to_dev(x0, torch.float64)))
    assert rel(g, g_ref) <= 1e-13 and maxrel(g, g_ref) <= 1e-13


@pytest.mark.parametrize("kind,shape", [("stencil1d", 5003), ("stencil1d", 20000),
                                        ("stencil3d", (16, 16, 16)), ("stencil3d", (20, 18, 17)),
                                        ("stencil3d", (64, 64, 64))])
def test_hartree(kind, shape):
    if kind == "stencil1d":
        prob, _ = W.ks1d(n=shape, p=2)
    else:
        prob, _, _ = W.ks3d(grid=shape, p=2)
    op = OracleProblem(prob)
    rho = W.random_uniform(7, prob.n, 0.0, 1.0)
    phi_ref = op.hartree(rho)
    dp = S.DeviceProblem.from_host(prob)
    phi = to_np(S.hartree(dp, to_dev(rho)))
    if kind == "stencil1d":
        # both sides pinned to an extended-precision evaluation of the Green's function
        exact = green_1d_extended(rho)
        assert rel(phi, exact) <= 1e-13
        assert rel(phi_ref, exact) <= 1e-15
        assert rel(phi, phi_ref) <= 1e-13
    else:
        assert rel(phi, phi_ref) <= 1e-13


@pytest.mark.parametrize("n,p", [(130, 20), (1000, 37), (5003, 100), (4096, 256), (2600, 300)])
def test_gram_fp64(n, p):
    prob, _ = W.ks1d(n=n, p=p)
    X = W.random_matrix(11, (n, p))
    G = W.random_matrix(12, (n, p))
    dp = S.DeviceProblem.from_host(prob)
    Sg, Wg = S.gram(dp, to_dev(X), to_dev(G), "fp64")
    Sg, Wg = to_np(Sg), to_np(Wg)
    assert rel(Sg, X.T @ X) <= 1e-13 and maxrel(Sg, X.T @ X) <= 1e-13
    assert rel(Wg, X.T @ G) <= 1e-13 and maxrel(Wg, X.T @ G) <= 1e-13
    assert np.array_equal(Sg, Sg.T)


@pytest.mark.parametrize("n,p", [(1000, 37), (5003, 100), (4096, 256)])
def test_gram_fp32(n, p):
    prob, _ = W.ks1d(n=n, p=p)
    X = W.random_matrix(11, (n, p)).astype(np.float32)
    G = W.random_matrix(12, (n, p)).astype(np.float32)
    dp = S.DeviceProblem.from_host(prob)
    Sg, Wg = S.gram(dp, to_dev(X), to_dev(G), "fp32")
    Xd, Gd = X.astype(np.float64), G.astype(np.float64)
    assert rel(to_np(Sg), Xd.T @ Xd) <= 2e-6
    assert rel(to_np(Wg), Xd.T @ Gd) <= 2e-6


@pytest.mark.parametrize("n,p", [(1000, 37), (5003, 100), (4096, 256), (700, 20), (2600, 300),
                                 (9001, 129)])
def test_gram_mixed_split_bf16(n, p):
    """Split-bf16 Gram (three bf16 products, float32 tiles, float64 across tiles).
    Each product carries a relative error of order 2^-16 (x = hi + lo leaves
    2^-16 |x|; the lo*lo term is dropped), so for these N(0,1) matrices the
    Frobenius error is ~2^-16 sqrt(p/n) relative: checked at 1e-5."""
    prob, _ = W.ks1d(n=n, p=p)
    X = W.random_matrix(11, (n, p)).astype(np.float32)
    G = W.random_matrix(12, (n, p)).astype(np.float32)
    dp = S.DeviceProblem.from_host(prob)
    Sg, Wg = S.gram(dp, to_dev(X), to_dev(G), "mixed")
    Xd, Gd = X.astype(np.float64), G.astype(np.float64)
    errS, errW = rel(to_np(Sg), Xd.T @ Xd), rel(to_np(Wg), Xd.T @ Gd)
    print(f"mixed gram n={n} p={p}: rel err S {errS:.2e} W {errW:.2e}")
    assert errS <= 1e-5 and errW <= 1e-5
    assert np.array_equal(to_np(Sg), to_np(Sg).T)


@pytest.mark.parametrize("n,p", [(130, 20), (1000, 37), (5003, 100), (2600, 300)])
def test_cholqr2(n, p):
    prob, _ = W.ks1d(n=n, p=p)
    X = W.random_matrix(13, (n, p)) + 0.1
    dp = S.DeviceProblem.from_host(prob)
    Q = to_np(S.cholqr2(dp, to_dev(X)))
    Q_ref = O.cholqr2(X)
    assert np.max(np.abs(Q - Q_ref)) <= 1e-11
    assert np.linalg.norm(Q.T @ Q - np.eye(p)) <= 1e-13 * np.sqrt(p) * 10


@pytest.mark.parametrize("which", ["quad", "ks1d", "ks3d"])
def test_eval(which):
    if which == "quad":
        prob, x0 = W.quad_tridiag(n=700, p=13)
    elif which == "ks1d":
        prob, x0 = W.ks1d(n=900, p=21)
    else:
        prob, x0, _ = W.ks3d(grid=(10, 9, 8), p=11)
    op = OracleProblem(prob)
    X = x0 + 0.01 * W.random_matrix(14, x0.shape)
    dp = S.DeviceProblem.from_host(prob)
    f, kkt, feas = S.evaluate(dp, to_dev(X))
    assert abs(f - op.f(X)) <= 1e-12 * abs(op.f(X))
    assert abs(kkt - O.kkt_residual(op, X)) <= 1e-11 * O.kkt_residual(op, X)
    assert abs(feas - O.feasibility(X)) <= 1e-12 * O.feasibility(X)
