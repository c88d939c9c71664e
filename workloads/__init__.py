"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module draws random numbers and lays them out; it holds none of the
method's arithmetic (no gradient, Gram, multiplier, step or
orthonormalization).  Both the CPU oracle and the GPU path consume exactly the
arrays produced here, so their results can be compared element by element.

Recipes follow the problems of Section 5.2 of the paper (Problem 1: the
simplified Kohn-Sham energy with a Hartree-like term; Problem 3: Rayleigh-Ritz
trace minimization) with the operators made explicit:

* ``stencil1d``: L = tridiag(-1, 2, -1) (1D Dirichlet Laplacian, unscaled),
  plus an optional diagonal potential ``v``;
* ``stencil3d``: L = the 7-point Dirichlet Laplacian on an (nx, ny, nz) grid
  (6 on the diagonal, -1 to each of the 6 neighbours), plus ``v``;
* ``dense``: a dense symmetric A = (B + B^T) / (2 sqrt(n)) + 4 I, B ~ N(0, 1).

The objective for every kind is
    f(X) = 1/2 tr(X^T (L + Diag v) X) + alpha/4 rho^T L^{-1} rho,
    rho = diag(X X^T),
with ``alpha = 0`` giving the quadratic problems (dense: L replaced by A).

Initial points are X0 = Q from the QR factorization of an n x p N(0,1)
matrix with diag(R) > 0, as in the experiments of Section 5.5.

Seeds: workload ``c`` (1..5) draws from ``numpy.random.default_rng(20181009 + c)``
in the fixed order operator data, then X0, then any auxiliary weights.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple, List

import numpy as np

SEED_BASE = 20181009

KIND_STENCIL1D = "stencil1d"
KIND_STENCIL3D = "stencil3d"
KIND_DENSE = "dense"


@dataclass
class Problem:
    """Description of one instance of min f(X) s.t. X^T X = I_p."""

    name: str
    kind: str
    n: int
    p: int
    alpha: float = 0.0
    v: Optional[np.ndarray] = None          # diagonal potential, float64, length n
    grid: Tuple[int, int, int] = (0, 1, 1)  # (nx, ny, nz), x fastest in the row index
    A: Optional[np.ndarray] = None          # dense operator (row-major n x n)
    s_bound: float = 0.0                    # upper bound of ||Hess f(0)||_2 (Section 5.1)
    meta: dict = field(default_factory=dict)
    block: int = 0                          # stencil1d: order of the tridiagonal blocks (0: one)
    gamma: float = 0.0                      # exchange weight of Problem 6
    Glin: Optional[np.ndarray] = None       # linear term of Problem 2, float64 n x p
    B: Optional[np.ndarray] = None          # right factor of Problem 4, float64 p x p

    def __post_init__(self):
        if self.kind == KIND_STENCIL1D and self.grid[0] == 0:
            self.grid = (self.n, 1, 1)
        if self.n < 2 * self.p:
            raise ValueError("the problem needs 2p <= n (Section 1)")


def rng_for(config: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + config)


def orthonormal_start(rng: np.random.Generator, n: int, p: int) -> np.ndarray:
    """X0 = Q of QR(N(0,1) n x p) with diag(R) > 0, float64, C-contiguous."""
    z = rng.standard_normal((n, p))
    q, r = np.linalg.qr(z)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return np.ascontiguousarray(q * s[None, :])


def quad_tridiag(n: int = 2000, p: int = 20, config: int = 1):
    """Quadratic f = 1/2 tr(X^T A X), A = tridiag(-1,2,-1) + Diag(u), u ~ U(0,1)."""
    rng = rng_for(config)
    u = rng.uniform(0.0, 1.0, n)
    x0 = orthonormal_start(rng, n, p)
    prob = Problem(name=f"quad_tridiag_n{n}_p{p}", kind=KIND_STENCIL1D, n=n, p=p,
                   alpha=0.0, v=u, grid=(n, 1, 1), s_bound=4.0 + float(u.max()))
    return prob, x0


def ks1d(n: int = 20000, p: int = 100, alpha: float = 1.0, config: int = 2,
         with_potential: bool = False):
    """1D Kohn-Sham-shaped f with the unscaled 1D Dirichlet Laplacian."""
    rng = rng_for(config)
    v = rng.uniform(0.0, 1.0, n) if with_potential else None
    x0 = orthonormal_start(rng, n, p)
    sb = 4.0 + (float(v.max()) if v is not None else 0.0)
    prob = Problem(name=f"ks1d_n{n}_p{p}", kind=KIND_STENCIL1D, n=n, p=p,
                   alpha=float(alpha), v=v, grid=(n, 1, 1), s_bound=sb)
    return prob, x0


def ks3d(grid=(64, 64, 64), p: int = 256, alpha: float = 1.0, config: int = 5):
    """3D Kohn-Sham-shaped f: 7-point Laplacian + Diag(V), V ~ U(0,1).

    Returns (problem, X0, w) where w ~ U(0,1) are the weights of the loss
    ||X^T Diag(w) X||_F^2 used by the adjoint.
    """
    rng = rng_for(config)
    nx, ny, nz = grid
    n = nx * ny * nz
    v = rng.uniform(0.0, 1.0, n)
    x0 = orthonormal_start(rng, n, p)
    w = rng.uniform(0.0, 1.0, n)
    prob = Problem(name=f"ks3d_{nx}x{ny}x{nz}_p{p}", kind=KIND_STENCIL3D, n=n, p=p,
                   alpha=float(alpha), v=v, grid=(nx, ny, nz),
                   s_bound=12.0 + float(v.max()))
    return prob, x0, w


def dense_quadratic(n: int = 32768, p: int = 512, config: int = 3,
                    dtype=np.float32, power_iters: int = 30):
    """Dense Rayleigh-Ritz instance A = (B + B^T)/(2 sqrt n) + 4 I, B ~ N(0,1).

    A is returned in ``dtype`` (float32 by default); the oracle and the GPU
    both consume exactly these values.  The returned ``s_bound`` is a power
    iteration estimate of ||A||_2 with a 5% margin (it only sets beta/eta0).
    """
    rng = rng_for(config)
    b = rng.standard_normal((n, n), dtype=np.float32)
    a = np.empty((n, n), dtype=dtype)
    scale = 1.0 / (2.0 * np.sqrt(n))
    blk = 2048
    for i0 in range(0, n, blk):
        i1 = min(n, i0 + blk)
        a[i0:i1, :] = ((b[i0:i1, :] + b[:, i0:i1].T) * scale).astype(dtype)
    del b
    a[np.arange(n), np.arange(n)] += dtype(4.0)
    x0 = orthonormal_start(rng, n, p)
    # spectral-norm estimate for the parameter rule (not part of the method)
    t = np.ones(n, dtype=np.float64) / np.sqrt(n)
    lam = 0.0
    for _ in range(power_iters):
        y = a @ t.astype(dtype)
        lam = float(np.linalg.norm(y))
        t = (y / lam).astype(np.float64)
    prob = Problem(name=f"dense_n{n}_p{p}", kind=KIND_DENSE, n=n, p=p, alpha=0.0,
                   A=a, grid=(n, 1, 1), s_bound=1.05 * lam)
    return prob, x0


def batched_ks1d(nprob: int = 256, config: int = 4, n_range=(1000, 20000),
                 p_range=(8, 128), alpha_range=(0.5, 2.0)):
    """Many independent 1D KS problems of uneven n and p.

    Operator data for all problems is drawn first (n, p, alpha per problem),
    then the X0 of each problem in order.
    """
    rng = rng_for(config)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=nprob)
    ps = rng.integers(p_range[0], p_range[1] + 1, size=nprob)
    alphas = rng.uniform(alpha_range[0], alpha_range[1], size=nprob)
    probs: List[Problem] = []
    x0s: List[np.ndarray] = []
    for b in range(nprob):
        n, p = int(ns[b]), int(ps[b])
        probs.append(Problem(name=f"batch{b}_n{n}_p{p}", kind=KIND_STENCIL1D, n=n, p=p,
                             alpha=float(alphas[b]), v=None, grid=(n, 1, 1),
                             s_bound=4.0))
    for b in range(nprob):
        x0s.append(orthonormal_start(rng, probs[b].n, probs[b].p))
    return probs, x0s


def ks1d_block(n: int = 10000, p: int = 1000, block: int = 5, alpha: float = 1.0,
               config: int = 6):
    """Problem 1 as in the parallel experiments of Section 5.5: L block-diagonal
    with tridiag(-1,2,-1) blocks of order 5, alpha = 1."""
    rng = rng_for(config)
    x0 = orthonormal_start(rng, n, p)
    prob = Problem(name=f"ks1d_block{block}_n{n}_p{p}", kind=KIND_STENCIL1D, n=n, p=p,
                   alpha=float(alpha), v=None, grid=(n, 1, 1), s_bound=4.0, block=int(block))
    return prob, x0


def ocqp_tridiag(n: int = 10000, p: int = 1000, config: int = 7):
    """Problem 2 as in Section 5.5: A = tridiag(-1, 2, -1), G = Random(n, p)
    (uniform on [-1, 1]), f = 1/2 tr(X^T A X) + tr(G^T X)."""
    rng = rng_for(config)
    g = rng.uniform(-1.0, 1.0, (n, p))
    x0 = orthonormal_start(rng, n, p)
    prob = Problem(name=f"ocqp_tridiag_n{n}_p{p}", kind=KIND_STENCIL1D, n=n, p=p, alpha=0.0,
                   v=None, grid=(n, 1, 1), s_bound=4.0, Glin=np.ascontiguousarray(g))
    return prob, x0


EXCHANGE_GAMMA = 2.0 * (3.0 / np.pi) ** (1.0 / 3.0)   # gamma of Problem 6


def ks_exchange(n: int = 10000, p: int = 1000, block: int = 5, config: int = 8):
    """Problem 6 as in Section 5.5: 1/2 tr(X^T L X) + 1/2 rho^T L^{-1} rho
    - 3/4 gamma rho^T rho^{1/3}, L as in ``ks1d_block`` (alpha = 2 in the
    alpha/4 convention of the other problems), gamma = 2 (3/pi)^{1/3}."""
    rng = rng_for(config)
    x0 = orthonormal_start(rng, n, p)
    prob = Problem(name=f"ks_exchange_block{block}_n{n}_p{p}", kind=KIND_STENCIL1D, n=n, p=p,
                   alpha=2.0, v=None, grid=(n, 1, 1), s_bound=4.0, block=int(block),
                   gamma=EXCHANGE_GAMMA)
    return prob, x0


def ocqp_dense(n: int = 1000, p: int = 20, config: int = 9, kappa: float = 1.0,
               theta: float = 1.01, zeta: float = 1.01, xi: float = 1.0):
    """Problem 2 of Section 5.2 with its generator: A = P Lambda P^T, P the Q
    factor of a U(0,1) n x n matrix, Lambda_ii = +-theta^{1-i} (+ with
    probability xi); G = kappa Q D, Q the columns of a U(0,1) n x p matrix
    scaled to unit norm, D_jj = zeta^{j-1}."""
    rng = rng_for(config)
    P, _ = np.linalg.qr(rng.uniform(0.0, 1.0, (n, n)))
    lam = theta ** (-np.arange(n, dtype=np.float64))
    lam = np.where(rng.uniform(0.0, 1.0, n) < xi, lam, -lam)
    A = (P * lam[None, :]) @ P.T
    A = 0.5 * (A + A.T)
    qt = rng.uniform(0.0, 1.0, (n, p))
    Q = qt / np.linalg.norm(qt, axis=0)[None, :]
    G = kappa * Q * (zeta ** np.arange(p, dtype=np.float64))[None, :]
    x0 = orthonormal_start(rng, n, p)
    prob = Problem(name=f"ocqp_dense_n{n}_p{p}", kind=KIND_DENSE, n=n, p=p, alpha=0.0,
                   A=np.ascontiguousarray(A), grid=(n, 1, 1),
                   s_bound=float(np.max(np.abs(lam))), Glin=np.ascontiguousarray(G))
    return prob, x0


def qap_dense(n: int = 1000, p: int = 20, config: int = 10):
    """Problem 4 of Section 5.2: f = 1/2 tr(A^T X B X^T), A = sym(randn(n)),
    B = sym(randn(p)); s = ||A||_2 ||B||_2."""
    rng = rng_for(config)
    a = rng.standard_normal((n, n))
    A = 0.5 * (a + a.T)
    b = rng.standard_normal((p, p))
    B = 0.5 * (b + b.T)
    x0 = orthonormal_start(rng, n, p)
    sa = float(np.max(np.abs(np.linalg.eigvalsh(A))))
    sb = float(np.max(np.abs(np.linalg.eigvalsh(B))))
    prob = Problem(name=f"qap_dense_n{n}_p{p}", kind=KIND_DENSE, n=n, p=p, alpha=0.0,
                   A=np.ascontiguousarray(A), grid=(n, 1, 1), s_bound=sa * sb,
                   B=np.ascontiguousarray(B))
    return prob, x0


def alternate_start(config: int, n: int, p: int, start: int) -> np.ndarray:
    """Another seeded X0 for the same operator (start >= 1; start 0 is the
    workload's own X0): the iteration count of the Barzilai-Borwein method
    varies with the start, so timings to a tolerance are also taken over a few."""
    rng = np.random.default_rng([SEED_BASE + config, 1000 + start])
    return orthonormal_start(rng, n, p)


def random_matrix(config: int, shape, salt: int = 0) -> np.ndarray:
    """A seeded N(0,1) matrix for unit tests of individual steps."""
    rng = np.random.default_rng([SEED_BASE + config, salt])
    return rng.standard_normal(shape)


def random_uniform(config: int, shape, lo=0.0, hi=1.0, salt: int = 0) -> np.ndarray:
    rng = np.random.default_rng([SEED_BASE + config, salt])
    return rng.uniform(lo, hi, shape)


# Named workloads with the sizes of the benchmark configurations.
FULL_SIZES = {
    1: dict(kind="quad_tridiag", n=2000, p=20),
    2: dict(kind="ks1d", n=20000, p=100),
    3: dict(kind="dense", n=32768, p=512),
    4: dict(kind="batched_ks1d", nprob=256),
    5: dict(kind="ks3d", grid=(64, 64, 64), p=256),
}

# The shapes of the parallel experiments of Section 5.5 (Figs. 7-11).
PARALLEL_SIZES = {
    "P1": dict(kind="ks1d_block", n=10000, ps=(500, 1000, 1500, 2000, 2500)),
    "P2": dict(kind="ocqp_tridiag", n=10000, ps=(500, 1000, 1500, 2000, 2500)),
    "P6": dict(kind="ks_exchange", n=10000, ps=(1000,)),
}
