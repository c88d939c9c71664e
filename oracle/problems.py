"""Objective, gradient, density and Hartree solve of the test problems (oracle).

Test infrastructure only (see the package docstring).

The problems are Problem 1 (simplified Kohn-Sham energy) and Problem 3
(Rayleigh-Ritz trace minimization) of Section 5.2, with the operators of the
synthetic workloads:

    f(X) = 1/2 tr(X^T H0 X) + alpha/4 rho(X)^T L^{-1} rho(X),
    rho(X) = diag(X X^T)            (the charge density of eq. (KS-energy)),
    H0 = L + Diag(v)  (stencil kinds)   or   H0 = A  (dense kind).

L is symmetric positive definite (Dirichlet boundary), so the pseudo-inverse
L^dagger of the paper is the inverse.  Differentiating,

    grad f(X) = H0 X + alpha * Diag(L^{-1} rho) X,

because d(rho_j)/dX_ji = 2 X_ji and L^{-1} is symmetric.

The Hartree solve phi = L^{-1} rho:

* 1D: a sparse LU factorization of the tridiagonal L (SuperLU via scipy),
  i.e. the plain definition, computed once per problem and reused, followed by
  one step of iterative refinement whose residual rho - L phi is formed in
  extended precision: L has condition number ~ n^2, so the bare LU solve
  carries ~10 n unit roundoffs of forward error, the refined one ~1;
* 3D: the exact eigen-decomposition of the Dirichlet 7-point Laplacian.
  Each 1D factor tridiag(-1,2,-1) of order m has the orthonormal sine
  eigenvectors sqrt(2/(m+1)) sin(j k pi/(m+1)) and eigenvalues
  4 sin^2(k pi / (2(m+1))), so L = S D S with S the tensor product of the
  orthonormal DST-I along each axis, and phi = S D^{-1} S rho.  The DST-I is
  taken from scipy.fft (a library primitive).  A sparse LU of the 3D
  operator is not used because its fill makes it take many minutes.

Further terms of the test problems of Section 5.2 (each absent when zero / None):

* a block-diagonal L = Diag(L_1, ..., L_s) of tridiag(-1,2,-1) blocks of order
  ``block`` (the last block may be shorter): the 1D operator of the parallel
  experiments of Section 5.5; its inverse is block-diagonal, each block the
  textbook Green's function of the block;
* the exchange term of Problem 6, -3/4 gamma rho^T rho^{1/3}, whose gradient is
  -2 gamma Diag(rho^{1/3}) X (d rho_j / d X_ji = 2 X_ji);
* the linear term tr(Glin^T X) of Problem 2, gradient Glin;
* the right factor B of Problem 4: f = 1/2 tr(A^T X B X^T) = 1/2 tr(X^T A X B)
  for symmetric A and B, gradient A X B.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def laplacian_1d(n: int, block: int = 0) -> sp.csr_matrix:
    """tridiag(-1, 2, -1) of order n (unscaled 1D Dirichlet Laplacian), or with
    ``block`` > 0 the block-diagonal matrix of such blocks of order ``block``
    (the last one shorter when block does not divide n)."""
    if block and block < n:
        sizes = [block] * (n // block) + ([n % block] if n % block else [])
        return sp.block_diag([laplacian_1d(m) for m in sizes], format="csr")
    e = np.ones(n)
    return sp.diags([-e[:-1], 2.0 * e, -e[:-1]], [-1, 0, 1], format="csr")


def laplacian_3d(grid) -> sp.csr_matrix:
    """7-point Dirichlet Laplacian on an (nx, ny, nz) grid, x fastest.

    Row index r = x + nx * (y + ny * z).  Built as a Kronecker sum of 1D
    operators, so it has 6 on the diagonal and -1 for each grid neighbour.
    """
    nx, ny, nz = grid
    ix, iy, iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    tx, ty, tz = laplacian_1d(nx), laplacian_1d(ny), laplacian_1d(nz)
    # x is the fastest index, so it is the last Kronecker factor
    lap = (sp.kron(sp.kron(iz, iy), tx) + sp.kron(sp.kron(iz, ty), ix)
           + sp.kron(sp.kron(tz, iy), ix))
    return lap.tocsr()


def laplacian_eigenvalues_1d(m: int) -> np.ndarray:
    """Eigenvalues 4 sin^2(k pi / (2(m+1))), k = 1..m, of tridiag(-1,2,-1)."""
    k = np.arange(1, m + 1, dtype=np.float64)
    return 4.0 * np.sin(k * np.pi / (2.0 * (m + 1))) ** 2


def laplacian_eigenvalues_3d(grid) -> np.ndarray:
    """Eigenvalues of the 3D operator as an (nz, ny, nx) array (sums of 1D ones)."""
    nx, ny, nz = grid
    lx = laplacian_eigenvalues_1d(nx)
    ly = laplacian_eigenvalues_1d(ny)
    lz = laplacian_eigenvalues_1d(nz)
    return lz[:, None, None] + ly[None, :, None] + lx[None, None, :]


class OracleProblem:
    """f, grad f and the Hartree solve for one workload (all float64)."""

    def __init__(self, prob):
        self.kind = prob.kind
        self.n = int(prob.n)
        self.p = int(prob.p)
        self.alpha = float(prob.alpha)
        self.grid = tuple(prob.grid)
        self.s_bound = float(prob.s_bound)
        self.block = int(getattr(prob, "block", 0) or 0)
        self.gamma = float(getattr(prob, "gamma", 0.0) or 0.0)
        gl = getattr(prob, "Glin", None)
        self.Glin = None if gl is None else np.asarray(gl, dtype=np.float64)
        b = getattr(prob, "B", None)
        self.B = None if b is None else np.asarray(b, dtype=np.float64)
        if prob.kind == "dense":
            self.A = np.asarray(prob.A, dtype=np.float64)
            self.L = None
            self.H0 = None
        else:
            if prob.kind == "stencil1d":
                self.L = laplacian_1d(self.n, self.block)
            elif prob.kind == "stencil3d":
                self.L = laplacian_3d(self.grid)
            else:
                raise ValueError(f"unknown problem kind {prob.kind}")
            if self.L.shape[0] != self.n:
                raise ValueError("grid does not match n")
            v = np.zeros(self.n) if prob.v is None else np.asarray(prob.v, np.float64)
            self.v = v
            self.H0 = (self.L + sp.diags(v)).tocsr()
            self.A = None
        self._lu = None

    # -- pieces of f -----------------------------------------------------
    @staticmethod
    def density(X: np.ndarray) -> np.ndarray:
        """rho = diag(X X^T): the squared norm of each row."""
        return np.einsum("ij,ij->i", X, X)

    def hartree(self, rho: np.ndarray) -> np.ndarray:
        """phi = L^{-1} rho (LU solve in 1D, sine-basis diagonalization in 3D)."""
        if self.L is None:
            raise ValueError("the dense problem has no Hartree term")
        rho = np.asarray(rho, dtype=np.float64)
        if self.kind == "stencil1d":
            if self._lu is None:
                self._lu = spla.splu(self.L.tocsc())
            phi = self._lu.solve(rho)
            # residual rho - T phi in extended precision, then one correction solve
            pe = phi.astype(np.longdouble)
            t = 2 * pe
            left = pe[:-1].copy()
            right = pe[1:].copy()
            if self.block and self.block < self.n:
                # no coupling across block boundaries
                cut = np.arange(self.block, self.n, self.block)
                left[cut - 1] = 0
                right[cut - 1] = 0
            t[1:] -= left
            t[:-1] -= right
            resid = (rho.astype(np.longdouble) - t).astype(np.float64)
            return phi + self._lu.solve(resid)
        nx, ny, nz = self.grid
        lam = laplacian_eigenvalues_3d(self.grid)
        r = rho.reshape(nz, ny, nx)
        t = sfft.dstn(r, type=1, norm="ortho")
        phi = sfft.dstn(t / lam, type=1, norm="ortho")
        return phi.reshape(-1)

    def apply_h0(self, X: np.ndarray) -> np.ndarray:
        """H0 X (sparse stencil or dense product)."""
        if self.A is not None:
            return self.A @ X
        return self.H0 @ X

    def _quad(self, X: np.ndarray) -> np.ndarray:
        """The gradient of the quadratic part: H0 X, or H0 X B (Problem 4)."""
        t = self.apply_h0(X)
        return t if self.B is None else t @ self.B

    # -- f and grad f ------------------------------------------------------
    def f(self, X: np.ndarray) -> float:
        val = 0.5 * float(np.sum(X * self._quad(X)))
        if self.Glin is not None:
            val += float(np.sum(self.Glin * X))
        if self.alpha != 0.0 or self.gamma != 0.0:
            rho = self.density(X)
            if self.alpha != 0.0:
                val += 0.25 * self.alpha * float(rho @ self.hartree(rho))
            if self.gamma != 0.0:
                val -= 0.75 * self.gamma * float(rho @ np.cbrt(rho))
        return val

    def grad(self, X: np.ndarray) -> np.ndarray:
        g = self._quad(X)
        if self.Glin is not None:
            g = g + self.Glin
        if self.alpha != 0.0 or self.gamma != 0.0:
            rho = self.density(X)
            if self.alpha != 0.0:
                phi = self.hartree(rho)
                g = g + self.alpha * phi[:, None] * X
            if self.gamma != 0.0:
                g = g - 2.0 * self.gamma * np.cbrt(rho)[:, None] * X
        return g

    def hess_vec(self, X: np.ndarray, xi: np.ndarray) -> np.ndarray:
        """Euclidean Hessian of f at X applied to xi.

        Differentiating grad f along xi: H0 xi + alpha Diag(phi) xi
        + alpha Diag(L^{-1} d rho) X with d rho = 2 rowdot(X, xi).
        """
        out = self._quad(xi)
        drho = 2.0 * np.einsum("ij,ij->i", X, xi)
        if self.alpha != 0.0:
            phi = self.hartree(self.density(X))
            dphi = self.hartree(drho)
            out = out + self.alpha * (phi[:, None] * xi + dphi[:, None] * X)
        if self.gamma != 0.0:
            # d/dt of -2 gamma rho^{1/3} X: -2 gamma (rho^{1/3} xi + rho^{-2/3} drho / 3 X)
            rho = self.density(X)
            c = np.cbrt(rho)
            out = out - 2.0 * self.gamma * (c[:, None] * xi
                                            + (drho / (3.0 * c * c))[:, None] * X)
        return out
