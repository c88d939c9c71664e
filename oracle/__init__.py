"""Plain FP64 CPU oracle of PLAM / PCAL (test infrastructure only).

This package is the independent reference the HIP path is checked against.
It is written from the paper (Gao, Liu, Yuan: "Parallelizable Algorithms for
Optimization Problems with Orthogonality Constraints") in float64 NumPy/SciPy,
step by step in the paper's order and notation, without blocking, fusion or
reordering.  It shares no code with the HIP library and never imports it.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from here; the product path must never route
through it.

Modules
-------
problems  : f, grad f, rho = diag(X X^T), the Hartree solve L^{-1} rho.
solver    : the PLAM / PCAL iteration, step-size rules, KKT measure,
            final CholeskyQR2.
rgd       : an independent Riemannian-gradient / QR-retraction solver used
            only to pin the converged objective of the nonlinear problems.
adjoint   : the implicit-differentiation reference for d loss(X*) / dV.
"""
