"""torch.autograd.Function around the PCAL solve and its adjoint.

``PCALSolve.apply(V, template, X0, opts)`` returns the orthonormal float64
stationary point X*(V) computed by ``stf_solve`` for the problem ``template``
with its diagonal potential replaced by V; the backward pass returns
dl/dV through ``pcal_adjoint_v`` (implicit differentiation on the horizontal
space, float64 conjugate gradients on the device).  The loss must be
invariant under X* -> X* Q for orthogonal Q (it is a function of the
subspace), which is what makes dl/dV well defined.
"""
from __future__ import annotations

import dataclasses

import torch

from . import stiefel as S


class PCALSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, template: S.DeviceProblem, X0: torch.Tensor, opts: S.SolveOptions,
                cg_tol: float = 1e-10, cg_maxit: int = 2000):
        if opts.precision != "fp64":
            raise ValueError("the differentiable solve runs the float64 form")
        dp = dataclasses.replace(template, v=V.detach().contiguous().to(torch.float64))
        X = X0.detach().clone().to(torch.float64).contiguous()
        stream = torch.cuda.Stream()
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            res, x64, lam = S.solve(dp, X, opts, want_x64=True, want_lambda=True, stream=stream)
        torch.cuda.current_stream().wait_stream(stream)
        if res["rc"] not in (0, 1):
            raise S.StiefelError(res["rc"], "PCALSolve.forward")
        ctx.dp = dp
        ctx.cg = (cg_tol, cg_maxit)
        ctx.info = res
        ctx.save_for_backward(x64, lam)
        return x64

    @staticmethod
    def backward(ctx, gX):
        x64, lam = ctx.saved_tensors
        gV, its, rr = S.adjoint_v(ctx.dp, x64, lam, gX.contiguous().to(torch.float64),
                                  cg_tol=ctx.cg[0], cg_maxit=ctx.cg[1])
        ctx.info["cg_iters"] = its
        ctx.info["cg_relres"] = rr
        return gV, None, None, None, None, None
