"""Python binding of the gfx950 PLAM / PCAL library (argument marshalling only).

Every step of the method runs in the HIP kernels of ``libstiefel.so``;
PyTorch is used only to own device memory and to name the stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np
import torch

from . import _lib as L

_PREC = {"fp64": L.PREC_FP64, "fp32": L.PREC_FP32, "mixed": L.PREC_MIXED,
         "mixed32": L.PREC_MIXED32}
_ETA = {"const": L.ETA_CONST, "diff": L.ETA_DIFF, "bb1": L.ETA_BB1, "bb2": L.ETA_BB2,
        "abb": L.ETA_ABB}
_KIND = {"stencil1d": L.KIND_STENCIL1D, "stencil3d": L.KIND_STENCIL3D, "dense": L.KIND_DENSE}
_VARIANT = {"plam": L.PLAM, "pcal": L.PCAL, "moptqr": L.MOPTQR}
_MULT = {"psi": L.MULT_PSI, "psi_phi": L.MULT_PSI_PHI, "dual": L.MULT_DUAL}


class StiefelError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {L.strerror(code)} (code {code})")
        self.code = code


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def storage_dtype(precision: str) -> torch.dtype:
    return torch.float64 if precision == "fp64" else torch.float32


@dataclass
class DeviceProblem:
    """A problem descriptor whose operator data lives on the GPU."""

    kind: str
    n: int
    p: int
    grid: Tuple[int, int, int]
    alpha: float
    v: Optional[torch.Tensor] = None     # float64, length n
    A: Optional[torch.Tensor] = None     # dense n x n, float64 or float32
    s_bound: float = 0.0
    name: str = ""
    block: int = 0                       # 1D: order of the tridiagonal blocks (0: one)
    gamma: float = 0.0                   # exchange weight (Problem 6)
    Glin: Optional[torch.Tensor] = None  # float64 n x p linear term (Problem 2)
    B: Optional[torch.Tensor] = None     # float64 p x p right factor (Problem 4)
    _c: Optional[L.StfProblem] = field(default=None, repr=False)

    @staticmethod
    def from_host(prob, device="cuda", A_dtype: Optional[torch.dtype] = None) -> "DeviceProblem":
        """Copy a ``workloads.Problem`` to the device."""
        v = None if prob.v is None else torch.as_tensor(np.ascontiguousarray(prob.v, np.float64),
                                                        device=device)
        A = None
        if prob.A is not None:
            dt = A_dtype or (torch.float32 if prob.A.dtype == np.float32 else torch.float64)
            A = torch.as_tensor(np.ascontiguousarray(prob.A), device=device).to(dt)
        grid = tuple(int(g) for g in prob.grid)

        def dev64(a):
            return None if a is None else torch.as_tensor(
                np.ascontiguousarray(a, np.float64), device=device)
        return DeviceProblem(kind=prob.kind, n=int(prob.n), p=int(prob.p), grid=grid,
                             alpha=float(prob.alpha), v=v, A=A, s_bound=float(prob.s_bound),
                             name=prob.name, block=int(getattr(prob, "block", 0) or 0),
                             gamma=float(getattr(prob, "gamma", 0.0) or 0.0),
                             Glin=dev64(getattr(prob, "Glin", None)),
                             B=dev64(getattr(prob, "B", None)))

    def c(self) -> L.StfProblem:
        cp = L.StfProblem()
        cp.kind = _KIND[self.kind]
        cp.p = self.p
        cp.n = self.n
        cp.grid[0], cp.grid[1], cp.grid[2] = self.grid
        cp.A_dtype = L.F64 if (self.A is None or self.A.dtype == torch.float64) else L.F32
        cp.alpha = self.alpha
        cp.v = _ptr(self.v)
        cp.A = _ptr(self.A)
        cp.block = int(self.block)
        cp.gamma = float(self.gamma)
        cp.Glin = _ptr(self.Glin)
        cp.B = _ptr(self.B)
        return cp


@dataclass
class SolveOptions:
    variant: str = "pcal"
    mult: str = "psi_phi"
    eta_rule: str = "abb"
    bb_index: str = "standard"
    precision: str = "fp64"
    max_iter: int = 3000
    kkt_every: int = 1
    orth_final: bool = True
    check_every: int = 50
    use_graph: bool = True
    profile: bool = False
    fused: bool = False
    beta: float = 1.0
    eta0: float = 1.0
    eta_const: float = 1.0
    tol: float = 1e-8
    feas_blowup: float = 1e3
    switch_tol: float = 0.0

    def c(self) -> L.StfOptions:
        o = L.StfOptions()
        o.variant = _VARIANT[self.variant]
        o.mult_rule = _MULT[self.mult]
        o.eta_rule = _ETA[self.eta_rule]
        o.bb_index = L.BB_LAGGED if self.bb_index == "lagged" else L.BB_STANDARD
        o.precision = _PREC[self.precision]
        o.max_iter = int(self.max_iter)
        o.kkt_every = int(self.kkt_every)
        o.orth_final = 1 if self.orth_final else 0
        o.check_every = int(self.check_every)
        o.use_graph = 1 if self.use_graph else 0
        o.profile = 1 if self.profile else 0
        o.fused = 1 if self.fused else 0
        o.beta = float(self.beta)
        o.eta0 = float(self.eta0)
        o.eta_const = float(self.eta_const)
        o.tol = float(self.tol)
        o.feas_blowup = float(self.feas_blowup)
        o.switch_tol = float(self.switch_tol)
        return o


def workspace_size(dp: DeviceProblem, opts: Optional[SolveOptions] = None) -> int:
    lib = L.load()
    cp = dp.c()
    co = opts.c() if opts is not None else None
    size = lib.stf_workspace_size(ctypes.byref(cp), ctypes.byref(co) if co is not None else None)
    if size == 0:
        raise StiefelError(L.E_INVALID, "stf_workspace_size")
    return int(size)


def alloc_workspace(dp: DeviceProblem, opts: Optional[SolveOptions] = None) -> torch.Tensor:
    return torch.empty(workspace_size(dp, opts), dtype=torch.uint8, device="cuda")


def solve(dp: DeviceProblem, X: torch.Tensor, opts: SolveOptions,
          workspace: Optional[torch.Tensor] = None, want_x64: bool = False,
          want_lambda: bool = False, stream=None, raise_on_error: bool = True,
          history: Optional[torch.Tensor] = None):
    """Run PLAM / PCAL in place on X (device, row-major n x p).

    history: optional device float64 tensor of shape (max_iter + 1, 4) that
    receives (KKT, feasibility, eta, k) per iteration.
    Returns (result dict, X64 or None, Lambda or None)."""
    lib = L.load()
    if X.dtype != storage_dtype(opts.precision) or not X.is_contiguous() or not X.is_cuda:
        raise ValueError("X must be a contiguous device tensor of the iteration dtype")
    if tuple(X.shape) != (dp.n, dp.p):
        raise ValueError("X has the wrong shape")
    cp, co = dp.c(), opts.c()
    if history is not None:
        if (history.dtype != torch.float64 or not history.is_cuda or not history.is_contiguous()
                or tuple(history.shape) != (opts.max_iter + 1, 4)):
            raise ValueError("history must be a contiguous device float64 (max_iter+1, 4) tensor")
        history.fill_(float("nan"))
        co.history = history.data_ptr()
    ws = workspace if workspace is not None else alloc_workspace(dp, opts)
    x64 = torch.empty((dp.n, dp.p), dtype=torch.float64, device=X.device) if want_x64 else None
    lam = torch.empty((dp.p, dp.p), dtype=torch.float64, device=X.device) if want_lambda else None
    res = L.StfResult()
    rc = lib.stf_solve(ctypes.byref(cp), ctypes.c_void_p(X.data_ptr()), ctypes.byref(co),
                       ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                       ctypes.c_void_p(_ptr(x64)) if x64 is not None else None,
                       ctypes.c_void_p(_ptr(lam)) if lam is not None else None,
                       ctypes.byref(res), _stream_handle(stream))
    out = _result_dict(res)
    out["rc"] = rc
    if rc < 0 and rc != L.E_DIVERGED and raise_on_error:
        raise StiefelError(rc, "stf_solve")
    return out, x64, lam


def _result_dict(res) -> dict:
    out = {k: getattr(res, k) for k, _ in L.StfResult._fields_ if k != "kernel_ms"}
    out["kernel_ms"] = {name: float(res.kernel_ms[i]) for i, name in enumerate(L.PROF_NAMES)}
    return out


def _opt_list(dps, opts):
    """One SolveOptions per problem (a single one is repeated)."""
    if isinstance(opts, SolveOptions):
        return [opts] * len(dps)
    if len(opts) != len(dps):
        raise ValueError("one SolveOptions per problem")
    return list(opts)


def _batch_args(dps, Xs, opts):
    if len(dps) != len(Xs) or not dps:
        raise ValueError("one X per problem, at least one problem")
    ol = _opt_list(dps, opts)
    cps = (L.StfProblem * len(dps))(*[dp.c() for dp in dps])
    cos = (L.StfOptions * len(dps))(*[o.c() for o in ol])
    for dp, X, o in zip(dps, Xs, ol):
        if X.dtype != storage_dtype(o.precision) or not X.is_contiguous() or not X.is_cuda:
            raise ValueError("each X must be a contiguous device tensor of the iteration dtype")
        if tuple(X.shape) != (dp.n, dp.p):
            raise ValueError("an X has the wrong shape")
    ptrs = (ctypes.c_void_p * len(Xs))(*[X.data_ptr() for X in Xs])
    return cps, cos, ptrs


def _vp(a):
    return ctypes.cast(a, ctypes.c_void_p)


def batched_workspace_size(dps, opts=None) -> int:
    """Workspace bytes of a batched solve; opts: one SolveOptions, a list, or None."""
    lib = L.load()
    cps = (L.StfProblem * len(dps))(*[dp.c() for dp in dps])
    cos = None if opts is None else (L.StfOptions * len(dps))(
        *[o.c() for o in _opt_list(dps, opts)])
    size = lib.stf_batched_workspace_size(len(dps), _vp(cps),
                                          _vp(cos) if cos is not None else None)
    if size == 0:
        raise StiefelError(L.E_INVALID, "stf_batched_workspace_size")
    return int(size)


def solve_batched(dps, Xs, opts, workspace: Optional[torch.Tensor] = None,
                  budgets=None, stream=None, raise_on_error: bool = True):
    """Solve many 1D problems together in place on their Xs (stf_solve_batched_ex).

    opts: one SolveOptions for all problems or a list with one per problem.
    budgets: optional (gram, residual) batch-wide workgroup budgets.
    Returns (list of result dicts, return code, loop ms per iteration)."""
    lib = L.load()
    cps, cos, ptrs = _batch_args(dps, Xs, opts)
    ws = workspace if workspace is not None else torch.empty(
        batched_workspace_size(dps, opts), dtype=torch.uint8, device="cuda")
    res = (L.StfResult * len(dps))()
    msi = ctypes.c_double(0.0)
    bg, br = budgets if budgets is not None else (0, 0)
    rc = lib.stf_solve_batched_ex(len(dps), _vp(cps), _vp(ptrs), _vp(cos),
                                  ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                  _vp(res), int(bg), int(br), ctypes.byref(msi),
                                  _stream_handle(stream))
    if rc < 0 and rc != L.E_DIVERGED and raise_on_error:
        raise StiefelError(rc, "stf_solve_batched_ex")
    return [_result_dict(r) for r in res], rc, float(msi.value)


def tune_batched(dps, Xs, opts, iters: int = 10, workspace: Optional[torch.Tensor] = None,
                 stream=None):
    """Pick the (gram, residual) budgets by timing (stf_batched_tune); Xs are advanced."""
    lib = L.load()
    cps, cos, ptrs = _batch_args(dps, Xs, opts)
    ws = workspace if workspace is not None else torch.empty(
        batched_workspace_size(dps, opts), dtype=torch.uint8, device="cuda")
    bg, br, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0.0)
    rc = lib.stf_batched_tune(len(dps), _vp(cps), _vp(ptrs), _vp(cos),
                              ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                              int(iters), ctypes.byref(bg), ctypes.byref(br), ctypes.byref(ms),
                              _stream_handle(stream))
    if rc < 0:
        raise StiefelError(rc, "stf_batched_tune")
    return (int(bg.value), int(br.value)), float(ms.value)


def gradient(dp: DeviceProblem, X: torch.Tensor, workspace=None, stream=None) -> torch.Tensor:
    lib = L.load()
    dt = L.F64 if X.dtype == torch.float64 else L.F32
    G = torch.empty_like(X)
    ws = workspace if workspace is not None else alloc_workspace(dp)
    cp = dp.c()
    rc = lib.stf_gradient(ctypes.byref(cp), ctypes.c_void_p(X.data_ptr()),
                          ctypes.c_void_p(G.data_ptr()), dt, ctypes.c_void_p(ws.data_ptr()),
                          ws.numel(), _stream_handle(stream))
    if rc:
        raise StiefelError(rc, "stf_gradient")
    return G


def hartree(dp: DeviceProblem, rho: torch.Tensor, workspace=None, stream=None) -> torch.Tensor:
    lib = L.load()
    phi = torch.empty_like(rho)
    ws = workspace if workspace is not None else alloc_workspace(dp)
    cp = dp.c()
    rc = lib.stf_hartree(ctypes.byref(cp), ctypes.c_void_p(rho.data_ptr()),
                         ctypes.c_void_p(phi.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                         ws.numel(), _stream_handle(stream))
    if rc:
        raise StiefelError(rc, "stf_hartree")
    return phi


def gram(dp: DeviceProblem, X: torch.Tensor, G: torch.Tensor, precision: str = "fp64",
         workspace=None, stream=None):
    lib = L.load()
    dt = L.F64 if X.dtype == torch.float64 else L.F32
    S = torch.empty((dp.p, dp.p), dtype=torch.float64, device=X.device)
    W = torch.empty_like(S)
    ws = workspace if workspace is not None else alloc_workspace(dp)
    cp = dp.c()
    rc = lib.stf_gram(ctypes.byref(cp), ctypes.c_void_p(X.data_ptr()),
                      ctypes.c_void_p(G.data_ptr()), dt, _PREC[precision],
                      ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(W.data_ptr()),
                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream))
    if rc:
        raise StiefelError(rc, "stf_gram")
    return S, W


def cholqr2(dp: DeviceProblem, X: torch.Tensor, workspace=None, stream=None) -> torch.Tensor:
    lib = L.load()
    Q = X.clone()
    ws = workspace if workspace is not None else alloc_workspace(dp)
    cp = dp.c()
    rc = lib.stf_cholqr2(ctypes.byref(cp), ctypes.c_void_p(Q.data_ptr()),
                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream))
    if rc:
        raise StiefelError(rc, "stf_cholqr2")
    return Q


def evaluate(dp: DeviceProblem, X: torch.Tensor, workspace=None, stream=None):
    """(f, ||G - X Psi(G^T X)||_F, ||X^T X - I||_F) of a float64 device X."""
    lib = L.load()
    out = (ctypes.c_double * 3)()
    ws = workspace if workspace is not None else alloc_workspace(dp)
    cp = dp.c()
    rc = lib.stf_eval(ctypes.byref(cp), ctypes.c_void_p(X.data_ptr()), out,
                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream))
    if rc:
        raise StiefelError(rc, "stf_eval")
    return float(out[0]), float(out[1]), float(out[2])


def adjoint_v(dp: DeviceProblem, Xstar: torch.Tensor, Lam: torch.Tensor, gradX: torch.Tensor,
              cg_tol: float = 1e-10, cg_maxit: int = 2000, workspace=None, stream=None):
    """dl/dV by implicit differentiation (pcal_adjoint_v); all tensors float64 on the device.

    Returns (gradV, cg_iters, cg_relres)."""
    lib = L.load()
    for t in (Xstar, Lam, gradX):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("adjoint inputs must be contiguous float64 device tensors")
    cp = dp.c()
    size = lib.stf_adjoint_workspace_size(ctypes.byref(cp))
    if size == 0:
        raise StiefelError(L.E_INVALID, "stf_adjoint_workspace_size")
    ws = workspace if workspace is not None else torch.empty(size, dtype=torch.uint8,
                                                             device=Xstar.device)
    gV = torch.empty(dp.n, dtype=torch.float64, device=Xstar.device)
    its = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    rc = lib.pcal_adjoint_v(ctypes.byref(cp), ctypes.c_void_p(Xstar.data_ptr()),
                            ctypes.c_void_p(Lam.data_ptr()), ctypes.c_void_p(gradX.data_ptr()),
                            ctypes.c_void_p(gV.data_ptr()), float(cg_tol), int(cg_maxit),
                            ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                            ctypes.byref(its), ctypes.byref(rr), _stream_handle(stream))
    if rc < 0:
        raise StiefelError(rc, "pcal_adjoint_v")
    return gV, int(its.value), float(rr.value)
