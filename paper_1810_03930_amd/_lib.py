"""ctypes declarations of the C ABI in include/stiefel.h.

Loading fails loudly when the shared library is missing: there is no CPU
fallback anywhere in the product path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstiefel.so")

# enums (mirrors of the #defines in stiefel.h)
KIND_STENCIL1D, KIND_STENCIL3D, KIND_DENSE = 0, 1, 2
F64, F32 = 0, 1
PLAM, PCAL, MOPTQR = 0, 1, 2
MULT_PSI, MULT_PSI_PHI, MULT_DUAL = 0, 1, 2
ETA_CONST, ETA_DIFF, ETA_BB1, ETA_BB2, ETA_ABB = 0, 1, 2, 3, 4
BB_STANDARD, BB_LAGGED = 0, 1
PREC_FP64, PREC_FP32, PREC_MIXED, PREC_MIXED32 = 0, 1, 2, 3
OK, MAX_ITER, TOL_UNMET = 0, 1, 2
E_INVALID, E_DIVERGED, E_HIP, E_UNSUPPORTED, E_WORKSPACE, E_CHOLESKY = -1, -2, -3, -4, -5, -6
E_SCRATCH = -7
NOALLOC_SCRATCH_BYTES = 64 << 20


class StfProblem(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("p", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("grid", ctypes.c_int32 * 3),
        ("A_dtype", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("v", ctypes.c_void_p),
        ("A", ctypes.c_void_p),
        ("block", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("Glin", ctypes.c_void_p),
        ("B", ctypes.c_void_p),
    ]


class StfOptions(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32),
        ("mult_rule", ctypes.c_int32),
        ("eta_rule", ctypes.c_int32),
        ("bb_index", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("kkt_every", ctypes.c_int32),
        ("orth_final", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("fused", ctypes.c_int32),
        ("beta", ctypes.c_double),
        ("eta0", ctypes.c_double),
        ("eta_const", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("feas_blowup", ctypes.c_double),
        ("switch_tol", ctypes.c_double),
        ("history", ctypes.c_void_p),
    ]


class StfResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("kkt0", ctypes.c_double),
        ("kkt_abs", ctypes.c_double),
        ("kkt_rel", ctypes.c_double),
        ("feas", ctypes.c_double),
        ("fval", ctypes.c_double),
        ("eta_last", ctypes.c_double),
        ("ms_loop", ctypes.c_double),
        ("ms_orth", ctypes.c_double),
        ("kernel_ms", ctypes.c_double * 8),
        ("prof_iters", ctypes.c_int32),
        ("switch_iter", ctypes.c_int32),
        ("restarted", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

PROF_NAMES = ["hartree", "grad", "gram", "stage1", "residual", "stage2", "update"]


_P = ctypes.POINTER
_VP = ctypes.c_void_p
_SZ = ctypes.c_size_t

# name -> (restype, argtypes)
SIGNATURES = {
    "stf_workspace_size": (_SZ, [_P(StfProblem), _P(StfOptions)]),
    "stf_solve": (ctypes.c_int, [_P(StfProblem), _VP, _P(StfOptions), _VP, _SZ, _VP, _VP,
                                 _P(StfResult), _VP]),
    "plam_solve": (ctypes.c_int, [_P(StfProblem), _VP, _P(StfOptions), _VP, _SZ, _VP, _VP,
                                  _P(StfResult), _VP]),
    "pcal_solve": (ctypes.c_int, [_P(StfProblem), _VP, _P(StfOptions), _VP, _SZ, _VP, _VP,
                                  _P(StfResult), _VP]),
    "stf_gradient": (ctypes.c_int, [_P(StfProblem), _VP, _VP, ctypes.c_int32, _VP, _SZ, _VP]),
    "stf_hartree": (ctypes.c_int, [_P(StfProblem), _VP, _VP, _VP, _SZ, _VP]),
    "stf_gram": (ctypes.c_int, [_P(StfProblem), _VP, _VP, ctypes.c_int32, ctypes.c_int32, _VP,
                                _VP, _VP, _SZ, _VP]),
    "stf_cholqr2": (ctypes.c_int, [_P(StfProblem), _VP, _VP, _SZ, _VP]),
    "stf_eval": (ctypes.c_int, [_P(StfProblem), _VP, _P(ctypes.c_double), _VP, _SZ, _VP]),
    "stf_adjoint_workspace_size": (_SZ, [_P(StfProblem)]),
    "pcal_adjoint_v": (ctypes.c_int, [_P(StfProblem), _VP, _VP, _VP, _VP, ctypes.c_double,
                                      ctypes.c_int32, _VP, _SZ, _P(ctypes.c_int32),
                                      _P(ctypes.c_double), _VP]),
    "stf_batched_workspace_size": (_SZ, [ctypes.c_int32, _VP, _VP]),
    "stf_solve_batched": (ctypes.c_int, [ctypes.c_int32, _VP, _VP, _VP, _VP, _SZ, _VP, _VP]),
    "pcal_solve_batched": (ctypes.c_int, [ctypes.c_int32, _VP, _VP, _VP, _VP, _SZ, _VP, _VP]),
    "stf_solve_batched_ex": (ctypes.c_int, [ctypes.c_int32, _VP, _VP, _VP, _VP, _SZ,
                                            _VP, ctypes.c_int32, ctypes.c_int32,
                                            _P(ctypes.c_double), _VP]),
    "stf_batched_tune": (ctypes.c_int, [ctypes.c_int32, _VP, _VP, _VP, _VP, _SZ,
                                        ctypes.c_int32, _P(ctypes.c_int32), _P(ctypes.c_int32),
                                        _P(ctypes.c_double), _VP]),
    "stf_gram_noalloc": (ctypes.c_int, [_P(StfProblem), _VP, _VP, ctypes.c_int32,
                                        ctypes.c_int32, _VP, _VP, _VP]),
    "stf_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "stf_version": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libstiefel.so and declare every exported entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_1810_03930_amd.build` "
            "(the HIP library is required; there is no fallback)")
    try:
        # bind to the HIP runtime torch has loaded (one runtime per process, so
        # torch's streams and device pointers are valid in the library)
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().stf_strerror(int(code)).decode()
