"""stf_gram_noalloc (the entry point that allocates nothing) against stf_gram,
through the C ABI: two calls in a row, the second with a smaller input, in
float64 (1e-13 relative, the bar of the float64 Gram steps; elementwise too)
and in the split-bf16 form (1e-13 against stf_gram's own split-bf16 result:
the same products, summed in another chunk order); and the refusal of a
problem whose partials cannot fit the static buffer."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from paper_1810_03930_amd import _lib as L
from paper_1810_03930_amd import stiefel as S
from tests.helpers import maxrel, rel, to_dev, to_np

pytestmark = pytest.mark.gpu


def _noalloc(dp, X, G, precision):
    lib = L.load()
    S_ = torch.empty((dp.p, dp.p), dtype=torch.float64, device="cuda")
    W_ = torch.empty_like(S_)
    cp = dp.c()
    dt = L.F64 if X.dtype == torch.float64 else L.F32
    rc = lib.stf_gram_noalloc(ctypes.byref(cp), ctypes.c_void_p(X.data_ptr()),
                              ctypes.c_void_p(G.data_ptr()), dt,
                              {"fp64": L.PREC_FP64, "fp32": L.PREC_FP32,
                               "mixed": L.PREC_MIXED}[precision],
                              ctypes.c_void_p(S_.data_ptr()), ctypes.c_void_p(W_.data_ptr()),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, to_np(S_), to_np(W_)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_gram_matches_stf_gram_twice(precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    # the first call covers many chunks and wide tiles, the second is smaller
    for call, (n, p) in enumerate([(200000, 300), (5003, 37)]):
        prob = W.Problem(name="g", kind="stencil1d", n=n, p=p, alpha=0.0)
        dp = S.DeviceProblem.from_host(prob)
        X = to_dev(W.random_matrix(60 + call, (n, p)), dt)
        G = to_dev(W.random_matrix(70 + call, (n, p)), dt)
        rc, Sn, Wn = _noalloc(dp, X, G, precision)
        assert rc == 0, L.strerror(rc)
        Sr, Wr = S.gram(dp, X, G, precision=precision)
        Sr, Wr = to_np(Sr), to_np(Wr)
        for a, b in ((Sn, Sr), (Wn, Wr)):
            assert rel(a, b) <= 1e-13 and maxrel(a, b) <= 1e-13, (call, n, p)


def test_noalloc_gram_refuses_what_does_not_fit():
    n, p = 8200, 4096
    prob = W.Problem(name="g", kind="stencil1d", n=n, p=p, alpha=0.0)
    dp = S.DeviceProblem.from_host(prob)
    X = torch.zeros((n, p), dtype=torch.float64, device="cuda")
    rc, _, _ = _noalloc(dp, X, X, "fp64")
    assert rc == L.E_SCRATCH
