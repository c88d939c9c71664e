"""The C-ABI library loads and exports every entry point include/stiefel.h declares.

Host-only: no call here touches a GPU (stf_workspace_size, stf_strerror and
stf_version are pure host functions; argument validation of the compute entry
points returns before any device work).
"""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_1810_03930_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in os.listdir(os.path.join(ROOT, "include"))
           if h.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M):
            name = m.group(1)
            if name not in ("if", "for", "while", "return", "sizeof"):
                names.append(name)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = declared_functions()
    assert "stf_solve" in names and "pcal_solve" in names and "plam_solve" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) <= set(L.SIGNATURES), \
        set(declared_functions()) - set(L.SIGNATURES)


def test_struct_layouts_match_header():
    # offsets and sizes that the C compiler gives the structs on x86-64
    assert ctypes.sizeof(L.StfProblem) == 88
    assert L.StfProblem.alpha.offset == 32 and L.StfProblem.A.offset == 48
    assert L.StfProblem.block.offset == 56 and L.StfProblem.gamma.offset == 64
    assert L.StfProblem.Glin.offset == 72 and L.StfProblem.B.offset == 80
    assert ctypes.sizeof(L.StfOptions) == 48 + 56
    assert L.StfOptions.beta.offset == 48 and L.StfOptions.history.offset == 96
    assert ctypes.sizeof(L.StfResult) == 8 + 8 * 8 + 8 * 8 + 16
    assert L.StfResult.restarted.offset == 144


@pytest.mark.skipif(shutil.which("gcc") is None or
                    not os.path.isdir("/opt/rocm/include"), reason="needs gcc and HIP headers")
def test_struct_layouts_match_c_compiler(tmp_path):
    """Every field offset and struct size of the binding, against what gcc
    makes of include/stiefel.h."""
    structs = {"stf_problem": L.StfProblem, "stf_options": L.StfOptions,
               "stf_result": L.StfResult}
    lines = ['#include <stdio.h>', '#include "stiefel.h"', "int main(void) {"]
    for cname, ct in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in ct._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.splitlines():
        cname, f, v = line.split()
        ct = structs[cname]
        got = ctypes.sizeof(ct) if f == "sizeof" else getattr(ct, f).offset
        assert got == int(v), (cname, f, got, v)


def _problem(kind=L.KIND_STENCIL1D, n=1000, p=10, grid=None):
    cp = L.StfProblem()
    cp.kind, cp.n, cp.p = kind, n, p
    g = grid or (n, 1, 1)
    cp.grid[0], cp.grid[1], cp.grid[2] = g
    cp.A_dtype = L.F64
    cp.alpha = 1.0
    return cp


def test_workspace_size_host_only():
    lib = L.load()
    ok = _problem()
    assert lib.stf_workspace_size(ctypes.byref(ok), None) > 1000 * 10 * 8
    bad = _problem(n=15, p=10)                 # n < 2p (Section 1 requires 2p <= n)
    assert lib.stf_workspace_size(ctypes.byref(bad), None) == 0
    bad3 = _problem(kind=L.KIND_STENCIL3D, n=1000, grid=(10, 10, 9))
    assert lib.stf_workspace_size(ctypes.byref(bad3), None) == 0
    dense_no_a = _problem(kind=L.KIND_DENSE)
    assert lib.stf_workspace_size(ctypes.byref(dense_no_a), None) == 0
    opt = L.StfOptions()
    opt.precision = L.PREC_FP64
    s64 = lib.stf_workspace_size(ctypes.byref(ok), ctypes.byref(opt))
    opt.variant = L.MOPTQR                     # the comparator keeps a second iterate
    s64m = lib.stf_workspace_size(ctypes.byref(ok), ctypes.byref(opt))
    opt.variant = L.PCAL
    opt.precision = L.PREC_FP32
    s32 = lib.stf_workspace_size(ctypes.byref(ok), ctypes.byref(opt))
    assert s64 > 0 and s32 > 0 and s64m >= s64 + 2 * 1000 * 10 * 8
    # the single-pass form keeps a second iterate and the row partials of rho
    opt.fused = 1
    s32f = lib.stf_workspace_size(ctypes.byref(ok), ctypes.byref(opt))
    opt.precision = L.PREC_FP64
    s64f = lib.stf_workspace_size(ctypes.byref(ok), ctypes.byref(opt))
    opt.variant = L.MOPTQR
    s64mf = lib.stf_workspace_size(ctypes.byref(ok), ctypes.byref(opt))
    assert s32f >= s32 + 1000 * 10 * 8 and s64f >= s64 + 1000 * 10 * 8
    # without options: room for every form
    assert lib.stf_workspace_size(ctypes.byref(ok), None) == max(s64mf, s32f)
    assert max(s64mf, s32f) >= max(s64m, s32, s64f)


def test_invalid_arguments_rejected_before_device_work():
    lib = L.load()
    bad = _problem(n=15, p=10)
    res = L.StfResult()
    opt = L.StfOptions()
    rc = lib.stf_solve(ctypes.byref(bad), None, ctypes.byref(opt), None, 0, None, None,
                       ctypes.byref(res), None)
    assert rc == L.E_INVALID
    ok = _problem()
    opt.variant = 7
    rc = lib.stf_solve(ctypes.byref(ok), ctypes.c_void_p(1), ctypes.byref(opt),
                       ctypes.c_void_p(1), 1, None, None, ctypes.byref(res), None)
    assert rc == L.E_INVALID
    # the Phi-corrected multiplier is a PCAL rule (eq. (lambda2))
    opt.variant, opt.mult_rule, opt.eta_rule, opt.kkt_every, opt.check_every = \
        L.PLAM, L.MULT_PSI_PHI, L.ETA_ABB, 1, 1
    opt.eta0, opt.tol = 1.0, 1e-8
    rc = lib.stf_solve(ctypes.byref(ok), ctypes.c_void_p(1), ctypes.byref(opt),
                       ctypes.c_void_p(1), 1, None, None, ctypes.byref(res), None)
    assert rc == L.E_UNSUPPORTED
    # too small a workspace is refused before anything is enqueued
    opt.mult_rule = L.MULT_PSI
    rc = lib.stf_solve(ctypes.byref(ok), ctypes.c_void_p(1), ctypes.byref(opt),
                       ctypes.c_void_p(1), 1, None, None, ctypes.byref(res), None)
    assert rc == L.E_WORKSPACE


def test_strerror_and_version():
    for code in [0, 1, 2, -1, -2, -3, -4, -5, -6, -7]:
        assert len(L.strerror(code)) > 5
    assert L.strerror(12345) == "unknown status"
    assert L.load().stf_version().decode().startswith("stiefel")


def _valid_options(prec=L.PREC_FP64):
    o = L.StfOptions()
    o.variant, o.mult_rule, o.eta_rule, o.precision = L.PCAL, L.MULT_PSI_PHI, L.ETA_ABB, prec
    o.max_iter, o.kkt_every, o.check_every = 10, 1, 5
    o.beta, o.eta0, o.tol = 10.0, 14.0, 1e-8
    return o


def test_batched_host_checks():
    lib = L.load()
    vp = lambda a: ctypes.cast(a, ctypes.c_void_p)
    probs = (L.StfProblem * 2)(_problem(n=1000, p=10), _problem(n=1500, p=40))
    assert lib.stf_batched_workspace_size(2, vp(probs), None) > 0
    opts = (L.StfOptions * 2)(_valid_options(), _valid_options())
    s64 = lib.stf_batched_workspace_size(2, vp(probs), vp(opts))
    assert s64 > 1000 * 10 * 8 + 1500 * 40 * 8
    # the grouped passes are the 1D ones
    p3 = (L.StfProblem * 1)(_problem(kind=L.KIND_STENCIL3D, n=1000, grid=(10, 10, 10)))
    assert lib.stf_batched_workspace_size(1, vp(p3), None) == 0
    # one storage dtype per batch
    mixed = (L.StfOptions * 2)(_valid_options(), _valid_options(L.PREC_FP32))
    assert lib.stf_batched_workspace_size(2, vp(probs), vp(mixed)) == 0
    res = (L.StfResult * 2)()
    ptrs = (ctypes.c_void_p * 2)(1, 1)
    assert lib.stf_solve_batched(0, vp(probs), vp(ptrs), vp(opts), ctypes.c_void_p(1), 1,
                                 vp(res), None) == L.E_INVALID
    p3b = (L.StfProblem * 2)(_problem(n=1000, p=10),
                             _problem(kind=L.KIND_STENCIL3D, n=1000, grid=(10, 10, 10)))
    assert lib.stf_solve_batched(2, vp(p3b), vp(ptrs), vp(opts), ctypes.c_void_p(1), 1,
                                 vp(res), None) == L.E_UNSUPPORTED
    assert lib.stf_solve_batched(2, vp(probs), vp(ptrs), vp(opts), ctypes.c_void_p(1), 1,
                                 vp(res), None) == L.E_WORKSPACE


def test_problem_terms_and_comparator_host_checks():
    """The Problem 2 / 4 / 6 terms, the block operator and MOptQR are validated on
    the host before any device work."""
    lib = L.load()
    res = L.StfResult()
    ok = _problem()
    ok.block = 5
    assert lib.stf_workspace_size(ctypes.byref(ok), None) > 0
    bad = _problem(kind=L.KIND_STENCIL3D, n=1000, grid=(10, 10, 10))
    bad.block = 5                               # blocks belong to the 1D operator
    assert lib.stf_workspace_size(ctypes.byref(bad), None) == 0
    neg = _problem()
    neg.block = -1
    assert lib.stf_workspace_size(ctypes.byref(neg), None) == 0
    rf = _problem()
    rf.B = 1                                    # right factor with a Hartree term
    assert lib.stf_workspace_size(ctypes.byref(rf), None) == 0
    rf.alpha = 0.0
    assert lib.stf_workspace_size(ctypes.byref(rf), None) > 0
    dn = _problem(kind=L.KIND_DENSE)
    dn.A = 1
    dn.alpha = 0.0
    dn.gamma = 1.0                              # the exchange term needs a density
    assert lib.stf_workspace_size(ctypes.byref(dn), None) == 0
    # MOptQR is a float64 comparator
    o = _valid_options(L.PREC_FP32)
    o.variant = L.MOPTQR
    rc = lib.stf_solve(ctypes.byref(_problem()), ctypes.c_void_p(1), ctypes.byref(o),
                       ctypes.c_void_p(1), 1, None, None, ctypes.byref(res), None)
    assert rc == L.E_UNSUPPORTED
    o.precision = L.PREC_FP64
    rc = lib.stf_solve(ctypes.byref(_problem()), ctypes.c_void_p(1), ctypes.byref(o),
                       ctypes.c_void_p(1), 1, None, None, ctypes.byref(res), None)
    assert rc == L.E_WORKSPACE
    # dual ascent for both variants; an unknown multiplier rule is refused
    o.variant, o.mult_rule = L.PLAM, L.MULT_DUAL
    rc = lib.stf_solve(ctypes.byref(_problem()), ctypes.c_void_p(1), ctypes.byref(o),
                       ctypes.c_void_p(1), 1, None, None, ctypes.byref(res), None)
    assert rc == L.E_WORKSPACE
    o.mult_rule = 9
    rc = lib.stf_solve(ctypes.byref(_problem()), ctypes.c_void_p(1), ctypes.byref(o),
                       ctypes.c_void_p(1), 1, None, None, ctypes.byref(res), None)
    assert rc == L.E_INVALID
    # the batched solver covers Problem 1 only
    vp = lambda a: ctypes.cast(a, ctypes.c_void_p)
    ex = _problem()
    ex.gamma = 1.0
    probs = (L.StfProblem * 1)(ex)
    assert lib.stf_batched_workspace_size(1, vp(probs), None) == 0


def test_single_pass_form_host_checks():
    """The single-pass form (options.fused) needs eta^k before the pass (the
    lagged pair, not eta_D), p > 64, PLAM / PCAL and the float64 or MIXED32
    precision (p <= 384 there); the rest is refused before any device work."""
    lib = L.load()
    res = L.StfResult()
    ok = _problem(n=4000, p=100)

    def rc_of(o, prob=ok):
        return lib.stf_solve(ctypes.byref(prob), ctypes.c_void_p(1), ctypes.byref(o),
                             ctypes.c_void_p(1), 1, None, None, ctypes.byref(res), None)

    o = _valid_options(L.PREC_FP64)
    o.fused, o.bb_index = 1, L.BB_LAGGED
    assert rc_of(o) == L.E_WORKSPACE            # accepted: only the workspace is short
    o.precision = L.PREC_MIXED32
    assert rc_of(o) == L.E_WORKSPACE
    for prec in (L.PREC_FP32, L.PREC_MIXED):
        o.precision = prec
        assert rc_of(o) == L.E_UNSUPPORTED
    o.precision = L.PREC_FP64
    o.bb_index = L.BB_STANDARD
    assert rc_of(o) == L.E_UNSUPPORTED
    o.bb_index, o.eta_rule = L.BB_LAGGED, L.ETA_DIFF
    assert rc_of(o) == L.E_UNSUPPORTED
    o.eta_rule = L.ETA_BB2
    assert rc_of(o) == L.E_WORKSPACE
    o.variant = L.MOPTQR
    assert rc_of(o) == L.E_UNSUPPORTED
    o.variant = L.PLAM
    o.mult_rule = L.MULT_DUAL
    assert rc_of(o) == L.E_WORKSPACE
    assert rc_of(o, _problem(n=4000, p=64)) == L.E_UNSUPPORTED
    o.precision = L.PREC_MIXED32
    assert rc_of(o, _problem(n=4000, p=416)) == L.E_UNSUPPORTED
    assert rc_of(o, _problem(n=4000, p=384)) == L.E_WORKSPACE
    # not in the batched solver
    vp = lambda a: ctypes.cast(a, ctypes.c_void_p)
    probs = (L.StfProblem * 1)(ok)
    opts = (L.StfOptions * 1)(_valid_options())
    opts[0].fused = 1
    ptrs = (ctypes.c_void_p * 1)(1)
    bres = (L.StfResult * 1)()
    assert lib.stf_solve_batched(1, vp(probs), vp(ptrs), vp(opts), ctypes.c_void_p(1), 1,
                                 vp(bres), None) == L.E_UNSUPPORTED
