"""Benchmark: PCAL on the 3D Kohn-Sham-shaped workload (64^3 grid, n = 262144, p = 256).

One "step" is one PCAL iteration (Algorithm 3): Hartree solve, gradient,
Gram products, p x p multiplier stage, residual / step-size pass, update.

Reported (one JSON line on stdout):
  value        PCAL iterations/s of the fast (reduced-precision) form, inputs
               resident in HBM, over exactly `--steps` iterations after
               `--warmup` untimed ones
  forms        per form (fp64 and the fast form): iterations/s, time to
               relative KKT <= 1e-6 (loop + CholeskyQR2 + float64 check),
               iterations to that point, f, KKT and feasibility at the end
  speedup      time-to-KKT of the fp64 form / that of the fast form
  roofline     the dominant kernel of the fast form's timed steps
  cpu_baseline the float64 oracle on this host's cores, on a bounded sample
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GRID = (64, 64, 64)
P = 256
ALPHA = 1.0
BETA = 2.0          # PCAL penalty for the 3D KS workloads (see the design notes)
TOL = 1e-6
MAX_ITER = 3000
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "mixed_bf16": 2500.0}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_algorithmic(name, n, p, s, kkt_every=1):
    """Algorithmic (bytes, flops) of one launch of a kernel group per iteration.

    s = bytes per element of X / G.  Bytes count each operand read or written
    once; flops count multiply-adds as 2.
    """
    nps = float(n) * p * s
    if name == "grad":        # read X (+ neighbours, cached), v, phi; write G
        return 2 * nps + 16.0 * n, 15.0 * n * p
    if name == "gram":        # read X, G; S upper half + W full
        return 2 * nps, 3.0 * n * p * p
    if name == "residual":    # read X, G, gradL_prev; write gradL; X M_L (+ X Psi)
        return 4 * nps, (2.0 + 2.0 / kkt_every) * n * p * p
    if name == "update":      # read X, gradL; write X and rho
        return 3 * nps + 8.0 * n, 4.0 * n * p
    if name == "hartree":     # six 1D sine transforms over the grid
        return 7 * 8.0 * n, 6 * 2.0 * n * max(GRID)
    return 0.0, 0.0


def run_form(dp, x0, precision, steps, warmup, S, torch):
    """Timed steps (profiled per kernel) and a time-to-KKT solve for one form."""
    dt = S.storage_dtype(precision)
    eta0 = BETA + dp.s_bound
    common = dict(variant="pcal", mult="psi_phi", eta_rule="abb", precision=precision,
                  beta=BETA, eta0=eta0)
    stream = torch.cuda.Stream()
    ws = S.alloc_workspace(dp, S.SolveOptions(**common))
    X = torch.empty((dp.n, dp.p), dtype=dt, device="cuda")
    x0_dev = torch.as_tensor(x0, device="cuda").to(dt)

    def fresh():
        X.copy_(x0_dev)
        torch.cuda.synchronize()

    with torch.cuda.stream(stream):
        # warmup: `warmup` untimed iterations
        fresh()
        S.solve(dp, X, S.SolveOptions(**common, tol=0.0, max_iter=max(1, warmup),
                                      orth_final=False, check_every=max(1, warmup),
                                      use_graph=False), workspace=ws, stream=stream)
        # timed: exactly `steps` iterations, every kernel group bracketed by events
        fresh()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, _, _ = S.solve(dp, X, S.SolveOptions(**common, tol=0.0, max_iter=steps,
                                                  orth_final=False, check_every=steps,
                                                  use_graph=False, profile=True),
                            workspace=ws, stream=stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # the loop also evaluates the stop test at k = steps (one extra partial pass)
        ms_step = res["ms_loop"] / steps
        prof_n = max(1, res["prof_iters"])
        kernel_avg_ms = {k: v / prof_n for k, v in res["kernel_ms"].items()}
        # time to relative KKT <= TOL from X0 resident in HBM, graph-replayed loop
        fresh()
        t0 = time.perf_counter()
        conv, x64, _ = S.solve(dp, X, S.SolveOptions(**common, tol=TOL, max_iter=MAX_ITER,
                                                     orth_final=True, check_every=50,
                                                     use_graph=True),
                               workspace=ws, stream=stream, want_x64=True)
        torch.cuda.synchronize()
        wall_kkt = time.perf_counter() - t0
    out = {
        "iters_per_s": 1000.0 / ms_step,
        "ms_per_step": ms_step,
        "timed_wall_s": wall,
        "kernel_avg_ms": kernel_avg_ms,
        "time_to_kkt_s": (conv["ms_loop"] + conv["ms_orth"]) / 1000.0,
        "time_to_kkt_wall_s": wall_kkt,
        "iters_to_kkt": conv["iters"],
        "status": conv["rc"],
        "kkt_rel": conv["kkt_rel"],
        "kkt_abs": conv["kkt_abs"],
        "feas": conv["feas"],
        "f": conv["fval"],
        "ms_orth": conv["ms_orth"],
    }
    return out, x64


def roofline_for(form, precision, n, p):
    s = 8 if precision == "fp64" else 4
    ka = form["kernel_avg_ms"]
    name = max(ka, key=lambda k: ka[k])
    ms = ka[name]
    by, fl = kernel_algorithmic(name, n, p, s)
    peak_key = "fp64" if precision == "fp64" else ("fp32" if precision == "fp32" else "mixed_bf16")
    t_mem = by / (HBM_PEAK_GBS * 1e9)
    t_mma = fl / (PEAK_TFLOPS[peak_key] * 1e12)
    if t_mma > t_mem:
        ach = fl / (ms * 1e-3) / 1e12
        peak = PEAK_TFLOPS[peak_key]
        return {"kernel": name, "bound": "mfma", "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "traffic": None,
                "avg_launch_ms": ms, "algorithmic_flops": fl}
    ach = by / (ms * 1e-3) / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None, "avg_launch_ms": ms,
            "algorithmic_bytes": by}


def cpu_baseline(prob, x0):
    """The float64 oracle, unchanged, on this host: per-iteration cost from a
    1-iteration and a 4-iteration run (the difference is 3 full iterations)."""
    from threadpoolctl import threadpool_info
    from oracle.problems import OracleProblem
    from oracle import solver as O
    op = OracleProblem(prob)
    cores = len(os.sched_getaffinity(0))
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    opt = dict(variant="pcal", beta=BETA, eta0=BETA + prob.s_bound, tol=0.0, orth_final=False)
    t0 = time.perf_counter()
    O.solve(op, x0, O.Options(max_iter=1, **opt))
    t1 = time.perf_counter()
    O.solve(op, x0, O.Options(max_iter=4, **opt))
    t2 = time.perf_counter()
    per_iter = ((t2 - t1) - (t1 - t0)) / 3.0
    return {"value": 1.0 / per_iter, "unit": "iters/s", "cores": int(min(cores, threads)),
            "kind": "oracle", "sample": "3 PCAL iterations of the 64^3 p=256 workload "
            f"(difference of a 4- and a 1-iteration float64 run; {t2 - t0:.1f} s total)",
            "s_per_iter": per_iter, "host_cores_visible": cores, "blas_threads": threads}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--fast-form", default="fp32", choices=["fp32", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1810_03930_amd import stiefel as S

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    log("generating the 64^3 p=256 workload (seeded)")
    prob, x0, _ = W.ks3d(grid=GRID, p=P, alpha=ALPHA)
    dp = S.DeviceProblem.from_host(prob)
    forms = {}
    for prec in ["fp64", args.fast_form]:
        log(f"form {prec}: {args.warmup} warmup + {args.steps} timed steps, then time-to-KKT")
        forms[prec], _ = run_form(dp, x0, prec, args.steps, args.warmup, S, torch)
        log(f"form {prec}: {json.dumps(forms[prec])}")
    fast = forms[args.fast_form]
    base = forms["fp64"]
    roof = roofline_for(fast, args.fast_form, prob.n, P)
    roof64 = roofline_for(base, "fp64", prob.n, P)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: float64 oracle on the host")
        cpu = cpu_baseline(prob, x0)
    line = {
        "metric": "PCAL iters/s + time-to-||KKT||<=1e-6, mixed vs FP64 form, n=262144 p=256",
        "value": fast["iters_per_s"],
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fast["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.fast_form == "fp32" else "f32+bf16x3",
        "data": "synthetic",
        "config": {"workload": "3D Kohn-Sham-shaped PCAL, 7-point Dirichlet Laplacian on a "
                               "64^3 grid + Diag(V), V~U(0,1), alpha=1, beta=2, ABB steps",
                   "n": prob.n, "p": P, "grid": list(GRID), "tol_rel_kkt": TOL,
                   "fast_form": args.fast_form},
        "time_to_kkt_s": {"fp64": base["time_to_kkt_s"], args.fast_form: fast["time_to_kkt_s"]},
        "speedup_time_to_kkt": base["time_to_kkt_s"] / fast["time_to_kkt_s"],
        "forms": forms,
        "roofline": roof,
        "roofline_fp64": roof64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
