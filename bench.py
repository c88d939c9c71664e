"""Benchmark: PCAL on the 3D Kohn-Sham-shaped workload (64^3 grid, n = 262144, p = 256).

One "step" is one PCAL iteration (Algorithm 3): Hartree solve, gradient,
Gram products, p x p multiplier stage, residual / step-size pass, update.

Reported (one JSON line on stdout):
  value        PCAL iterations/s of the fast form (mixed32: split-bf16 MFMA
               products, float32 storage, no float64 master), inputs
               resident in HBM, over exactly `--steps` iterations after
               `--warmup` untimed ones (device events around the loop)
  forms        per form (fp64 and the fast form): iterations/s, per-kernel
               average times, time to relative KKT <= 1e-6 (loop +
               CholeskyQR2 + float64 check; the fast form hands over to
               float64 at relative KKT 1e-4) from 15 seeded starts, the
               median and the reached/total count, f, KKT and feasibility
  speedup      median time-to-KKT of the fp64 form / that of the fast form
  result_error_vs_fp64  per reduced-precision form: f, KKT, feasibility and
               the subspace distance of its returned point against fp64's
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
BETA = 4.0          # PCAL penalty for the 3D KS workload (above its p-th eigenvalue)
TOL = 1e-6
SWITCH_TOL = 1e-4   # relative KKT at which the fast form continues in float64
BATCH_SWITCH_TOL = 1e-3
MAX_ITER = 6000
HBM_PEAK_GBS = 8000.0
FORM_DTYPE = {"fp32": "f32", "mixed": "bf16x3/bf16x6 MFMA, f32 storage, f64 master",
              "mixed32": "bf16x3/bf16x6 MFMA, f32 storage, no f64 master"}
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "mixed_bf16": 2500.0}
# --single-pass: the lagged Barzilai-Borwein pair (as printed in Section 5.1)
# with eta^k and nu^k found before the row-block pass, which then writes
# X^{k+1} itself (options.fused; the forms that have it)
SINGLE_PASS = False
SINGLE_PASS_FORMS = ("fp64", "mixed32")


def form_options(precision):
    """Step-rule indexing and pass structure of a form's solves."""
    if SINGLE_PASS:
        return {"bb_index": "lagged", "fused": precision in SINGLE_PASS_FORMS}
    return {"bb_index": "standard", "fused": False}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def rho_slots(p, precision):
    """Row partials of rho written by the single-pass residual: one per
    64-column block (split bf16) or per 32 columns (float64)."""
    ncb = (p + 63) // 64
    return 2 * ncb if precision == "fp64" else ncb


def kernel_algorithmic(name, n, p, precision, fused=False):
    """Algorithmic (bytes, flops) of one launch of a kernel per iteration.

    Bytes count each operand read or written once (neighbour rows of the
    stencil count once); flops count a multiply-add as 2 and only the
    mathematical products (not the extra split-bf16 products).
    """
    npe = float(n) * p
    s = 8 if precision == "fp64" else 4
    master = precision in ("fp32", "mixed")   # float64 master iterate beside the float32 X
    if name == "grad":        # read X (the float64 master when there is one) + v, phi; write G
        return npe * ((8 if master or precision == "fp64" else 4) + s) + 16.0 * n, 14.0 * npe
    if name == "gram":        # read X, G: upper halves of S and W (W = X^T H X is symmetric)
        return 2 * npe * s, 2.0 * n * p * (p + 1)
    if name == "residual":    # read X, G, gradL^{k-1}; write gradL over G: G - X M_L
        if fused:             # + X^{k+1} and the row partials of rho
            return 5 * npe * s + 8.0 * n * rho_slots(p, precision), 2.0 * n * p * p + 4.0 * npe
        return 4 * npe * s, 2.0 * n * p * p
    if name == "update" and fused:   # the row partials of rho summed: read slots x n, write n
        return 8.0 * n * (rho_slots(p, precision) + 1), float(n) * rho_slots(p, precision)
    if name == "update":      # read X (or the master), gradL; write X (+ master), rho
        if precision == "fp64":
            by = 3 * npe * 8
        elif master:
            by = npe * (8 + 4 + 8 + 4)
        else:
            by = 3 * npe * 4
        return by + 8.0 * n, 4.0 * npe
    if name == "hartree":     # six 1D sine transforms over the grid
        return 7 * 8.0 * n, 6 * 2.0 * n * max(GRID)
    return 0.0, 0.0


def run_form(dp, x0, precision, steps, warmup, S, torch, ttk=True, starts=()):
    """Timed steps, a per-kernel profile and a time-to-KKT solve for one form."""
    dt = S.storage_dtype(precision)
    eta0 = BETA + dp.s_bound
    common = dict(variant="pcal", mult="psi_phi", eta_rule="abb", precision=precision,
                  beta=BETA, eta0=eta0, **form_options(precision))
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
        # timed: exactly `steps` iterations (plus the stop test at k = steps);
        # HIP events on the solver's stream bracket the loop
        fresh()
        t0 = time.perf_counter()
        res, _, _ = S.solve(dp, X, S.SolveOptions(**common, tol=0.0, max_iter=steps,
                                                  orth_final=False, check_every=steps,
                                                  use_graph=False),
                            workspace=ws, stream=stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms_step = res["ms_loop"] / steps
        # per-kernel averages: the same iterations with every kernel bracketed by events
        fresh()
        prof, _, _ = S.solve(dp, X, S.SolveOptions(**common, tol=0.0, max_iter=steps,
                                                   orth_final=False, check_every=steps,
                                                   use_graph=False, profile=True),
                             workspace=ws, stream=stream)
        torch.cuda.synchronize()
        prof_n = max(1, prof["prof_iters"])
        kernel_avg_ms = {k: v / prof_n for k, v in prof["kernel_ms"].items()}
        if not ttk:
            return {"iters_per_s": 1000.0 / ms_step, "ms_per_step": ms_step,
                    "timed_wall_s": wall, "kernel_avg_ms": kernel_avg_ms,
                    "kernel_sum_ms": sum(kernel_avg_ms.values())}, None
        # time to relative KKT <= TOL from X0 resident in HBM, graph-replayed loop
        sw = SWITCH_TOL if precision != "fp64" else 0.0

        x64_first = []

        def solve_to_tol():
            # a start whose final CholeskyQR2 fails (a rank-deficient iterate
            # after an unconverged run) counts as not reached
            t = time.perf_counter()
            try:
                r, x64, _ = S.solve(dp, X, S.SolveOptions(**common, tol=TOL, max_iter=MAX_ITER,
                                                          orth_final=True, check_every=50,
                                                          use_graph=True, switch_tol=sw),
                                    workspace=ws, stream=stream, want_x64=not x64_first,
                                    raise_on_error=False)
                torch.cuda.synchronize()
                if r["rc"] < 0:
                    # e.g. a rank-deficient final iterate (CholeskyQR2 fails):
                    # not reached; the iteration count and hand-over are kept,
                    # the time is the host's wall clock of the call
                    r["error"] = S.L.strerror(r["rc"])
                    r["kkt_rel"] = None
                    r["ms_loop"] = (time.perf_counter() - t) * 1000.0
                    r["ms_orth"] = 0.0
                    return r
                if not x64_first:
                    x64_first.append(x64)
                return r
            except S.StiefelError as e:
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t) * 1000.0
                return {"rc": e.code, "error": str(e), "iters": MAX_ITER, "switch_iter": -1,
                        "kkt_rel": None, "kkt_abs": None, "feas": None, "fval": None,
                        "ms_loop": ms, "ms_orth": 0.0}

        fresh()
        t0 = time.perf_counter()
        conv = solve_to_tol()
        wall_kkt = time.perf_counter() - t0
        # the same solve from other seeded starts (the iteration count is chaotic)
        more = []
        for xs in starts:
            X.copy_(torch.as_tensor(xs, device="cuda").to(dt))
            torch.cuda.synchronize()
            more.append(solve_to_tol())
    runs = [conv] + more
    x_first = x64_first[0] if x64_first else None
    ttk_all = [(r["ms_loop"] + r["ms_orth"]) / 1000.0 for r in runs]
    reached = [r["rc"] == 0 and r["kkt_rel"] is not None and r["kkt_rel"] <= TOL for r in runs]
    # a start that did not reach the tolerance counts as infinitely slow
    med = float(np.median([t if ok else np.inf for t, ok in zip(ttk_all, reached)]))
    out = {
        "iters_per_s": 1000.0 / ms_step,
        "ms_per_step": ms_step,
        "timed_wall_s": wall,
        "kernel_avg_ms": kernel_avg_ms,
        "kernel_sum_ms": sum(kernel_avg_ms.values()),
        "time_to_kkt_s": (conv["ms_loop"] + conv["ms_orth"]) / 1000.0,
        "time_to_kkt_wall_s": wall_kkt,
        "iters_to_kkt": conv["iters"],
        "switch_iter": conv["switch_iter"],
        "status": conv["rc"],
        "kkt_rel": conv["kkt_rel"],
        "kkt_abs": conv["kkt_abs"],
        "feas": conv["feas"],
        "f": conv["fval"],
        "ms_orth": conv["ms_orth"],
        "time_to_kkt_s_per_start": ttk_all,
        "iters_to_kkt_per_start": [r["iters"] for r in runs],
        "switch_iter_per_start": [r.get("switch_iter", -1) for r in runs],
        "restarted_per_start": [int(r.get("restarted", 0)) for r in runs],
        "kkt_rel_per_start": [r["kkt_rel"] for r in runs],
        "reached_per_start": reached,
        "reached": f"{sum(reached)}/{len(reached)}",
        "time_to_kkt_s_median": med if np.isfinite(med) else None,
        # the mean over the starts (None when one did not reach the tolerance)
        "time_to_kkt_s_mean": float(np.mean(ttk_all)) if all(reached) else None,
        **form_options(precision),
    }
    return out, x_first


def faster_on(base, fast):
    """Number of starts on which `fast` reached the tolerance before `base`."""
    def t(f, i):
        return f["time_to_kkt_s_per_start"][i] if f["reached_per_start"][i] else np.inf
    n = len(base["reached_per_start"])
    return sum(1 for i in range(n) if t(fast, i) < t(base, i))


KERNEL_NAMES = {"grad": "k_grad_stencil", "gram": "k_gram", "residual": "k_residual",
                "update": "k_update", "hartree": "k_dst_xy + k_dst_z"}
# the device function that does the work of each timed kernel, per form
KERNEL_BODY = {("fp64", "residual"): "body_residual", ("fp64", "gram"): "body_gram_lds",
               ("fp64", "grad"): "body_grad_line", ("fp64", "update"): "body_update",
               ("mixed", "residual"): "body_residual_bf6_lds",
               ("mixed", "gram"): "body_gram_bf3_lds", ("mixed", "grad"): "body_grad_line",
               ("mixed", "update"): "body_update",
               ("mixed32", "residual"): "body_residual_bf6_lds",
               ("mixed32", "gram"): "body_gram_bf3_lds", ("mixed32", "grad"): "body_grad_line",
               ("mixed32", "update"): "k_update_v"}
# kernels that differ from KERNEL_NAMES in one form (the 3D gradient walks
# runs of rows)
KERNEL_NAMES_FORM = {("fp64", "grad"): "k_grad_line", ("mixed", "grad"): "k_grad_line",
                     ("fp32", "grad"): "k_grad_line", ("mixed32", "grad"): "k_grad_line",
                     ("mixed32", "update"): "k_update_v"}


def body_digest(name):
    """sha256 of a device function's source text in the kernel file (from its
    definition line to the closing brace in column 0)."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_1810_03930_amd", "csrc", "stf_kernels.hip")
    with open(src) as f:
        text = f.read()
    m = re.search(r"^(__device__ __forceinline__|__global__ __launch_bounds__\(\d+\)) void "
                  + re.escape(name) + r"\(", text, re.M)
    if not m:
        return None
    end = text.find("\n}\n", m.start())
    return hashlib.sha256(text[m.start():end + 3].encode()).hexdigest()


def traffic_for(kernel, precision):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE counter
    runs, when they were taken on the kernel's current source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    body = KERNEL_BODY.get((precision, kernel))
    if not body or not os.path.exists(path):
        return None
    with open(path) as f:
        tab = json.load(f)
    ent = tab.get(f"{precision}/{kernel}")
    if not ent or ent.get("body") != body or ent.get("source_sha256") != body_digest(body):
        return None
    return ent.get("bytes_per_launch")


def roofline_for(form, precision, n, p):
    ka = {k: v for k, v in form["kernel_avg_ms"].items() if k in KERNEL_NAMES}
    name = max(ka, key=lambda k: ka[k])
    ms = ka[name]
    fused = form_options(precision)["fused"]
    by, fl = kernel_algorithmic(name, n, p, precision, fused)
    # the arithmetic that bounds each kernel: the float64 MFMA/vector peak, or
    # the split-bf16 products (3 for the Gram, 6 for the residual) at bf16 peak
    mults = {"gram": 3.0, "residual": 6.0}
    if precision == "fp64":
        t_mma = fl / (PEAK_TFLOPS["fp64"] * 1e12)
        peak_f = PEAK_TFLOPS["fp64"]
    elif precision == "fp32":
        t_mma = fl / (PEAK_TFLOPS["fp32"] * 1e12)
        peak_f = PEAK_TFLOPS["fp32"]
    else:
        t_mma = fl * mults.get(name, 0.0) / (PEAK_TFLOPS["mixed_bf16"] * 1e12)
        peak_f = PEAK_TFLOPS["mixed_bf16"] / mults.get(name, 1.0)
    t_mem = by / (HBM_PEAK_GBS * 1e9)
    traffic = None if fused else traffic_for(name, precision)
    kname = KERNEL_NAMES_FORM.get((precision, name), KERNEL_NAMES[name])
    if fused and name == "update":
        kname = "k_rho_reduce"
    common = {"kernel": kname,
              "group": name, "avg_launch_ms": ms,
              "algorithmic_bytes": by, "algorithmic_flops": fl,
              "traffic": traffic}
    if t_mma > t_mem and name in mults:
        ach = fl / (ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": ach, "peak": peak_f, "unit": "TFLOP/s",
                "frac": ach / peak_f, **common}
    ach = by / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, **common}


def cpu_baseline(prob, x0):
    """The float64 oracle, unchanged, on this host: per-iteration cost from a
    1-iteration and a 9-iteration run (the difference is 8 full iterations;
    about 10-15 s of host work in all)."""
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
    O.solve(op, x0, O.Options(max_iter=9, **opt))
    t2 = time.perf_counter()
    per_iter = ((t2 - t1) - (t1 - t0)) / 8.0
    return {"value": 1.0 / per_iter, "unit": "iters/s", "cores": int(min(cores, threads)),
            "kind": "oracle", "sample": "8 PCAL iterations of the 64^3 p=256 workload "
            f"(difference of a 9- and a 1-iteration float64 run; {t2 - t0:.1f} s total)",
            "s_per_iter": per_iter, "host_cores_visible": cores, "blas_threads": threads}


def batched_main(args, torch, S, W):
    """Config 4: 256 independent 1D Kohn-Sham problems (uneven n, p, alpha),
    batched vs one problem after another."""
    probs, x0s = W.batched_ks1d(nprob=256)
    dps = [S.DeviceProblem.from_host(p) for p in probs]

    def opts(prec, max_iter, tol, use_graph=True, check_every=50):
        out = []
        # float32 forms hand over to float64 at 1e-3: with beta up to ~6e5 the
        # split-bf16 Gram error stalls them near 1e-4
        sw = BATCH_SWITCH_TOL if (prec != "fp64" and tol > 0) else 0.0
        for prob in probs:
            b = prob.alpha * prob.p * prob.n / 8.0 + 10.0   # above the Hartree scale
            out.append(S.SolveOptions(variant="pcal", mult="psi_phi", eta_rule="abb",
                                      precision=prec, beta=b, eta0=b + prob.s_bound, tol=tol,
                                      max_iter=max_iter, orth_final=tol > 0,
                                      use_graph=use_graph, check_every=check_every,
                                      switch_tol=sw))
        return out

    stream = torch.cuda.Stream()
    out = {}
    # the batched solver has the float64, FP32 and MIXED kernel sets
    fast = "mixed" if args.fast_form == "mixed32" else args.fast_form
    for prec in ["fp64", fast]:
        dt = S.storage_dtype(prec)
        Xs = [torch.as_tensor(x0, device="cuda").to(dt).contiguous() for x0 in x0s]
        x0d = [X.clone() for X in Xs]
        ws = torch.empty(S.batched_workspace_size(dps, opts(prec, 1, 0.0)), dtype=torch.uint8,
                         device="cuda")

        def reload():
            for X, X0 in zip(Xs, x0d):
                X.copy_(X0)
            torch.cuda.synchronize()

        with torch.cuda.stream(stream):
            log(f"batched {prec}: autotune")
            budgets, _ = S.tune_batched(dps, Xs, opts(prec, 4, 0.0), iters=4, workspace=ws,
                                        stream=stream)
            reload()
            S.solve_batched(dps, Xs, opts(prec, args.warmup, 0.0, check_every=args.warmup),
                            workspace=ws, budgets=budgets, stream=stream)
            reload()
            log(f"batched {prec}: {args.steps} timed iterations, budgets {budgets}")
            res, rc, msi = S.solve_batched(dps, Xs, opts(prec, args.steps, 0.0,
                                                         check_every=args.steps),
                                           workspace=ws, budgets=budgets, stream=stream)
            torch.cuda.synchronize()
            agg = len(probs) * 1000.0 / msi
            # the same iterations one problem after another (single-problem solver)
            log(f"batched {prec}: serial reference")
            reload()
            t_serial = 0.0
            for dp, X, o in zip(dps, Xs, opts(prec, args.steps, 0.0, check_every=args.steps)):
                r, _, _ = S.solve(dp, X, o, stream=stream)
                t_serial += r["ms_loop"]
            torch.cuda.synchronize()
            agg_serial = len(probs) * args.steps * 1000.0 / t_serial
            # every problem to relative KKT <= TOL (or MAX_ITER)
            reload()
            log(f"batched {prec}: time to KKT")
            rk, rck, _ = S.solve_batched(dps, Xs, opts(prec, MAX_ITER, TOL), workspace=ws,
                                         budgets=budgets, stream=stream)
            torch.cuda.synchronize()
            # the same solves one problem after another (the single-problem
            # solver, one graph-replayed loop per problem)
            reload()
            log(f"batched {prec}: time to KKT one problem after another")
            t_serial_kkt = 0.0
            conv_serial = 0
            for dp, X, o in zip(dps, Xs, opts(prec, MAX_ITER, TOL)):
                r, _, _ = S.solve(dp, X, o, stream=stream, raise_on_error=False)
                t_serial_kkt += r["ms_loop"] + r["ms_orth"]
                conv_serial += int(r["rc"] == 0)
            torch.cuda.synchronize()
        conv = sum(1 for r in rk if r["status"] == 0)
        out[prec] = {"aggregate_iters_per_s": agg, "ms_per_batch_iter": msi,
                     "serial_aggregate_iters_per_s": agg_serial,
                     "speedup_vs_serial": agg / agg_serial, "budgets": list(budgets),
                     "time_to_kkt_s": (rk[0]["ms_loop"] + rk[0]["ms_orth"]) / 1000.0,
                     "serial_time_to_kkt_s": t_serial_kkt / 1000.0,
                     "serial_converged": conv_serial,
                     "converged": conv, "max_iters": max(r["iters"] for r in rk),
                     "switched": sum(1 for r in rk if r["switch_iter"] >= 0),
                     "worst_kkt_rel": max(r["kkt_rel"] for r in rk)}
        log(f"batched {prec}: {json.dumps(out[prec])}")
        del Xs, x0d, ws
    fast_form = fast
    fast = out[fast_form]
    line = {
        "metric": "batched PCAL aggregate iters/s, 256 x 1D KS (uneven n, p, alpha)",
        "value": fast["aggregate_iters_per_s"], "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": fast["ms_per_batch_iter"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": FORM_DTYPE[fast_form],
        "data": "synthetic",
        "config": {"workload": "256 x 1D Kohn-Sham-shaped PCAL, n~U[1000,20000], "
                               "p~U[8,128], alpha~U[0.5,2], beta = alpha p n / 8 + 10",
                   "nprob": len(probs), "sum_np": int(sum(p.n * p.p for p in probs))},
        "forms": out,
    }
    print(json.dumps(line), flush=True)


def _timed_and_profiled(dp, x0, opts, steps, warmup, S, torch):
    """ms per iteration over exactly `steps` iterations (device events) and the
    per-group averages of a second, profiled pass."""
    stream = torch.cuda.Stream()
    ws = S.alloc_workspace(dp, opts)
    X = torch.empty((dp.n, dp.p), dtype=torch.float64, device="cuda")
    x0d = torch.as_tensor(x0, device="cuda")
    base = {k: getattr(opts, k) for k in opts.__dataclass_fields__}
    with torch.cuda.stream(stream):
        X.copy_(x0d)
        torch.cuda.synchronize()
        S.solve(dp, X, S.SolveOptions(**{**base, "tol": 0.0, "max_iter": max(1, warmup),
                                        "orth_final": False, "check_every": max(1, warmup),
                                        "use_graph": False}), workspace=ws, stream=stream)
        X.copy_(x0d)
        torch.cuda.synchronize()
        r, _, _ = S.solve(dp, X, S.SolveOptions(**{**base, "tol": 0.0, "max_iter": steps,
                                                   "orth_final": False, "check_every": steps,
                                                   "use_graph": False}),
                          workspace=ws, stream=stream)
        X.copy_(x0d)
        torch.cuda.synchronize()
        pr, _, _ = S.solve(dp, X, S.SolveOptions(**{**base, "tol": 0.0, "max_iter": steps,
                                                    "orth_final": False, "check_every": steps,
                                                    "use_graph": False, "profile": True}),
                           workspace=ws, stream=stream)
        torch.cuda.synchronize()
        # to the tolerance, graph-replayed
        X.copy_(x0d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            c, _, _ = S.solve(dp, X, opts, workspace=ws, stream=stream)
        except S.StiefelError as e:
            c = {"rc": e.code, "iters": None, "kkt_rel": None, "fval": None, "feas": None,
                 "ms_loop": None, "ms_orth": None}
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    n_it = max(1, pr["prof_iters"])
    km = {k: v / n_it for k, v in pr["kernel_ms"].items()}
    return {"ms_per_iter": r["ms_loop"] / steps,
            "func_ms": km["hartree"] + km["grad"],
            "blas3_ms": km["gram"] + km["stage1"] + km["residual"] + km["stage2"],
            "orth_ms": km["update"],
            "kernel_avg_ms": km,
            "to_tol": {"rc": c["rc"], "iters": c["iters"], "kkt_rel": c["kkt_rel"],
                       "f": c["fval"], "feas": c["feas"], "ms_loop": c["ms_loop"],
                       "ms_orth": c["ms_orth"], "wall_s": wall}}


def parallel_main(args, torch, S, W):
    """The workloads of the parallel experiments of Section 5.5 (Figs. 7-11):
    Problem 1 with the block-diagonal 5 x 5 operator, Problem 2 with the
    tridiagonal A and a uniform random G, Problem 6 (exchange term), n = 10000,
    PCAL (beta = 1) against MOptQR with the Cholesky-QR retraction, both float64
    with ABB steps, max 1000 iterations, tol 1e-8.  Per iteration the time is
    split as in the paper: Func (Hartree + gradient), BLAS3 (Grams, p x p
    stages, the row-block product) and Orth (the PCAL update, or MOptQR's
    retraction: V, V^T V, Cholesky, inverse, V R^{-1})."""
    ps = [int(v) for v in args.parallel_p.split(",")]
    n = 10000
    rows = []
    for name, gen in [("P1", W.ks1d_block), ("P2", W.ocqp_tridiag), ("P6", W.ks_exchange)]:
        for p in ps:
            if name == "P6" and p != 1000 and not args.parallel_all:
                continue
            prob, x0 = gen(n=n, p=p)
            dp = S.DeviceProblem.from_host(prob)
            for solver in ["pcal", "moptqr"]:
                # PCAL takes the paper's beta = 1; where that diverges (the
                # p-th eigenvalue of the operator is at or above beta), once
                # more with beta above the spectrum bound
                betas = [1.0, prob.s_bound + 1.0] if solver == "pcal" else [0.0]
                for beta in betas:
                    opts = S.SolveOptions(variant=solver,
                                          mult="psi_phi" if solver == "pcal" else "psi",
                                          eta_rule="abb", precision="fp64", beta=beta,
                                          eta0=beta + prob.s_bound, tol=1e-8, max_iter=1000,
                                          orth_final=True, check_every=50, use_graph=True)
                    log(f"parallel {name} n={n} p={p} {solver} beta={beta}")
                    r = _timed_and_profiled(dp, x0, opts, args.steps, args.warmup, S, torch)
                    r.update({"problem": name, "n": n, "p": p, "solver": solver, "beta": beta})
                    log(json.dumps(r))
                    rows.append(r)
                    if r["to_tol"]["rc"] != -2:
                        break
            del dp
            torch.cuda.empty_cache()
    print(json.dumps({"metric": "Section 5.5 workloads: PCAL vs MOptQR, float64, one GPU",
                      "unit": "ms/iteration", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "data": "synthetic", "rows": rows}), flush=True)


def dense_main(args, torch, S, W):
    """The dense Rayleigh-Ritz workload: A = (B + B^T)/(2 sqrt n) + 4I in
    float32, B ~ N(0,1), n = 32768, p = 512.  Forms: float64 (A widened
    exactly, float64 MFMA products), float32 MFMA, and the split-bf16 form
    (A X as three bf16 MFMA products with float32 accumulation, split-bf16
    Grams) handing over to float64 at 1e-4.  Per-iteration costs, the dense
    product's roofline, and time to relative KKT 1e-6."""
    n, p = args.dense_n, args.dense_p
    log(f"generating the dense workload n={n} p={p} (seeded)")
    prob, x0 = W.dense_quadratic(n=n, p=p, dtype=np.float32)
    dp = S.DeviceProblem.from_host(prob)
    beta = prob.s_bound + 0.1          # above the p-th eigenvalue (positive definite A)
    stream = torch.cuda.Stream()
    out = {}
    for prec in args.dense_forms.split(","):
        sw = 1e-4 if prec in ("mixed", "mixed32", "fp32") else 0.0
        opts = S.SolveOptions(variant="pcal", mult="psi_phi", eta_rule="abb", precision=prec,
                              beta=beta, eta0=beta + prob.s_bound, tol=TOL,
                              max_iter=args.dense_max_iter, orth_final=True, check_every=20,
                              use_graph=True, switch_tol=sw)
        dt = S.storage_dtype(prec)
        ws = S.alloc_workspace(dp, opts)
        X = torch.empty((n, p), dtype=dt, device="cuda")
        x0d = torch.as_tensor(x0, device="cuda").to(dt)
        base = {k: getattr(opts, k) for k in opts.__dataclass_fields__}
        with torch.cuda.stream(stream):
            X.copy_(x0d)
            torch.cuda.synchronize()
            S.solve(dp, X, S.SolveOptions(**{**base, "tol": 0.0, "max_iter": args.warmup,
                                            "orth_final": False, "use_graph": False,
                                            "check_every": max(1, args.warmup)}),
                    workspace=ws, stream=stream)
            X.copy_(x0d)
            torch.cuda.synchronize()
            pr, _, _ = S.solve(dp, X, S.SolveOptions(**{**base, "tol": 0.0,
                                                        "max_iter": args.steps,
                                                        "orth_final": False,
                                                        "use_graph": False, "profile": True,
                                                        "check_every": args.steps}),
                               workspace=ws, stream=stream)
            X.copy_(x0d)
            torch.cuda.synchronize()
            r, _, _ = S.solve(dp, X, S.SolveOptions(**{**base, "tol": 0.0,
                                                       "max_iter": args.steps,
                                                       "orth_final": False, "use_graph": False,
                                                       "check_every": args.steps}),
                              workspace=ws, stream=stream)
            X.copy_(x0d)
            torch.cuda.synchronize()
            log(f"dense {prec}: solve to {TOL}")
            try:
                c, _, _ = S.solve(dp, X, opts, workspace=ws, stream=stream)
            except S.StiefelError as e:
                c = {"rc": e.code, "iters": None, "kkt_rel": None, "fval": None,
                     "ms_loop": None, "ms_orth": None, "switch_iter": None}
            torch.cuda.synchronize()
        n_it = max(1, pr["prof_iters"])
        km = {k: v / n_it for k, v in pr["kernel_ms"].items()}
        flops = 2.0 * n * n * p
        if prec == "fp64":
            peak, unit_peak = PEAK_TFLOPS["fp64"], "fp64"
        elif prec == "fp32":
            peak, unit_peak = PEAK_TFLOPS["fp32"], "fp32"
        else:
            peak, unit_peak = PEAK_TFLOPS["mixed_bf16"] / 3.0, "bf16 peak / 3 products"
        ach = flops / (km["grad"] * 1e-3) / 1e12
        out[prec] = {"ms_per_iter": r["ms_loop"] / args.steps, "kernel_avg_ms": km,
                     "dense_product": {"achieved_tflops": ach, "peak_tflops": peak,
                                       "peak_of": unit_peak, "frac": ach / peak},
                     "to_tol": {"rc": c["rc"], "iters": c["iters"], "kkt_rel": c["kkt_rel"],
                                "f": c["fval"], "switch_iter": c.get("switch_iter"),
                                "s": None if c["ms_loop"] is None
                                else (c["ms_loop"] + c["ms_orth"]) / 1000.0}}
        log(f"dense {prec}: {json.dumps(out[prec])}")
        del ws, X, x0d
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "dense Rayleigh-Ritz PCAL, n=%d p=%d: ms/iteration and time to "
                      "relative KKT 1e-6 per form" % (n, p), "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "data": "synthetic", "forms": out}), flush=True)


def sweep_main(args, torch, S, W):
    """The parameter studies of Section 5.3 on GPU (Problems 1-4 at n = 1000,
    p = 20; Problem 1 with the 3D Kohn-Sham operator on a 10^3 grid): step-size rules
    (Fig. 1) at beta = s + 0.1, beta in {0, 0.01s, 0.1s, s + 0.1, 10s + 1}
    with ABB steps (Figs. 2-3), and the closed-form multipliers against dual
    ascent (PLAM-DA / PCAL-DA, Fig. 4).  Iterations and time to relative KKT
    1e-8 (max 3000), float64."""
    probs = {"P1": W.ks3d(grid=(10, 10, 10), p=20)[:2],
             "P2": W.ocqp_dense(n=1000, p=20),
             "P3": W.ocqp_dense(n=1000, p=20, kappa=0.0),
             "P4": W.qap_dense(n=1000, p=20)}
    stream = torch.cuda.Stream()
    rows = []
    for pname, (prob, x0) in probs.items():
        if pname == "P3":
            prob.Glin = None
        dp = S.DeviceProblem.from_host(prob)
        s = prob.s_bound
        runs = []
        for var in ["plam", "pcal"]:
            for rule in ["const", "diff", "bb1", "bb2", "abb"]:
                runs.append(("eta", var, "psi_phi" if var == "pcal" else "psi", rule, s + 0.1))
            for bname, b in [("0", 0.0), ("0.01s", 0.01 * s), ("0.1s", 0.1 * s),
                             ("s+0.1", s + 0.1), ("10s+1", 10 * s + 1)]:
                runs.append(("beta=" + bname, var, "psi_phi" if var == "pcal" else "psi",
                             "abb", b))
            b = s + 0.1 if var == "plam" else 1.0
            runs.append(("closed_form", var, "psi_phi" if var == "pcal" else "psi", "abb", b))
            runs.append(("dual_ascent", var, "dual", "abb", b))
        for study, var, mult, rule, beta in runs:
            eta0 = beta + s
            o = S.SolveOptions(variant=var, mult=mult, eta_rule=rule, precision="fp64",
                               beta=beta, eta0=eta0, eta_const=eta0, tol=1e-8, max_iter=3000,
                               orth_final=True, check_every=100, use_graph=True)
            X = torch.as_tensor(x0, device="cuda").contiguous()
            with torch.cuda.stream(stream):
                try:
                    r, _, _ = S.solve(dp, X, o, stream=stream, raise_on_error=False)
                except S.StiefelError as e:
                    r = {"rc": e.code, "iters": None, "kkt_rel": None, "fval": None,
                         "ms_loop": None, "ms_orth": None}
            torch.cuda.synchronize()
            rows.append({"problem": pname, "study": study, "variant": var, "mult": mult,
                         "eta_rule": rule, "beta": beta, "rc": r["rc"], "iters": r["iters"],
                         "kkt_rel": r["kkt_rel"], "f": r["fval"], "ms": r["ms_loop"]})
            log(json.dumps(rows[-1]))
    print(json.dumps({"metric": "Section 5.3 parameter studies on GPU (iterations to 1e-8)",
                      "n_gpus": 1, "data": "synthetic", "rows": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--fast-form", default="mixed32", choices=["fp32", "mixed", "mixed32"])
    ap.add_argument("--extra-forms", default="",
                    help="comma-separated further forms to measure beside fp64 and the fast form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--starts", type=int, default=15,
                    help="seeded starting points of the time-to-KKT solves (the median is reported)")
    ap.add_argument("--skip-ttk", action="store_true",
                    help="skip the time-to-KKT solves (short runs under hardware counters)")
    ap.add_argument("--batched", action="store_true",
                    help="measure the batched solver on the 256-problem 1D workload instead")
    ap.add_argument("--parallel", action="store_true",
                    help="measure the Section 5.5 workloads (PCAL vs MOptQR, n = 10000)")
    ap.add_argument("--parallel-p", default="1000",
                    help="comma-separated p of --parallel (the paper: 500,1000,1500,2000,2500)")
    ap.add_argument("--parallel-all", action="store_true",
                    help="run Problem 6 at every p too (the paper: p = 1000 only)")
    ap.add_argument("--dense", action="store_true",
                    help="measure the dense Rayleigh-Ritz workload (n = 32768, p = 512)")
    ap.add_argument("--dense-n", type=int, default=32768)
    ap.add_argument("--dense-p", type=int, default=512)
    ap.add_argument("--dense-forms", default="fp64,fp32,mixed")
    ap.add_argument("--dense-max-iter", type=int, default=3000)
    ap.add_argument("--sweep", action="store_true",
                    help="run the Section 5.3 step-size / beta / dual-ascent studies")
    ap.add_argument("--single-pass", action="store_true",
                    help="lagged Barzilai-Borwein pair and the single-pass iteration "
                         "(options.fused) in the forms that have it (fp64, mixed32)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="first run a plain 512 MiB device copy 3 times: the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    global SINGLE_PASS
    SINGLE_PASS = bool(args.single_pass)
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
    if args.copy_ref:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.batched:
        batched_main(args, torch, S, W)
        return
    if args.parallel:
        parallel_main(args, torch, S, W)
        return
    if args.sweep:
        sweep_main(args, torch, S, W)
        return
    if args.dense:
        dense_main(args, torch, S, W)
        return
    log("generating the 64^3 p=256 workload (seeded)")
    prob, x0, _ = W.ks3d(grid=GRID, p=P, alpha=ALPHA)
    dp = S.DeviceProblem.from_host(prob)
    starts = [W.alternate_start(5, prob.n, P, s) for s in range(1, args.starts)]
    forms = {}
    finals = {}
    extra = [f for f in args.extra_forms.split(",") if f and f not in ("fp64", args.fast_form)]
    for prec in ["fp64", args.fast_form] + extra:
        log(f"form {prec}: {args.warmup} warmup + {args.steps} timed steps, then time-to-KKT")
        forms[prec], finals[prec] = run_form(dp, x0, prec, args.steps, args.warmup, S, torch,
                                             ttk=not args.skip_ttk, starts=starts)
        log(f"form {prec}: {json.dumps(forms[prec])}")
    fast = forms[args.fast_form]
    base = forms["fp64"]
    # per-result error of each reduced-precision form against the float64 form
    # (seed 0's returned points): objective, KKT and feasibility, and the
    # distance of the subspaces ||X X^T - Y Y^T||_F (X* is unique only up to
    # X* Q), via ||X^T X||^2 + ||Y^T Y||^2 - 2 ||X^T Y||^2
    errors = {}
    if finals.get("fp64") is not None:
        Y = finals["fp64"]
        for prec, Xf in finals.items():
            if prec == "fp64" or Xf is None:
                continue
            a = (torch.linalg.norm(Xf.T @ Xf) ** 2 + torch.linalg.norm(Y.T @ Y) ** 2
                 - 2 * torch.linalg.norm(Xf.T @ Y) ** 2).item()
            fb, ff = base["f"], forms[prec]["f"]
            errors[prec] = {
                "f_rel_diff": None if (fb is None or ff is None) else abs(ff - fb) / abs(fb),
                "kkt_rel": forms[prec]["kkt_rel"], "kkt_rel_fp64": base["kkt_rel"],
                "feas": forms[prec]["feas"], "feas_fp64": base["feas"],
                "projector_distance": float(np.sqrt(max(a, 0.0)))}
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
        "dtype": FORM_DTYPE[args.fast_form],
        "data": "synthetic",
        "config": {"workload": "3D Kohn-Sham-shaped PCAL, 7-point Dirichlet Laplacian on a "
                               "64^3 grid + Diag(V), V~U(0,1), alpha=1, beta=4, ABB steps",
                   "n": prob.n, "p": P, "grid": list(GRID), "tol_rel_kkt": TOL,
                   "fast_form": args.fast_form, "switch_tol": SWITCH_TOL,
                   "bb_index": form_options(args.fast_form)["bb_index"],
                   "single_pass": form_options(args.fast_form)["fused"]},
        "time_to_kkt_s": None if args.skip_ttk else
        {"fp64": base["time_to_kkt_s"], args.fast_form: fast["time_to_kkt_s"]},
        "time_to_kkt_s_median": None if args.skip_ttk else
        {**{f: forms[f]["time_to_kkt_s_median"] for f in forms}, "starts": args.starts},
        # seed 0 alone: only when both forms reached the tolerance from it
        "speedup_time_to_kkt": None if (args.skip_ttk or not base["reached_per_start"][0]
                                        or not fast["reached_per_start"][0]) else
        base["time_to_kkt_s"] / fast["time_to_kkt_s"],
        "speedup_time_to_kkt_median": None if (args.skip_ttk or not fast["time_to_kkt_s_median"]
                                               or not base["time_to_kkt_s_median"]) else
        base["time_to_kkt_s_median"] / fast["time_to_kkt_s_median"],
        "reached": None if args.skip_ttk else {f: forms[f]["reached"] for f in forms},
        "time_to_kkt_s_mean": None if args.skip_ttk else
        {f: forms[f]["time_to_kkt_s_mean"] for f in forms},
        # starts (of the same seeded set) on which the fast form reaches the
        # tolerance sooner than FP64 (an unreached start counts as infinitely slow)
        "faster_on_starts": None if args.skip_ttk else
        f"{faster_on(base, fast)}/{len(base['reached_per_start'])}",
        "iters_per_s": {f: forms[f]["iters_per_s"] for f in forms},
        "result_error_vs_fp64": errors,
        "forms": forms,
        "roofline": roof,
        "roofline_fp64": roof64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
