#!/usr/bin/env python3
"""Headline benchmark: solves/s of 128^3 anisotropic Helmholtz to 1e-8 relative
error, FP32-mixed batched solver vs the plain FP64 solver, with p50/p99 latency.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--nrhs B] [--n 128]

Workload (helmholtz128): grid 128^3 on [-1,1]^3, omega = 8 pi (8 wavelengths
across the box), eps^{-1}(x) = I + b(x)(A + 0.05 i I) with a seeded symmetric
A of norm 0.5 and the C-infinity bump b of radius 0.8, plane waves along B
seeded directions (gradient of exp(i omega d.x) as incident field).
A step is one batched mixed-precision solve of the B right-hand sides to a
true relative residual of 1e-9 (error <= 1e-8); inputs are resident in HBM
before the timed region.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MI355X_HBM_PEAK_GBS = 8000.0
METRIC = "solves/s to 1e-8 rel err (128³ Helmholtz), mixed vs FP64; p50/p99 latency"


def pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def cpu_baseline(n: int, omega: float, matvecs_per_solve: float, budget_s: float = 30.0):
    """The oracle (NumPy FP64, window FFT route) timed on the host: one plan
    setup and one matvec at the benchmark's grid, scaled to solves/s with the
    GPU FP64 solver's matvec count."""
    from oracle import operator as op
    from vie_inputs import generators as gen
    prob = gen.helmholtz_problem(n, omega, "helmholtz128", nrhs=1)
    t0 = time.perf_counter()
    A = op.Operator(prob.kind, prob.coef, prob.omega)
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    A.apply(prob.inc[0])
    mv = time.perf_counter() - t0
    solve_s = mv * matvecs_per_solve
    from oracle import tables as tb
    return {"value": 1.0 / solve_s, "unit": "solves/s", "cores": tb.WORKERS, "kind": "oracle",
            "sample": (f"one FP64 matvec of the oracle at {n}^3 ({mv:.2f} s; scipy.fft with "
                       f"{tb.WORKERS} workers, the rest single-threaded numpy; table setup {setup:.1f} s "
                       f"not counted) x {matvecs_per_solve:.1f} matvecs per solve (the GPU FP64 "
                       f"GMRES count for the same right-hand sides)"),
            "matvec_s": mv, "setup_s": setup}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--nrhs", type=int, default=8, help="right-hand sides per batched step")
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--restart", type=int, default=40)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--latency-solves", type=int, default=8, help="single-RHS mixed solves for p50/p99")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(right-hand sides and requests would shard across GPUs with no exchange).",
              file=sys.stderr)
        return 2

    import torch
    from paper_1805_04791_amd import vie
    from vie_inputs import generators as gen

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    n, B = args.n, args.nrhs
    omega = 8.0 * math.pi * n / 128.0 if n != 128 else 8.0 * math.pi
    prob = gen.helmholtz_problem(n, omega, "helmholtz128", nrhs=B)
    dev = torch.device("cuda:0")
    inc = torch.from_numpy(prob.inc).to(dev)
    torch.cuda.synchronize()

    plan = vie.Plan(vie.HELMHOLTZ, prob.coef, omega=omega, precision=vie.PREC_MIXED, max_rhs=B)
    print(f"[bench] plan ready: n={n} nrhs={B} omega={omega:.4f} "
          f"max||H||={plan.info()['max_contrast_norm']:.3f}", file=sys.stderr, flush=True)

    def solve(x_inc, fp64=False):
        return plan.solve(x_inc, tol=args.tol, restart=args.restart, fp64=fp64, want_field=False)

    for _ in range(args.warmup):
        solve(inc)
    torch.cuda.synchronize()

    # ---- timed region: K batched mixed solves, kernels timed with HIP events
    plan.profile(True)
    step_s, stats_all = [], []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for k in range(args.steps):
        t0 = time.perf_counter()
        d_mixed, _, st, rc = solve(inc)
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - t0)
        stats_all.extend(st)
        print(f"[bench] step {k}: {step_s[-1]*1e3:.1f} ms, iters {[s['iters'] for s in st]}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    prof = plan.profile_read()
    plan.profile(False)
    solves = args.steps * B
    value = solves / total

    # ---- plain FP64 GPU solver on the same batch
    fp64 = {}
    if not args.no_fp64 and args.fp64_steps > 0:
        ts = []
        for k in range(args.fp64_steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            d64, _, st64, _ = solve(inc, fp64=True)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        err = float(torch.linalg.vector_norm(d_mixed - d64) / torch.linalg.vector_norm(d64))
        fp64 = {"fp64_solves_per_s": B * len(ts) / sum(ts),
                "fp64_ms_per_step": 1e3 * sum(ts) / len(ts),
                "fp64_matvecs_per_solve": float(np.mean([s["matvecs_fp64"] for s in st64])),
                "mixed_vs_fp64_rel_diff": err}

    # ---- single right-hand-side latency
    lat = []
    for k in range(args.latency_solves):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solve(inc[k % B:k % B + 1])
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)

    # ---- roofline of the dominant kernel family (HIP events, algorithmic bytes)
    fam, (ms, cnt, by) = max(prof.items(), key=lambda kv: kv[1][0])
    achieved = by / (ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": fam, "achieved": achieved, "peak": MI355X_HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / MI355X_HBM_PEAK_GBS, "traffic": None,
            "avg_launch_us": 1e3 * ms / cnt, "bytes_per_launch": by / cnt}
    breakdown = {k: {"ms": v[0], "launches": v[1], "GB/s": v[2] / (v[0] * 1e-3) / 1e9 if v[0] > 0 else None}
                 for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}

    cpu = None
    if not args.no_cpu_baseline:
        mv = fp64.get("fp64_matvecs_per_solve") or float(np.mean([s["matvecs_fp32"] + s["matvecs_fp64"]
                                                                  for s in stats_all]))
        print("[bench] timing the CPU oracle ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(n, omega, mv)

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * total / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64 FFT apply + c128 Krylov (mixed)",
        "data": "synthetic",
        "config": {"workload": f"helmholtz{n}: anisotropic Helmholtz {n}^3, omega={omega:.6g}, "
                               f"eps^-1 = I + b(x)(A + 0.05i I), {B} seeded plane waves per step",
                   "n": n, "omega": omega, "nrhs_per_step": B, "tol_true_residual": args.tol,
                   "restart": args.restart, "solver": "GMRES + FP64 iterative refinement"},
        "latency_ms": {"batch_p50": 1e3 * pct(step_s, 50), "batch_p99": 1e3 * pct(step_s, 99),
                       "single_p50": 1e3 * pct(lat, 50) if lat else None,
                       "single_p99": 1e3 * pct(lat, 99) if lat else None},
        "iters_per_solve": float(np.mean([s["iters"] for s in stats_all])),
        "matvecs_fp32_per_solve": float(np.mean([s["matvecs_fp32"] for s in stats_all])),
        "matvecs_fp64_per_solve": float(np.mean([s["matvecs_fp64"] for s in stats_all])),
        "max_rel_residual": float(max(s["rel_residual"] for s in stats_all)),
        **fp64,
        "roofline": roof,
        "kernels": breakdown,
        "cpu_baseline": cpu,
    }
    if fp64:
        out["speedup_mixed_vs_fp64"] = value / fp64["fp64_solves_per_s"]
    print(json.dumps(out), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
