#!/usr/bin/env python3
"""Headline benchmark: solves/s of 128^3 anisotropic Helmholtz to 1e-8 relative
error, FP32-mixed batched solver vs the plain FP64 solver, with p50/p99 latency.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--nrhs B] [--n 128] [--workload NAME]

Workload (helmholtz128): grid 128^3 on [-1,1]^3, omega = 8 pi (8 wavelengths
across the box), eps^{-1}(x) = I + b(x)(A + 0.05 i I) with a seeded symmetric
A of norm 0.5 and the C-infinity bump b of radius 0.8, plane waves along B
seeded directions (gradient of exp(i omega d.x) as incident field).
A step is one batched mixed-precision solve of the B right-hand sides to a
true relative residual of 1e-9 (error <= 1e-8); inputs are resident in HBM
before the timed region.  Prints one JSON line.

--workload measures the other configurations instead (same JSON layout):
  laplace32    anisotropic Laplace 32^3, eps = I + b A, E0 = z; FP64 to 1e-10
  helmholtz64  anisotropic Helmholtz 64^3, omega = 4 pi; FP64 to 1e-10
  maxwell128   full Maxwell 128^3 (eps and mu), omega = 8 pi; mixed to 1e-9
  batched96    Helmholtz 96^3, omega = 6 pi, 64 plane waves per step; mixed to 1e-9
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
# Vector ALU peak reachable by this library: 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops (FMA) x 2.4 GHz.  FP64 and FP32 alike: the published 157.3 TFLOP/s
# FP32 figure counts packed (two-per-lane) FP32 instructions, which the
# library is compiled without.
MI355X_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
METRIC = "solves/s to 1e-8 rel err (128³ Helmholtz), mixed vs FP64; p50/p99 latency"
# name: (right-hand sides per step, true relative residual, the solver `value` reports)
WORKLOADS = {"helmholtz128": (8, 1e-9, "mixed"), "laplace32": (1, 1e-10, "fp64"),
             "helmholtz64": (8, 1e-10, "fp64"), "maxwell128": (8, 1e-9, "mixed"),
             "batched96": (64, 1e-9, "mixed")}


def pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def make_problem(workload: str, n: int, nrhs: int):
    from vie_inputs import generators as gen
    if workload == "helmholtz128":
        omega = 8.0 * math.pi * n / 128.0 if n != 128 else 8.0 * math.pi
        return gen.helmholtz_problem(n, omega, "helmholtz128", nrhs=nrhs)
    return gen.config_problem(workload, nrhs=nrhs)


def cpu_baseline(workload: str, n: int, matvecs_per_solve: float):
    """The oracle (NumPy FP64, window FFT route) timed on the host: one plan
    setup and one matvec at the benchmark's grid, scaled to solves/s with the
    GPU FP64 solver's matvec count."""
    from oracle import operator as op
    prob = make_problem(workload, n, 1)
    t0 = time.perf_counter()
    A = op.Operator(prob.kind, prob.coef, prob.omega, mu=prob.mu)
    setup = time.perf_counter() - t0
    from oracle import tables as tb
    t0 = time.perf_counter()
    A.apply(prob.inc[0])
    mv = time.perf_counter() - t0
    # the same matvec with one FFT worker
    workers = tb.WORKERS
    tb.WORKERS = 1
    try:
        t0 = time.perf_counter()
        A.apply(prob.inc[0])
        mv1 = time.perf_counter() - t0
    finally:
        tb.WORKERS = workers
    solve_s = mv * matvecs_per_solve
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return {"value": 1.0 / solve_s, "unit": "solves/s", "cores": workers, "kind": "oracle",
            "sample": (f"one FP64 matvec of the oracle at {prob.n}^3 ({mv:.2f} s; scipy.fft with "
                       f"{workers} workers, the rest single-threaded numpy; table setup {setup:.1f} s "
                       f"not counted) x {matvecs_per_solve:.1f} matvecs per solve (the GPU FP64 "
                       f"GMRES count for the same right-hand sides)"),
            "matvec_s": mv, "matvec_s_1_worker": mv1, "value_1_worker": 1.0 / (mv1 * matvecs_per_solve),
            "setup_s": setup, "cpu_model": model}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="helmholtz128")
    ap.add_argument("--n", type=int, default=128, help="grid of the helmholtz128 workload")
    ap.add_argument("--nrhs", type=int, default=0, help="right-hand sides per batched step (0: the workload's)")
    ap.add_argument("--tol", type=float, default=0.0, help="true relative residual (0: the workload's)")
    ap.add_argument("--restart", type=int, default=40)
    ap.add_argument("--inner-tol", type=float, default=0.0,
                    help="relative residual reduction of each FP32 inner cycle (0: the library's, 1e-5)")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--latency-solves", type=int, default=20, help="single-RHS mixed solves for p50/p99")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-post", action="store_true", help="skip timing the post-processing calls")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run a plain fp32 copy kernel (x * 1.0) over this many MiB, three times, "
                         "as the reference for hardware byte counters")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path "
              "(right-hand sides and requests would shard across GPUs with no exchange).",
              file=sys.stderr)
        return 2

    import torch
    from paper_1805_04791_amd import vie
    from vie_inputs import generators as gen

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.calibrate_copy_mib > 0:
        src = torch.ones(args.calibrate_copy_mib * 2 ** 18, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        print(f"[bench] calibration copy: {args.calibrate_copy_mib} MiB read and written, 3 times",
              file=sys.stderr, flush=True)
    wl = args.workload
    B = args.nrhs or WORKLOADS[wl][0]
    tol = args.tol or WORKLOADS[wl][1]
    primary_fp64 = WORKLOADS[wl][2] == "fp64"
    prob = make_problem(wl, args.n, B)
    n, omega = prob.n, prob.omega
    dev = torch.device("cuda:0")
    inc = torch.from_numpy(prob.inc).to(dev)
    torch.cuda.synchronize()

    plan = vie.Plan(prob.kind, prob.coef, omega=omega, mu=prob.mu, precision=vie.PREC_MIXED, max_rhs=B)
    print(f"[bench] plan ready: {wl} n={n} nrhs={B} omega={omega:.4f} "
          f"max||H||={plan.info()['max_contrast_norm']:.3f}", file=sys.stderr, flush=True)

    def solve(x_inc, fp64=primary_fp64):
        return plan.solve(x_inc, tol=tol, restart=args.restart, inner_tol=args.inner_tol, fp64=fp64,
                          want_field=False)

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

    # ---- the other solver on the same batch: plain FP64 (or mixed, when the
    # workload's own figure is the FP64 solver's)
    fp64 = {}
    if not args.no_fp64 and args.fp64_steps > 0:
        ts = []
        for k in range(args.fp64_steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            d64, _, st64, _ = solve(inc, fp64=not primary_fp64)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        err = float(torch.linalg.vector_norm(d_mixed - d64) / torch.linalg.vector_norm(d64))
        other = "mixed" if primary_fp64 else "fp64"
        fp64 = {f"{other}_solves_per_s": B * len(ts) / sum(ts),
                f"{other}_ms_per_step": 1e3 * sum(ts) / len(ts),
                f"{other}_matvecs_per_solve": float(np.mean([s["matvecs_fp64"] + s["matvecs_fp32"] for s in st64])),
                "mixed_vs_fp64_rel_diff": err}

    # ---- single right-hand-side latency (one untimed solve first: the first
    # single-RHS apply tunes its tiles and captures its graphs)
    lat = []
    if args.latency_solves > 0:
        solve(inc[0:1])
        torch.cuda.synchronize()
    for k in range(args.latency_solves):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solve(inc[k % B:k % B + 1])
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)

    # ---- roofline of the dominant kernel family (HIP events, algorithmic
    # bytes and nominal flops): ALU-bound when its arithmetic intensity is
    # above the ridge point peak_flops / peak_bandwidth
    fam, (ms, cnt, by, fl) = max(prof.items(), key=lambda kv: kv[1][0])
    ridge = MI355X_VALU_PEAK_TFLOPS * 1e12 / (MI355X_HBM_PEAK_GBS * 1e9)
    alu = fl / by > ridge
    # HBM bytes per launch from the committed counter summary of this kernel
    # and workload, if the device sources are unchanged since it was taken
    from paper_1805_04791_amd import profiling
    tag = f"helmholtz{n}" if wl == "helmholtz128" else wl
    tr = profiling.read_traffic(os.path.join(ROOT, "profiles", f"{fam}.{tag}.traffic.md"))
    digest = profiling.source_digest()
    traffic = tr[0] if tr is not None and tr[2] == digest else None
    if alu:
        achieved, peak, unit = fl / (ms * 1e-3) / 1e12, MI355X_VALU_PEAK_TFLOPS, "TFLOP/s"
    else:
        achieved, peak, unit = by / (ms * 1e-3) / 1e9, MI355X_HBM_PEAK_GBS, "GB/s"
    roof = {"bound": "alu" if alu else "hbm", "kernel": fam, "achieved": achieved, "peak": peak,
            "unit": unit, "frac": achieved / peak, "traffic": traffic,
            "avg_launch_us": 1e3 * ms / cnt, "bytes_per_launch": by / cnt, "flops_per_launch": fl / cnt,
            "flop_per_byte": fl / by, "ridge_flop_per_byte": ridge,
            "hbm_GBs": by / (ms * 1e-3) / 1e9, "source_digest": digest}
    breakdown = {k: {"ms": v[0], "launches": v[1],
                     "GB/s": v[2] / (v[0] * 1e-3) / 1e9 if v[0] > 0 else None,
                     "TFLOP/s": v[3] / (v[0] * 1e-3) / 1e12 if v[0] > 0 else None}
                 for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])}

    # post-processing of the batch's densities: potential on the grid, fields at
    # 64 points outside the support, far-field patterns in 256 directions
    post = {}
    if not args.no_post:
        rng = np.random.default_rng(7)
        pts = rng.standard_normal((64, 3))
        pts = 2.5 * pts / np.linalg.norm(pts, axis=1, keepdims=True)
        dirs = rng.standard_normal((256, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        calls = [("fields_at_64_points", lambda: plan.fields_at(d_mixed, pts))]
        if prob.kind != vie.MAXWELL:
            calls.insert(0, ("potential", lambda: plan.potential(d_mixed)))
        if omega > 0:
            calls.append(("far_field_256_dirs", lambda: plan.far_field(d_mixed, dirs)))
        for name, fn in calls:
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            post[name] = 1e3 * (time.perf_counter() - t0)

    # achievable HBM bandwidth on this device: a plain 2 GiB device-to-device copy
    src = torch.empty(2 ** 29, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    roof["copy_GBs"] = copy_gbs
    roof["hbm_frac_of_copy"] = roof["hbm_GBs"] / copy_gbs

    # the whole FFT matvec of the timed solver (its five passes, in the
    # precision the Krylov iteration applies): algorithmic bytes over time
    suffix = "_fp64" if primary_fp64 else "_fp32"
    passes = [v for k, v in prof.items() if k.startswith("fft_") and k.endswith(suffix)]
    matvec = None
    if passes:
        mv_ms, mv_by = sum(v[0] for v in passes), sum(v[2] for v in passes)
        mv_n = max(v[1] for v in passes)
        matvec = {"precision": suffix[1:], "passes": len(passes), "us_per_apply": 1e3 * mv_ms / mv_n,
                  "bytes_per_apply": mv_by / mv_n, "hbm_GBs": mv_by / (mv_ms * 1e-3) / 1e9}
        matvec["frac_of_hbm_peak"] = matvec["hbm_GBs"] / MI355X_HBM_PEAK_GBS
        matvec["frac_of_copy"] = matvec["hbm_GBs"] / copy_gbs

    cpu = None
    if not args.no_cpu_baseline:
        mv = (float(np.mean([s["matvecs_fp64"] for s in stats_all])) if primary_fp64 else
              fp64.get("fp64_matvecs_per_solve") or float(np.mean([s["matvecs_fp32"] + s["matvecs_fp64"]
                                                                   for s in stats_all])))
        print("[bench] timing the CPU oracle ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl, args.n, mv)

    if wl == "helmholtz128":
        desc = (f"helmholtz{n}: anisotropic Helmholtz {n}^3, omega={omega:.6g}, "
                f"eps^-1 = I + b(x)(A + 0.05i I), {B} seeded plane waves per step")
    else:
        desc = f"{wl}: {n}^3, omega={omega:.6g}, {B} right-hand sides per step, {prob.ncomp} unknowns per point"
    out = {
        "metric": METRIC if wl == "helmholtz128" else f"solves/s to rel residual {tol:g} ({wl})",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * total / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "c128 (FP64 apply and Krylov)" if primary_fp64 else "c64 FFT apply + c128 Krylov (mixed)",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "omega": omega, "nrhs_per_step": B, "tol_true_residual": tol,
                   "restart": args.restart,
                   "solver": "GMRES (FP64)" if primary_fp64 else "GMRES + FP64 iterative refinement"},
        "latency_ms": {"batch_p50": 1e3 * pct(step_s, 50), "batch_p99": 1e3 * pct(step_s, 99),
                       "single_p50": 1e3 * pct(lat, 50) if lat else None,
                       "single_p99": 1e3 * pct(lat, 99) if lat else None},
        "iters_per_solve": float(np.mean([s["iters"] for s in stats_all])),
        "matvecs_fp32_per_solve": float(np.mean([s["matvecs_fp32"] for s in stats_all])),
        "matvecs_fp64_per_solve": float(np.mean([s["matvecs_fp64"] for s in stats_all])),
        "max_rel_residual": float(max(s["rel_residual"] for s in stats_all)),
        **fp64,
        "roofline": roof,
        "matvec": matvec,
        "postprocess_ms_per_batch": post,
        "kernels": breakdown,
        "cpu_baseline": cpu,
    }
    if fp64 and not primary_fp64:
        out["speedup_mixed_vs_fp64"] = value / fp64["fp64_solves_per_s"]
    elif fp64:
        out["speedup_mixed_vs_fp64"] = fp64["mixed_solves_per_s"] / value
    print(json.dumps(out), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
