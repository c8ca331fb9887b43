#!/usr/bin/env python3
"""Headline benchmark: solves/s of 128^3 anisotropic Helmholtz to 1e-8 relative
error, FP32-mixed batched solver vs the plain FP64 solver, with p50/p99 latency.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--nrhs B] [--n 128] [--workload NAME]

Workload (helmholtz128): grid 128^3 on [-1,1]^3, omega = 8 pi (8 wavelengths
across the box), eps^{-1}(x) = I + b(x)(A + 0.05 i I) with a seeded symmetric
A of norm 0.5 and the C-infinity bump b of radius 0.8, plane waves along B
seeded directions (gradient of exp(i omega d.x) as incident field).
A step is one batched mixed-precision solve of the B right-hand sides (64 by
default) to a true relative residual of 1e-9 (error <= 1e-8); inputs are
resident in HBM before the timed region, which runs with kernel timing off
(the solver's applies replay from captured hipGraphs).  The per-kernel
HIP-event times (and the roofline of the dominant kernel) come from a second,
profiled pass over the same steps.  The oracle leg (CPU) times the oracle's
matvec for the CPU baseline and checks the timed batch against the oracle:
the oracle's true residual of the GPU solutions, and one oracle GMRES solve
to 1e-13 compared element by element (err_vs_oracle).  Prints one JSON line.

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
# Published vector peaks (256 CUs, 2.4 GHz): FP32 157.3 TFLOP/s (counting the
# two-per-lane packed FMA), FP64 78.6 TFLOP/s.  The library is compiled
# without packed FP32, so its FP32 kernels can issue at most half the
# published FP32 rate (78.6 TFLOP/s of FMAs); both are reported.
MI355X_FP32_PEAK_TFLOPS = 157.3
MI355X_FP64_PEAK_TFLOPS = 78.6
MI355X_FP32_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
METRIC = "solves/s to 1e-8 rel err (128³ Helmholtz), mixed vs FP64; p50/p99 latency"
# name: (right-hand sides per step, true relative residual, the solver `value` reports)
WORKLOADS = {"helmholtz128": (64, 1e-9, "mixed"), "laplace32": (1, 1e-10, "fp64"),
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


def cpu_model():
    """The host CPU as lscpu reports it: model name, then family / model /
    stepping and the logical CPUs visible (a virtual machine may report only a
    generic name); else /proc/cpuinfo's model name."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        f = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                f.setdefault(k.strip(), v.strip())
        if "Model name" in f:
            extra = ", ".join(f"{k.lower()} {f[k]}" for k in ("CPU family", "Model", "Stepping") if k in f)
            if "CPU(s)" in f:
                extra += f", {f['CPU(s)']} logical CPUs visible"
            return f"{f['Model name']} ({extra})" if extra else f["Model name"]
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        return None


def oracle_leg(workload: str, n: int, matvecs_per_solve: float, inc, dens, dens64, residual_rhs):
    """The oracle (NumPy FP64, window FFT route) on the host.

    * CPU baseline: one plan setup and one matvec at the benchmark's grid,
      scaled to solves/s with the GPU FP64 solver's matvec count; the same
      matvec with one FFT worker.
    * Parity of the timed batch: the oracle's true relative residual
      ||b - A x|| / ||b|| of the GPU mixed solutions of the right-hand sides
      `residual_rhs`, and one oracle GMRES solve (right-hand side 0, to a
      residual of 1e-13) against the GPU mixed and FP64 solutions of the same
      right-hand side, element by element (relative l2)."""
    from oracle import operator as op
    from oracle import solve as sv
    from oracle import tables as tb
    prob = make_problem(workload, n, 1)
    t0 = time.perf_counter()
    A = op.Operator(prob.kind, prob.coef, prob.omega, mu=prob.mu)
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    A.apply(inc[0])
    mv = time.perf_counter() - t0
    workers = tb.WORKERS
    tb.WORKERS = 1
    try:
        t0 = time.perf_counter()
        A.apply(inc[0])
        mv1 = time.perf_counter() - t0
    finally:
        tb.WORKERS = workers
    solve_s = mv * matvecs_per_solve
    cpu = {"value": 1.0 / solve_s, "unit": "solves/s", "cores": workers, "kind": "oracle",
           "sample": (f"one FP64 matvec of the oracle at {prob.n}^3 ({mv:.2f} s; scipy.fft with "
                      f"{workers} workers, the rest numpy; table setup {setup:.1f} s not counted) x "
                      f"{matvecs_per_solve:.1f} matvecs per solve (the GPU FP64 GMRES count for the same "
                      f"right-hand sides)"),
           "matvec_s": mv, "matvec_s_1_worker": mv1, "value_1_worker": 1.0 / (mv1 * matvecs_per_solve),
           "setup_s": setup, "cpu_model": cpu_model()}
    t0 = time.perf_counter()
    res = []
    for r in residual_rhs:
        b = A.rhs(inc[r])
        res.append(float(np.linalg.norm(b - A.apply(dens[r])) / np.linalg.norm(b)))
    x0, info = sv.gmres(A.apply, A.rhs(inc[0]), tol=1e-13, restart=100)
    ref = float(np.linalg.norm(x0))
    parity = {"oracle_rel_residual_max": max(res), "oracle_residual_rhs": list(residual_rhs),
              "err_vs_oracle": float(np.linalg.norm(dens[0] - x0)) / ref,
              "err_vs_oracle_fp64": float(np.linalg.norm(dens64[0] - x0)) / ref if dens64 is not None else None,
              "oracle_solve": {"rhs": 0, "tol": 1e-13, "matvecs": info["matvecs"],
                               "rel_residual": info["rel_residual"]},
              "oracle_parity_s": time.perf_counter() - t0}
    return cpu, parity


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
    ap.add_argument("--latency-solves", type=int, default=30, help="single-RHS mixed solves for p50/p99")
    ap.add_argument("--profile-steps", type=int, default=2,
                    help="steps of the second pass, timed per kernel with HIP events (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (CPU baseline and parity)")
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

    # ---- timed region: K batched mixed solves (kernel timing off, so the
    # solver's applies replay from their captured hipGraphs)
    step_s, stats_all = [], []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for k in range(args.steps):
        t0 = time.perf_counter()
        d_mixed, _, st, rc = solve(inc)
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - t0)
        stats_all.extend(st)
        print(f"[bench] step {k}: {step_s[-1]*1e3:.1f} ms, iters {[s['iters'] for s in st][:8]}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    solves = args.steps * B
    value = solves / total

    # ---- profiled pass over the same steps: per-kernel HIP events on the
    # launch stream (eager launches), algorithmic bytes and nominal flops
    prof = {}
    prof_step_ms = None
    if args.profile_steps > 0:
        plan.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.profile_steps):
            solve(inc)
        torch.cuda.synchronize()
        prof_step_ms = 1e3 * (time.perf_counter() - t0) / args.profile_steps
        prof = plan.profile_read()
        plan.profile(False)
        print(f"[bench] profiled pass: {prof_step_ms:.1f} ms per step", file=sys.stderr, flush=True)

    # ---- the other solver on the same batch: plain FP64 (or mixed, when the
    # workload's own figure is the FP64 solver's)
    fp64 = {}
    d64_host = None
    if not args.no_fp64 and args.fp64_steps > 0:
        # one untimed solve first, as for the timed steps (the other precision
        # tunes its tiles and captures its graphs at its first applies)
        solve(inc, fp64=not primary_fp64)
        ts = []
        for k in range(args.fp64_steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            d64, _, st64, _ = solve(inc, fp64=not primary_fp64)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        err = float(torch.linalg.vector_norm(d_mixed - d64) / torch.linalg.vector_norm(d64))
        d64_host = d64.cpu().numpy()
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

    # ---- roofline of the dominant kernel family (HIP events of the profiled
    # pass, algorithmic bytes, nominal flops): compute-bound when its
    # arithmetic intensity exceeds the ridge of the published peaks of its
    # precision, else HBM-bound; the byte rate against 8 TB/s is reported
    # either way
    roof, breakdown = None, {}
    if prof:
        fam, (ms, cnt, by, fl) = max(prof.items(), key=lambda kv: kv[1][0])
        fp32 = fam.endswith("_fp32")
        peak_tf = MI355X_FP32_PEAK_TFLOPS if fp32 else MI355X_FP64_PEAK_TFLOPS
        ridge = peak_tf * 1e12 / (MI355X_HBM_PEAK_GBS * 1e9)
        alu = fl / by > ridge
        from paper_1805_04791_amd import profiling
        tag = f"helmholtz{n}" if wl == "helmholtz128" else wl
        tr = profiling.read_traffic(os.path.join(ROOT, "profiles", f"{fam}.{tag}.traffic.md"))
        digest = profiling.source_digest()
        traffic = tr[0] if tr is not None and tr[2] == digest else None
        hbm_gbs = by / (ms * 1e-3) / 1e9
        tflops = fl / (ms * 1e-3) / 1e12
        if alu:
            achieved, peak, unit = tflops, peak_tf, "TFLOP/s"
        else:
            achieved, peak, unit = hbm_gbs, MI355X_HBM_PEAK_GBS, "GB/s"
        roof = {"bound": "alu" if alu else "hbm", "kernel": fam, "achieved": achieved, "peak": peak,
                "unit": unit, "frac": achieved / peak, "traffic": traffic,
                "avg_launch_us": 1e3 * ms / cnt, "bytes_per_launch": by / cnt, "flops_per_launch": fl / cnt,
                "flop_per_byte": fl / by, "ridge_flop_per_byte": ridge,
                "hbm_GBs": hbm_gbs, "hbm_frac": hbm_gbs / MI355X_HBM_PEAK_GBS,
                "valu_nominal_TFLOPs": tflops, "valu_frac_published": tflops / peak_tf,
                "valu_frac_unpacked": tflops / (MI355X_FP32_UNPACKED_TFLOPS if fp32 else MI355X_FP64_PEAK_TFLOPS),
                "timing": f"HIP events on the launch stream, {args.profile_steps} profiled steps",
                "source_digest": digest}
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
    if roof:
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

    cpu, parity = None, {}
    if not args.no_cpu_baseline:
        mv = (float(np.mean([s["matvecs_fp64"] for s in stats_all])) if primary_fp64 else
              fp64.get("fp64_matvecs_per_solve") or float(np.mean([s["matvecs_fp32"] + s["matvecs_fp64"]
                                                                   for s in stats_all])))
        print("[bench] oracle leg (CPU): baseline timing and parity of the timed batch ...",
              file=sys.stderr, flush=True)
        # the oracle's residual of every right-hand side of the batch, or of 8
        # seeded ones of a larger batch
        rr = list(range(B)) if B <= 8 else sorted(int(i) for i in np.random.default_rng(5).choice(B, 8, replace=False))
        cpu, parity = oracle_leg(wl, args.n, mv, prob.inc, d_mixed.cpu().numpy(), d64_host, rr)
        print(f"[bench] oracle: err {parity['err_vs_oracle']:.2e}, residual max "
              f"{parity['oracle_rel_residual_max']:.2e}", file=sys.stderr, flush=True)

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
        **parity,
        "roofline": roof,
        "matvec": matvec,
        "postprocess_ms_per_batch": post,
        "kernels": breakdown,
        "profiled_ms_per_step": prof_step_ms,
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
