#!/usr/bin/env python3
"""Benchmark of the online reduced Navier-Stokes stage on one MI355X.

One step = the whole hot path for one batch of synthetic requests, inputs already resident
in HBM: theta(mu) evaluation, the batched Newton solve (Jacobian + residual contraction on
MFMA, pivoted LU, update, stopping test) and the a posteriori pressure recovery.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched_n50]

Prints one JSON line (see the keys below). Progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks
    "fp64_mfma_tflops": 78.6,
    "fp64_vector_tflops": 78.6,
    "fp32_mfma_tflops": 157.3,
    "hbm_gbs": 8000.0,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batched_n50")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--plain", type=int, default=256,
                    help="requests timed on the plain B=1 path (0 = skip)")
    ap.add_argument("--check", type=int, default=64, help="requests re-solved by the oracle")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the bench, one plain device copy of this many MiB (the "
                         "reference kernel for scaling HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        log("bench.py: only --gpus 1 is supported (the solves are independent per parameter;"
            " see DESIGN.md for how the path would shard)")
        sys.exit(2)

    import torch
    from paper_1807_11866_amd import rbns
    from rbinputs import get_config, make_tensor_set, draw_mu

    cfg = get_config(args.workload)
    log(f"[bench] generating tensors for {args.workload}")
    ts = make_tensor_set(cfg)
    B, N, Np = cfg["B"], cfg["N"], cfg["Np"]
    mu_h = draw_mu(cfg)
    dev = torch.device("cuda", 0)
    mu = torch.as_tensor(mu_h, device=dev)

    s = rbns.Solver(ts, device=0)
    f64 = dict(dtype=torch.float64, device=dev)
    th = dict(ta=torch.empty(B, ts.Q, **f64), tc=torch.empty(B, ts.Qc, **f64),
              tf=torch.empty(B, ts.Qf, **f64), tb=torch.empty(B, ts.Qb, **f64))
    out = dict(u=torch.empty(B, N, **f64), iters=torch.empty(B, dtype=torch.int32, device=dev),
               status=torch.empty(B, dtype=torch.int32, device=dev))
    pout = dict(p=torch.empty(B, Np, **f64), pstatus=torch.empty(B, dtype=torch.int32, device=dev))
    stream = torch.cuda.current_stream()

    def step():
        rbns.rb_theta(s.ctx, s.set, B, mu, th["ta"], th["tc"], th["tf"], th["tb"], stream)
        s.solve(th, out=out, tol=cfg["tol"], max_iter=cfg["max_iter"], stream=stream)
        s.pressure(th, out["u"], out=pout, stream=stream)

    log(f"[bench] warmup {args.warmup} steps (B={B}, N={N})")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    rbns.rb_timing_enable(s.ctx, True)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rbns.rb_timing_enable(s.ctx, False)
    fams = {f: rbns.rb_timing_read(s.ctx, f) for f in ("jacobian", "lu", "pressure")}
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = B * args.steps / elapsed
    log(f"[bench] {ms_per_step:.3f} ms/step, {value:.4g} solves/s; kernels: {fams}")

    iters = out["iters"].cpu().numpy()
    status = out["status"].cpu().numpy()
    pstatus = pout["pstatus"].cpu().numpy()

    # ---- roofline of the dominant kernel (algorithmic flops / live HIP-event durations) ----
    K = ts.Q + ts.Qc * N
    jac_flops_unit = 2.0 * N * N * K                     # per (request, Newton iteration)
    lu_flops_unit = 2.0 / 3.0 * N ** 3 + 2.0 * N * N * 2  # LU + triangular solves + J u
    units = float(iters.sum()) * args.steps
    jac_ms, jac_n = fams["jacobian"]
    lu_ms, lu_n = fams["lu"]
    pr_ms, pr_n = fams["pressure"]
    dominant = max(fams, key=lambda f: fams[f][0])
    if dominant == "jacobian":
        achieved = units * jac_flops_unit / (jac_ms * 1e-3) / 1e12
        roof = dict(bound="mfma", achieved=achieved, peak=PEAK["fp64_mfma_tflops"],
                    unit="TFLOP/s", kernel="jac_f64_kernel (MFMA-F64 Jacobian + residual)")
    elif dominant == "lu":
        achieved = units * lu_flops_unit / (lu_ms * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=PEAK["fp64_vector_tflops"],
                    unit="TFLOP/s", kernel="lu_f64_kernel (FP64 VALU pivoted LU)")
    else:
        pflops = 2.0 * Np * N * K + 2.0 / 3.0 * Np ** 3
        achieved = B * args.steps * pflops / (pr_ms * 1e-3) / 1e12
        roof = dict(bound="mfma", achieved=achieved, peak=PEAK["fp64_mfma_tflops"],
                    unit="TFLOP/s", kernel="pressure_f64_kernel")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["avg_launch_ms"] = {f: (fams[f][0] / fams[f][1] if fams[f][1] else None) for f in fams}
    roof["launches"] = {f: fams[f][1] for f in fams}
    roof["total_ms"] = {f: fams[f][0] for f in fams}

    # ---- parity of the timed outputs against the oracle on a sample ----
    extra = {}
    if args.check > 0:
        import oracle
        idx = np.linspace(0, B - 1, args.check).astype(int)
        r = oracle.solve_batch(oracle.OracleSet(ts), mu_h[idx], pressure_np=Np,
                               tol=cfg["tol"], maxit=cfg["max_iter"])
        u = out["u"].cpu().numpy()[idx]
        p = pout["p"].cpu().numpy()[idx]
        eu = np.linalg.norm(u - r["u"], axis=1) / np.linalg.norm(r["u"], axis=1)
        ep = np.linalg.norm(p - r["p"], axis=1) / np.linalg.norm(r["p"], axis=1)
        extra["max_rel_err_u"] = float(eu.max())
        extra["max_rel_err_p"] = float(ep.max())
        extra["checked_requests"] = int(len(idx))

    # ---- plain per-solve GPU path: the same library, B = 1 sequential calls ----
    if args.plain > 0:
        P = min(args.plain, B)
        th1 = {k: v[:1].clone() for k, v in th.items()}
        o1 = dict(u=torch.empty(1, N, **f64), iters=torch.empty(1, dtype=torch.int32, device=dev),
                  status=torch.empty(1, dtype=torch.int32, device=dev))
        p1 = dict(p=torch.empty(1, Np, **f64), pstatus=torch.empty(1, dtype=torch.int32, device=dev))
        for _ in range(3):
            rbns.rb_theta(s.ctx, s.set, 1, mu[:1], th1["ta"], th1["tc"], th1["tf"], th1["tb"], stream)
            s.solve(th1, out=o1, stream=stream)
            s.pressure(th1, o1["u"], out=p1, stream=stream)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for i in range(P):
            rbns.rb_theta(s.ctx, s.set, 1, mu[i:i + 1], th1["ta"], th1["tc"], th1["tf"],
                          th1["tb"], stream)
            s.solve(th1, out=o1, tol=cfg["tol"], max_iter=cfg["max_iter"], stream=stream)
            s.pressure(th1, o1["u"], out=p1, stream=stream)
            torch.cuda.synchronize()
        tp1 = time.perf_counter()
        extra["plain_value"] = P / (tp1 - tp0)
        extra["plain_requests"] = P
        extra["speedup_vs_plain"] = value / extra["plain_value"]
        log(f"[bench] plain B=1 path: {extra['plain_value']:.4g} solves/s")

    # ---- CPU baseline: the oracle as it stands, bounded sample of the same workload ----
    cpu = None
    if not args.no_cpu:
        import oracle
        oset = oracle.OracleSet(ts)
        done, tc0 = 0, time.perf_counter()
        threads = 0
        chunk = 512
        while time.perf_counter() - tc0 < args.cpu_seconds:
            sel = np.arange(done, done + chunk) % B
            r = oracle.solve_batch(oset, mu_h[sel], pressure_np=Np, tol=cfg["tol"],
                                   maxit=cfg["max_iter"], nthreads=0)
            threads = r["threads"]
            done += chunk
        tc1 = time.perf_counter()
        cpu = dict(value=done / (tc1 - tc0), unit="solves/s", cores=int(threads), kind="oracle",
                   sample=f"{done} requests of the {args.workload} workload (velocity Newton + "
                          f"pressure recovery, FP64, OpenMP over requests), {tc1 - tc0:.1f} s")
        log(f"[bench] cpu oracle: {cpu['value']:.4g} solves/s on {threads} threads")

    res = {
        "metric": "reduced NS solves/sec at N=50 (batched, velocity Newton + pressure recovery)",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": N, "B": B, "Q": ts.Q, "Qc": ts.Qc,
                   "Qf": ts.Qf, "Np": Np, "Qb": ts.Qb, "tol": cfg["tol"],
                   "max_iter": cfg["max_iter"], "parallelism": "single_gpu"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "newton_iters_hist": np.bincount(iters).tolist(),
        "status_hist": np.bincount(status, minlength=5).tolist(),
        "pressure_status_hist": np.bincount(pstatus, minlength=5).tolist(),
        **extra,
    }
    print(json.dumps(res), flush=True)
    s.close()
    if args.copy_mib > 0:
        n = args.copy_mib << 17                      # doubles
        x = torch.ones(n, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log(f"[bench] copy reference: {args.copy_mib} MiB read + {args.copy_mib} MiB written")


if __name__ == "__main__":
    main()
