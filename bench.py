#!/usr/bin/env python3
"""Benchmark of the online reduced Navier-Stokes stage on one MI355X.

One step = the whole hot path for one batch of synthetic requests, inputs already resident
in HBM: theta(mu) evaluation, the batched Newton solve (Jacobian + residual contraction on
MFMA, pivoted LU, update, stopping test) and the a posteriori pressure recovery.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched_n50]

Besides the batched FP64 headline (`value`), the JSON line carries, on the same N = 50
tensor set and parameters: the plain per-solve GPU path (the same library, one request per
call), the mixed-precision batched path (BF16 hi/lo tensors on MFMA + one FP64-residual
refinement step; --mixed-prec bf16 for plain BF16 tensors and three steps),
and the continuous-batching server under Poisson arrivals (throughput, p50/p99 latency);
each with its maximum relative error against the FP64 oracle on a checked sample.
Progress goes to stderr.
"""

from __future__ import annotations

import argparse
import hashlib
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

# Sources whose change invalidates the HBM byte counts recorded under profiles/.
TRAFFIC_SOURCES = ("paper_1807_11866_amd/csrc/rb_kernels.hpp",
                   "paper_1807_11866_amd/csrc/rb_common.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_digest():
    h = hashlib.sha256()
    for p in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from profiles/traffic.json, if recorded for the
    current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sources_digest") != sources_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("hbm_bytes_per_launch")


def rel_err(a, b):
    nb = np.linalg.norm(b, axis=-1)
    return np.linalg.norm(a - b, axis=-1) / np.where(nb > 0, nb, 1.0)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo, as lscpu reports it)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(ts, mu_h, cfg, args):
    """The oracle (velocity Newton + pressure recovery, FP64) on the host cores: first on all
    threads (OpenMP over requests, chunks of 512 requests), then on one core one request per
    call, for the per-solve p50/p99; each for half of --cpu-seconds."""
    import oracle  # CPU reference (test infrastructure)
    oset = oracle.OracleSet(ts)
    B, Np = mu_h.shape[0], ts.Np
    half = 0.5 * args.cpu_seconds
    done, tc0, threads = 0, time.perf_counter(), 0
    while time.perf_counter() - tc0 < half:
        sel = np.arange(done, done + 512) % B
        r = oracle.solve_batch(oset, mu_h[sel], pressure_np=Np, tol=cfg["tol"],
                               maxit=cfg["max_iter"], nthreads=0)
        threads = r["threads"]
        done += 512
    tc1 = time.perf_counter()
    per = []
    t1c = time.perf_counter()
    while time.perf_counter() - t1c < half:
        i = len(per) % B
        ta = time.perf_counter()
        oracle.solve_batch(oset, mu_h[i:i + 1], pressure_np=Np, tol=cfg["tol"],
                           maxit=cfg["max_iter"], nthreads=1)
        per.append(time.perf_counter() - ta)
    per_ms = 1e3 * np.asarray(per)
    cpu = dict(value=done / (tc1 - tc0), unit="solves/s", cores=int(threads), kind="oracle",
               cpu_model=cpu_model(),
               sample=f"{done} requests of the {args.workload} workload on {threads} threads "
                      f"(velocity Newton + pressure recovery, FP64, OpenMP over requests, "
                      f"{tc1 - tc0:.1f} s); then {len(per)} requests one per call on 1 core",
               single_core=dict(value=len(per) / per_ms.sum() * 1e3, unit="solves/s", cores=1,
                                requests=len(per), p50_ms=float(np.percentile(per_ms, 50)),
                                p99_ms=float(np.percentile(per_ms, 99))))
    log(f"[bench] cpu oracle: {cpu['value']:.4g} solves/s on {threads} threads, "
        f"{cpu['single_core']['value']:.4g} solves/s on 1 core "
        f"(p50 {cpu['single_core']['p50_ms']:.3f} ms, p99 {cpu['single_core']['p99_ms']:.3f} ms)")
    return cpu


def other_workload(args):
    """The other synthetic workloads, each timed the same way (inputs resident, HIP-event
    kernel timing, oracle check on a sample):
      single_n10      the plain single solve (B = 1 per call, FP64)
      mixed_n100      B = 32768 at N = 100: BF16 hi/lo tensors (--mixed-prec), FP32 LU, one
                      FP64-residual refinement step
      uneven_n20_100  B = 16384 with N in {20,...,100} in one call (FP32 + refinement)
      serve_n150      the server under Poisson arrivals, N ~ U{20..150}, FP32 + two refinement
                      steps, three lanes (--serve-prec, --serve-lanes)
    """
    import torch
    from paper_1807_11866_amd import rbns
    from rbinputs import get_config, make_tensor_set, draw_mu, draw_basis_sizes
    from rbinputs.synth import draw_arrivals
    import oracle  # CPU reference (test infrastructure)

    name = args.workload
    cfg = get_config(name)
    log(f"[bench] generating tensors for {name}")
    ts = make_tensor_set(cfg)
    dev = torch.device("cuda", 0)
    f64 = dict(dtype=torch.float64, device=dev)
    s = rbns.Solver(ts, device=0)
    stream = torch.cuda.current_stream()
    extra, roof, dtype = {}, None, "f64"
    B = cfg.get("B", 1)
    mu_h = draw_mu(cfg, B)
    mu = torch.as_tensor(mu_h, device=dev)
    th = s.theta(mu)
    torch.cuda.synchronize()
    fam_names = ("jacobian", "lu", "residual", "pressure", "stokes")

    def timed(step, nsteps, nwarm, ctx=None):
        ctx = s.ctx if ctx is None else ctx
        for _ in range(nwarm):
            step()
        torch.cuda.synchronize()
        rbns.rb_timing_enable(ctx, True)
        t0 = time.perf_counter()
        for _ in range(nsteps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rbns.rb_timing_enable(ctx, False)
        return t1 - t0, {f: rbns.rb_timing_read(ctx, f) for f in fam_names}

    if name == "single_n10":
        metric = "reduced NS solves/sec at N=10 (plain single solve, B=1 per call)"
        out = dict(u=torch.empty(1, ts.N, **f64), iters=torch.empty(1, dtype=torch.int32, device=dev),
                   status=torch.empty(1, dtype=torch.int32, device=dev))
        pout = dict(p=torch.empty(1, ts.Np, **f64),
                    pstatus=torch.empty(1, dtype=torch.int32, device=dev))
        th1 = s.theta(mu[:1])

        def step():
            rbns.rb_theta(s.ctx, s.set, 1, mu[:1], th1["ta"], th1["tc"], th1["tf"], th1["tb"], stream)
            s.solve(th1, out=out, tol=cfg["tol"], max_iter=cfg["max_iter"], stream=stream)
            s.pressure(th1, out["u"], out=pout, stream=stream)
            torch.cuda.synchronize()
        el, fams = timed(step, max(args.steps, 200), args.warmup)
        n = max(args.steps, 200)
        value, steps = n / el, n
        ms_step = 1e3 * el / n
        r = oracle.solve_batch(oracle.OracleSet(ts), mu_h[:1], pressure_np=ts.Np)
        extra["max_rel_err_u"] = float(rel_err(out["u"].cpu().numpy(), r["u"]).max())
        extra["max_rel_err_p"] = float(rel_err(pout["p"].cpu().numpy(), r["p"]).max())
        extra["mean_ms_per_solve"] = 1e3 * el / n
    elif name in ("mixed_n100", "uneven_n20_100"):
        uneven = name == "uneven_n20_100"
        x3 = args.mixed_prec == "bf16x3"
        prec = (rbns.RB_PREC_F32 if uneven else
                rbns.RB_PREC_BF16X3 if x3 else rbns.RB_PREC_BF16)
        refine = (2 if uneven else args.mixed_refine if args.mixed_refine >= 0 else
                  1 if x3 else 3)
        dtype = "f32" if uneven else args.mixed_prec
        Nreq = draw_basis_sizes(cfg, B) if uneven else np.full(B, ts.N, np.int32)
        Nd = torch.as_tensor(Nreq, device=dev, dtype=torch.int32)
        out = dict(u=torch.empty(B, ts.N, **f64), iters=torch.empty(B, dtype=torch.int32, device=dev),
                   status=torch.empty(B, dtype=torch.int32, device=dev))
        pout = dict(p=torch.empty(B, ts.Np, **f64), pstatus=torch.empty(B, dtype=torch.int32, device=dev))

        def step():
            rbns.rb_theta(s.ctx, s.set, B, mu, th["ta"], th["tc"], th["tf"], th["tb"], stream)
            if uneven:
                s.solve_uneven(th, Nd, tol=cfg["tol"], max_iter=cfg["max_iter"], precision=prec,
                               refine_steps=refine, out=out, stream=stream)
            else:
                s.solve(th, out=out, tol=cfg["tol"], max_iter=cfg["max_iter"], precision=prec,
                        refine_steps=refine, stream=stream)
                s.pressure(th, out["u"], out=pout, stream=stream)
        nsteps = max(3, args.steps // 4)
        el, fams = timed(step, nsteps, max(2, args.warmup // 2))
        value, steps = B * nsteps / el, nsteps
        ms_step = 1e3 * el / nsteps
        if uneven:
            # The graph replays carry no per-launch events: a second context on plain launches
            # (the same kernels) gives the kernel-family times of the roofline, and a fresh
            # N mix every step gives the rate when no shape repeats.
            os.environ["RB_UNEVEN_GRAPHS"] = "0"
            s2 = rbns.Solver(ts, device=0)
            del os.environ["RB_UNEVEN_GRAPHS"]
            th2 = s2.theta(mu)
            out2 = {k: torch.empty_like(v) for k, v in out.items()}

            def step2():
                s2.solve_uneven(th2, Nd, tol=cfg["tol"], max_iter=cfg["max_iter"],
                                precision=prec, refine_steps=refine, out=out2, stream=stream)
            el2, fams = timed(step2, nsteps, 1, ctx=s2.ctx)
            extra["eager_ms_per_step"] = 1e3 * el2 / nsteps
            extra["kernel_timing"] = "plain-launch pass with the same kernels as the graph replay"
            mixes = [torch.as_tensor(draw_basis_sizes(cfg, B, seed_offset=1000 + k), device=dev,
                                     dtype=torch.int32) for k in range(nsteps + 1)]
            s2.solve_uneven(th2, mixes[-1], tol=cfg["tol"], max_iter=cfg["max_iter"],
                            precision=prec, refine_steps=refine, out=out2, stream=stream)
            torch.cuda.synchronize()
            tf0 = time.perf_counter()
            for k in range(nsteps):
                s.solve_uneven(th, mixes[k], tol=cfg["tol"], max_iter=cfg["max_iter"],
                               precision=prec, refine_steps=refine, out=out2, stream=stream)
            torch.cuda.synchronize()
            extra["fresh_mix_solves_s"] = B * nsteps / (time.perf_counter() - tf0)
            log(f"[bench] uneven: graph replay {value:.4g} solves/s, plain launches "
                f"{B / (el2 / nsteps):.4g}, fresh N mix every call {extra['fresh_mix_solves_s']:.4g}")
            Nreq_t = Nreq
            s2.close()
        metric = ("reduced NS solves/sec, uneven N in {20..100} in one call (FP32 + FP64 "
                  "refinement)" if uneven else
                  f"reduced NS solves/sec at N=100 ({args.mixed_prec.upper()} MFMA + "
                  f"{refine} FP64-residual refinement step(s), velocity + pressure)")
        idx = np.linspace(0, B - 1, max(args.check, 1)).astype(int)
        r = oracle.solve_batch(oracle.OracleSet(ts), mu_h[idx], Nreq=Nreq[idx],
                               pressure_np=0 if uneven else ts.Np)
        extra["max_rel_err_u"] = float(rel_err(out["u"].cpu().numpy()[idx], r["u"]).max())
        if not uneven:
            extra["max_rel_err_p"] = float(rel_err(pout["p"].cpu().numpy()[idx], r["p"]).max())
        extra["checked_requests"] = int(len(idx))
        extra["refine_steps"] = refine
        extra["status_hist"] = np.bincount(out["status"].cpu().numpy(), minlength=5).tolist()
        extra["iters_hist"] = np.bincount(out["iters"].cpu().numpy()).tolist()
        K = ts.Q + ts.Qc * Nreq.astype(float)
        its = out["iters"].cpu().numpy().astype(float)
        # low-precision updates; the first one of a request starting from u = 0 takes its
        # Jacobian A(mu) from the "stokes" assembly, not the contraction
        lp_upd = np.maximum(its - refine, 1) - (1 if fams["stokes"][1] else 0)
        jac_flops = float((2.0 * Nreq ** 2 * K * np.maximum(lp_upd, 0)).sum()) * nsteps
        res_flops = float((2.0 * Nreq ** 2 * K * refine).sum()) * nsteps
        # algorithmic flops (BF16x3 issues three MFMAs per product) against the dense peak
        peak_j = 157.3 if prec == rbns.RB_PREC_F32 else 2516.6
        kern = {}
        for f, (ms, n) in fams.items():
            kern[f] = dict(total_ms=ms, launches=n)
        if fams["jacobian"][0] > 0:
            kern["jacobian"].update(achieved_tflops=jac_flops / (fams["jacobian"][0] * 1e-3) / 1e12,
                                    peak_tflops=peak_j, bound="mfma")
        if fams["residual"][0] > 0:
            kern["residual"].update(achieved_tflops=res_flops / (fams["residual"][0] * 1e-3) / 1e12,
                                    peak_tflops=78.6, bound="mfma")
        if fams["lu"][0] > 0:       # FP32 LU (both phases): 2N^3/3 + 4N^2 per Newton update
            lu_flops = float(((2.0 / 3.0 * Nreq ** 3 + 4.0 * Nreq ** 2) * its).sum()) * nsteps
            kern["lu"].update(achieved_tflops=lu_flops / (fams["lu"][0] * 1e-3) / 1e12,
                              peak_tflops=157.3, bound="alu")
        dominant = max(fams, key=lambda f: fams[f][0])
        d = kern[dominant]
        roof = dict(bound=d.get("bound", "alu"), achieved=d.get("achieved_tflops"),
                    peak=d.get("peak_tflops", 78.6), unit="TFLOP/s", kernel=dominant,
                    traffic=None, kernels=kern)
        roof["frac"] = roof["achieved"] / roof["peak"] if roof["achieved"] else None
    elif name == "serve_n150":
        sp = {"f32": (rbns.RB_PREC_F32, 2), "bf16x3": (rbns.RB_PREC_BF16X3, 1),
              "bf16": (rbns.RB_PREC_BF16, 4)}
        prec, refine = sp[args.serve_prec]
        metric = (f"served reduced NS solves/sec, N ~ U{{20..150}}, Poisson arrivals "
                  f"({args.serve_prec.upper()} + {refine} FP64-residual refinement step(s))")
        dtype = args.serve_prec
        rates = [float(x) for x in (args.serve_rates or "20000,50000,100000,200000").split(",")
                 if x.strip()]
        srv = rbns.Server(s, precision=prec, refine_steps=refine, max_iter=cfg["max_iter"],
                          tol=cfg["tol"], max_batch=4096, lanes=args.serve_lanes)
        extra["refine_steps"] = refine
        extra["lanes"] = args.serve_lanes
        served = {}
        Bp = 8192
        mu_s = draw_mu(cfg, Bp)
        N_s = draw_basis_sizes(cfg, Bp)
        idx = np.arange(0, Bp, Bp // max(args.check, 1))
        ref = oracle.solve_batch(oracle.OracleSet(ts), mu_s[idx], Nreq=N_s[idx])
        pos = {int(b): k for k, b in enumerate(idx)}
        try:
            for rate in rates:
                arr = draw_arrivals(cfg, rate, args.serve_seconds)
                n = len(arr)
                sel = np.arange(n) % Bp
                lat = np.full(n, np.nan)
                stat = np.full(n, -1, dtype=np.int64)
                errs = []
                got, i = 0, 0
                t0s = time.perf_counter()
                while i < n or got < n:
                    now = time.perf_counter() - t0s
                    j = int(np.searchsorted(arr, now, side="right"))
                    if j > i:
                        srv.submit(mu_s[sel[i:j], 0], mu_s[sel[i:j], 1], N_s[sel[i:j]],
                                   tags=np.arange(i, j))
                        i = j
                    ra = srv.poll_array()
                    if len(ra):
                        tg = ra["tag"]
                        lat[tg] = ra["latency_ms"]
                        stat[tg] = ra["status"]
                        got += len(ra)
                        for rr in ra:
                            m = pos.get(int(sel[int(rr["tag"])]))
                            if m is not None and len(errs) < 4 * len(idx):
                                nn = int(rr["N"])
                                errs.append(float(rel_err(rr["u"][:nn], ref["u"][m, :nn])))
                    elif i >= n:
                        time.sleep(2e-5)
                t1s = time.perf_counter()
                served[f"{int(rate)}"] = dict(offered_req_s=rate, requests=n, value=n / (t1s - t0s),
                                              p50_ms=float(np.percentile(lat, 50)),
                                              p99_ms=float(np.percentile(lat, 99)),
                                              max_ms=float(np.nanmax(lat)),
                                              status_hist=np.bincount(stat, minlength=6).tolist(),
                                              max_rel_err_u=max(errs) if errs else None)
                log(f"[bench] served at {rate:.3g} req/s: p50 {served[f'{int(rate)}']['p50_ms']:.3f} ms, "
                    f"p99 {served[f'{int(rate)}']['p99_ms']:.3f} ms")
        finally:
            srv.stop()
        top = served[f"{int(rates[-1])}"]
        value, steps = top["value"], len(rates)
        ms_step = None                            # open-loop serving: no step
        extra["served"] = served
        extra["p99_ms"] = top["p99_ms"]
        fams = {}
    else:
        raise SystemExit(f"unknown workload {name}")

    res = {"metric": metric, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": {"workload": name, "N": ts.N, "B": B, "Q": ts.Q, "Qc": ts.Qc,
                      "parallelism": "single_gpu"},
           "roofline": roof, "cpu_baseline": None, "kernel_ms": fams, **extra}
    print(json.dumps(res), flush=True)
    s.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batched_n50")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--plain", type=int, default=256,
                    help="requests timed on the plain one-request-per-call path (0 = skip)")
    ap.add_argument("--check", type=int, default=64, help="requests re-solved by the oracle")
    ap.add_argument("--mixed-refine", type=int, default=-2,
                    help="refinement steps of the mixed-precision leg (-1 = skip; default "
                         "1 for bf16x3, 3 for bf16)")
    ap.add_argument("--mixed-prec", choices=("bf16x3", "bf16"), default="bf16x3",
                    help="tensor format of the mixed-precision leg / workload")
    ap.add_argument("--serve-rates", default=None,
                    help="Poisson arrival rates (req/s) of the serving leg ('' = skip; default "
                         "20000,50000,100000,200000,1000000, and 20000,50000,100000,200000 "
                         "for serve_n150)")
    ap.add_argument("--serve-seconds", type=float, default=1.5)
    ap.add_argument("--serve-prec", choices=("f32", "bf16x3", "bf16"), default="f32",
                    help="tensor format of the serve_n150 workload")
    ap.add_argument("--serve-lanes", type=int, default=3,
                    help="server lanes (batches in flight) of the serve_n150 workload")
    ap.add_argument("--coupled", type=int, default=1,
                    help="time the coupled stabilised (naive) solver against the block method "
                         "at m = 10, 20, 30 (0 = skip)")
    ap.add_argument("--assemble", type=int, default=1,
                    help="time the offline convection-tensor assembly on the GPU (0 = skip)")
    ap.add_argument("--reconstruct", type=int, default=1,
                    help="time the combined-basis pressure reconstruction (0 = skip)")
    ap.add_argument("--autotune", action="store_true",
                    help="run the library's autotuner on the batch before the warm-up")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the bench, one plain device copy of this many MiB (the "
                         "reference kernel for scaling HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        log("bench.py: only --gpus 1 is supported (the solves are independent per parameter;"
            " DESIGN.md describes how the path would shard)")
        sys.exit(2)

    if not args.workload.startswith("batched_"):
        other_workload(args)
        return
    if args.workload != "batched_n50":
        # another batched tensor set (batched_n50_q50: the paper-shaped term counts): the
        # batched FP64 step and its roofline only
        args.plain, args.coupled, args.reconstruct, args.mixed_refine = 0, 0, 0, -1
        args.assemble = 0
        args.serve_rates = ""

    import torch
    from paper_1807_11866_amd import rbns
    from rbinputs import get_config, make_tensor_set, draw_mu
    from rbinputs.synth import draw_arrivals

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

    if args.autotune:
        rbns.rb_theta(s.ctx, s.set, B, mu, th["ta"], th["tc"], th["tf"], th["tb"], stream)
        tuned = s.autotune(th, tol=cfg["tol"], max_iter=cfg["max_iter"], stream=stream)
        torch.cuda.synchronize()
        log(f"[bench] autotuned (row splits, LDS pivot broadcast) = {tuned}")
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
    stokes_ms, stokes_n = rbns.rb_timing_read(s.ctx, "stokes")
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = B * args.steps / elapsed
    log(f"[bench] {ms_per_step:.3f} ms/step, {value:.4g} solves/s; kernels: {fams}")

    iters = out["iters"].cpu().numpy()
    status = out["status"].cpu().numpy()
    pstatus = pout["pstatus"].cpu().numpy()

    # ---- rooflines (algorithmic flops / live HIP-event durations of each family) ----------
    # unit = one (request, Newton update); launches of a family include the ones in which
    # every request had already converged (they exit at once).
    K = ts.Q + ts.Qc * N
    units = float(iters.sum()) * args.steps
    # the first update of every request starts from u = 0: its Jacobian A(mu) comes from the
    # "stokes" assembly, not the contraction, which does the other updates
    units_fam = {"jacobian": units - float(B) * stokes_n, "lu": units}
    per_unit = {
        "jacobian": 2.0 * N * N * K,                        # J (and A u) contraction
        "lu": 2.0 / 3.0 * N ** 3 + 2.0 * N * N * 2,         # LU + triangular solves + J u
    }
    pflops = 2.0 * Np * N * K + 2.0 / 3.0 * Np ** 3 + 2.0 * Np * Np * 2
    kern = {}
    for f, (ms, n) in fams.items():
        work = per_unit[f] * units_fam[f] if f in per_unit else pflops * B * args.steps
        kern[f] = dict(total_ms=ms, launches=n, avg_launch_ms=(ms / n if n else None),
                       achieved_tflops=work / (ms * 1e-3) / 1e12 if ms > 0 else None)
    names = {"jacobian": ("contract_f64_kernel<kModeJac> (MFMA-F64 Jacobian + A(mu)u)", "mfma",
                          PEAK["fp64_mfma_tflops"]),
             "lu": ("lu_f64_kernel (FP64 register LU + update) + newton_tail_f64_kernel", "alu",
                    PEAK["fp64_vector_tflops"]),
             "pressure": ("contract_f64_kernel<kModePressure> + pressure solve (plu_mfma_f64_kernel for Np <= 31)", "mfma",
                          PEAK["fp64_mfma_tflops"])}
    for f in kern:
        kern[f]["kernel"], kern[f]["bound"], kern[f]["peak_tflops"] = names[f]
        a = kern[f]["achieved_tflops"]
        kern[f]["frac"] = a / names[f][2] if a else None
        kern[f]["traffic"] = recorded_traffic(f)        # HBM bytes per launch (profiled)
    dominant = max(fams, key=lambda f: fams[f][0])
    d = kern[dominant]
    roof = dict(bound=d["bound"], achieved=d["achieved_tflops"], peak=d["peak_tflops"],
                unit="TFLOP/s", frac=d["frac"], kernel=d["kernel"],
                avg_launch_ms=d["avg_launch_ms"],
                units_per_launch=(units_fam[dominant] / d["launches"] if dominant != "pressure"
                                  else B),
                work_per_unit_flop=(per_unit.get(dominant, pflops)))
    roof["traffic"] = recorded_traffic(dominant)
    roof["jacobian_contraction"] = kern["jacobian"]
    roof["kernels"] = kern
    if stokes_n:                            # HBM-bound: J written once per request
        sb = 8.0 * N * N * B * args.steps
        roof["stokes_jacobian"] = dict(
            kernel="stokes_jacobian_kernel (first Jacobian A(mu) from the affine operators)",
            bound="hbm", total_ms=stokes_ms, launches=stokes_n, avg_launch_ms=stokes_ms / stokes_n,
            achieved_gbs=sb / (stokes_ms * 1e-3) / 1e9, peak_gbs=PEAK["hbm_gbs"],
            frac=sb / (stokes_ms * 1e-3) / 1e9 / PEAK["hbm_gbs"],
            traffic=recorded_traffic("stokes"))

    # ---- parity of the timed outputs against the oracle on a sample ------------------------
    extra = {}
    idx = np.linspace(0, B - 1, max(args.check, 1)).astype(int)
    ref = None
    if args.check > 0:
        import oracle  # CPU reference (test infrastructure)
        ref = oracle.solve_batch(oracle.OracleSet(ts), mu_h[idx], pressure_np=Np,
                                 tol=cfg["tol"], maxit=cfg["max_iter"])
        u = out["u"].cpu().numpy()[idx]
        p = pout["p"].cpu().numpy()[idx]
        extra["max_rel_err_u"] = float(rel_err(u, ref["u"]).max())
        extra["max_rel_err_p"] = float(rel_err(p, ref["p"]).max())
        extra["checked_requests"] = int(len(idx))

    # ---- pressure reconstruction from a combined basis (p = Pc u) -------------------------
    # Offline step with the library itself: the 15 x 15 Gauss training ensemble solved and its
    # pressure recovered on the GPU, Pc = P pinv(U) (minimum-norm snapshot coefficients, the
    # paper's second combined-basis construction). Online: one matrix-vector product per
    # request, timed on the same batch as the headline, error against the recovered pressure.
    if args.reconstruct:
        from rbinputs.synth import gauss_grid_mu
        mtr = gauss_grid_mu(cfg)
        thr = s.theta(torch.as_tensor(mtr, device=dev))
        otr = s.solve(thr, tol=cfg["tol"], max_iter=cfg["max_iter"], stream=stream)
        ptr = s.pressure(thr, otr["u"], stream=stream)
        torch.cuda.synchronize()
        Ut, Pt = otr["u"].cpu().numpy(), ptr["p"].cpu().numpy()
        Pc = Pt.T @ np.linalg.pinv(Ut.T, rcond=1e-8)
        dPc = torch.as_tensor(Pc, device=dev)
        prc = torch.empty(B, Np, **f64)
        for _ in range(3):
            s.reconstruct(dPc, out["u"], out=prc, stream=stream)
        torch.cuda.synchronize()
        rbns.rb_timing_enable(s.ctx, True)
        nrc = 50
        tr0 = time.perf_counter()
        for _ in range(nrc):
            s.reconstruct(dPc, out["u"], out=prc, stream=stream)
        torch.cuda.synchronize()
        tr1 = time.perf_counter()
        rbns.rb_timing_enable(s.ctx, False)
        kms, kn = rbns.rb_timing_read(s.ctx, "reconstruct")
        pr = prc.cpu().numpy()
        prv = pout["p"].cpu().numpy()
        erc = rel_err(pr, prv)
        extra["reconstructed"] = dict(
            value=B * nrc / (tr1 - tr0), unit="pressures/s", kernel_us=1e3 * kms / max(kn, 1),
            recovery_kernel_us=1e3 * kern["pressure"]["avg_launch_ms"],
            training_parameters=int(len(mtr)),
            rel_diff_vs_recovered_p50=float(np.median(erc)),
            rel_diff_vs_recovered_max=float(erc.max()))
        if ref is not None:
            extra["reconstructed"]["max_rel_err_p_vs_oracle_recovery"] = float(
                rel_err(pr[idx], ref["p"]).max())
        log(f"[bench] reconstruction: {extra['reconstructed']['kernel_us']:.1f} us per batch, "
            f"max rel. difference from recovery {erc.max():.2e}")

    # ---- the paper's naive solver: Newton on the coupled stabilised system (eqn block) -----
    # Velocity, supremizer and pressure spaces of equal size m (the paper's comparison, with
    # 3m unknowns) against the block method (velocity-only Newton at m + pressure recovery),
    # same library, same batch of parameters, same stopping rule, FP64. Pressure form with
    # the identity weight only (B_vp = 0), so both reach the same (u, p).
    if args.coupled:
        from rbinputs.synth import make_coupled_set
        cfg1 = get_config(args.workload, Qb=1)
        base1 = make_tensor_set(cfg1)
        mu_c = torch.as_tensor(mu_h, device=dev)
        cres = {}
        for m in (10, 20, 30):
            ts_b = base1.leading(m, m)
            ts_c = make_coupled_set(cfg1, m, m)
            sb, sc = rbns.Solver(ts_b, device=0), rbns.Solver(ts_c, device=0)
            thb = sb.theta(mu_c)
            thc = dict(ta=torch.cat([thb["ta"], torch.ones_like(thb["ta"][:, :1])], 1).contiguous(),
                       tc=thb["tc"], tf=thb["tf"])
            ob = dict(u=torch.empty(B, m, **f64), iters=torch.empty(B, dtype=torch.int32, device=dev),
                      status=torch.empty(B, dtype=torch.int32, device=dev))
            pb = dict(p=torch.empty(B, m, **f64), pstatus=torch.empty(B, dtype=torch.int32, device=dev))
            oc = dict(u=torch.empty(B, 3 * m, **f64), iters=torch.empty(B, dtype=torch.int32, device=dev),
                      status=torch.empty(B, dtype=torch.int32, device=dev))

            def blk():
                sb.solve(thb, out=ob, tol=cfg["tol"], max_iter=cfg["max_iter"], stream=stream)
                sb.pressure(thb, ob["u"], out=pb, stream=stream)

            def nai():
                sc.solve(thc, out=oc, tol=cfg["tol"], max_iter=cfg["max_iter"], stream=stream)
            tms = {}
            for name, fn in (("block", blk), ("naive", nai)):
                for _ in range(2):
                    fn()
                torch.cuda.synchronize()
                nrep = 5
                t0c = time.perf_counter()
                for _ in range(nrep):
                    fn()
                torch.cuda.synchronize()
                tms[name] = (time.perf_counter() - t0c) / nrep
            x = oc["u"].cpu().numpy()
            ub, pp = ob["u"].cpu().numpy(), pb["p"].cpu().numpy()
            cres[str(m)] = dict(unknowns_block=m, unknowns_naive=3 * m,
                                block_solves_s=B / tms["block"], naive_solves_s=B / tms["naive"],
                                speedup_block_vs_naive=tms["naive"] / tms["block"],
                                max_rel_diff_u=float(rel_err(x[:, :m], ub).max()),
                                max_rel_diff_p=float(rel_err(x[:, 2 * m:], pp).max()),
                                max_abs_s=float(np.abs(x[:, m:2 * m]).max()),
                                naive_status_hist=np.bincount(oc["status"].cpu().numpy(),
                                                              minlength=5).tolist())
            log(f"[bench] m={m}: block {B / tms['block']:.4g} solves/s, naive {B / tms['naive']:.4g} "
                f"solves/s ({tms['naive'] / tms['block']:.1f}x)")
            sb.close()
            sc.close()
        extra["coupled_vs_block"] = cres

    # ---- offline: the convection tensors by quadrature on the GPU (eqn tensor) -------------
    if args.assemble:
        from rbinputs.synth import quadrature_fields
        fq = quadrature_fields(N, Np, cfg["kmax"], cfg["G_quad"], ts.Q, ts.Qc, ts.Qb,
                               cfg["seeds"])
        Xq = fq["phi"].shape[-1]
        phiT = torch.as_tensor(np.ascontiguousarray(fq["phi"].transpose(2, 1, 0)), device=dev)
        dphiT = torch.as_tensor(np.ascontiguousarray(fq["dphi"].transpose(3, 1, 2, 0)), device=dev)
        cout = torch.empty(ts.Qc, N, N, N, **f64)
        rbns.rb_assemble_convection(s.ctx, N, N, Xq, ts.Qc, phiT, dphiT, phiT, fq["M"],
                                    fq["w"], cout, stream)           # warm (workspace)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        nas = 5
        ev0.record(stream)
        for _ in range(nas):
            rbns.rb_assemble_convection(s.ctx, N, N, Xq, ts.Qc, phiT, dphiT, phiT, fq["M"],
                                        fq["w"], cout, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ams = ev0.elapsed_time(ev1) / nas
        aflop = 8.0 * N * Xq * N * N + 8.0 * Xq * N * N        # four base contractions + D_b
        dif = float(np.abs(cout.cpu().numpy() - ts.C).max() / np.abs(ts.C).max())
        extra["assembly"] = dict(ms=ams, tensor=f"C [{ts.Qc}][{N}][{N}][{N}] from {Xq} points",
                                 achieved_tflops=aflop / (ams * 1e-3) / 1e12,
                                 frac_fp64_mfma=aflop / (ams * 1e-3) / 1e12 / PEAK["fp64_mfma_tflops"],
                                 max_rel_diff_vs_generator=dif)
        log(f"[bench] tensor assembly: {ams:.3f} ms, {extra['assembly']['achieved_tflops']:.1f} "
            f"TFLOP/s, max rel. difference {dif:.1e}")

    # ---- plain per-solve GPU path: the same library, one request per call ------------------
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
        extra["plain"] = dict(value=P / (tp1 - tp0), unit="solves/s", requests=P,
                              mean_ms=1e3 * (tp1 - tp0) / P)
        extra["speedup_batched_vs_plain"] = value / extra["plain"]["value"]
        log(f"[bench] plain path: {extra['plain']['value']:.4g} solves/s")

    # ---- mixed precision: BF16 tensors on MFMA, FP32 LU, FP64-residual refinement ----------
    mprec = rbns.RB_PREC_BF16X3 if args.mixed_prec == "bf16x3" else rbns.RB_PREC_BF16
    if args.mixed_refine == -2:
        args.mixed_refine = 1 if args.mixed_prec == "bf16x3" else 3
    if args.mixed_refine >= 0:
        mo = dict(u=torch.empty(B, N, **f64), iters=torch.empty(B, dtype=torch.int32, device=dev),
                  status=torch.empty(B, dtype=torch.int32, device=dev))

        def mstep():
            rbns.rb_theta(s.ctx, s.set, B, mu, th["ta"], th["tc"], th["tf"], th["tb"], stream)
            s.solve(th, out=mo, tol=cfg["tol"], max_iter=cfg["max_iter"],
                    precision=mprec, refine_steps=args.mixed_refine, stream=stream)
            s.pressure(th, mo["u"], out=pout, stream=stream)
        for _ in range(2):
            mstep()
        torch.cuda.synchronize()
        nm = max(3, args.steps // 2)
        tm0 = time.perf_counter()
        for _ in range(nm):
            mstep()
        torch.cuda.synchronize()
        tm1 = time.perf_counter()
        mix = dict(value=B * nm / (tm1 - tm0), unit="solves/s", refine_steps=args.mixed_refine,
                   dtype=f"{args.mixed_prec} tensors / fp32 accumulate + lu / fp64 residual "
                         "and iterate",
                   status_hist=np.bincount(mo["status"].cpu().numpy(), minlength=5).tolist())
        if ref is not None:
            mix["max_rel_err_u"] = float(rel_err(mo["u"].cpu().numpy()[idx], ref["u"]).max())
            mix["max_rel_err_p"] = float(rel_err(pout["p"].cpu().numpy()[idx], ref["p"]).max())
        extra["mixed_" + args.mixed_prec] = mix
        log(f"[bench] mixed {args.mixed_prec} + {args.mixed_refine} refinement steps: "
            f"{mix['value']:.4g} solves/s")

    # ---- served: continuous batching under Poisson arrivals --------------------------------
    srates = ("20000,50000,100000,200000,1000000" if args.serve_rates is None
              else args.serve_rates)
    rates = [float(r) for r in srates.split(",") if r.strip()]
    if rates:
        served = {}
        srv = rbns.Server(s, precision=rbns.RB_PREC_F64, max_iter=cfg["max_iter"],
                          tol=cfg["tol"], max_batch=4096, lanes=3, pressure=True)
        try:
            srv.submit(mu_h[:256, 0], mu_h[:256, 1], N)      # warm the lanes
            got = 0
            while got < 256:
                got += len(srv.poll_array())
                time.sleep(1e-4)
            pos = {int(b): k for k, b in enumerate(idx)}
            for rate in rates:
                arr = draw_arrivals(cfg, rate, args.serve_seconds)
                n = len(arr)
                sel = np.arange(n) % B
                st0 = srv.stats()
                lat = np.full(n, np.nan)
                qw = np.full(n, np.nan)
                stat = np.full(n, -1, dtype=np.int64)
                chk = [k for k in range(n) if int(sel[k]) in pos][:len(idx)]
                chk_set = {k: m for m, k in enumerate(chk)}
                cu = np.zeros((len(chk), N))
                cp = np.zeros((len(chk), Np))
                got = 0
                i = 0
                t0s = time.perf_counter()
                while i < n or got < n:
                    now = time.perf_counter() - t0s
                    j = int(np.searchsorted(arr, now, side="right"))
                    if j > i:
                        srv.submit(mu_h[sel[i:j], 0], mu_h[sel[i:j], 1], N, tags=np.arange(i, j))
                        i = j
                    ra = srv.poll_array()
                    if len(ra):
                        tg = ra["tag"]
                        lat[tg] = ra["latency_ms"]
                        qw[tg] = ra["queue_ms"]
                        stat[tg] = ra["status"]
                        got += len(ra)
                        for r in ra:
                            m = chk_set.get(int(r["tag"]))
                            if m is not None:
                                cu[m] = r["u"][:N]
                                cp[m] = r["p"][:Np]
                    elif i >= n:
                        time.sleep(2e-5)
                t1s = time.perf_counter()
                st1 = srv.stats()
                ent = dict(offered_req_s=rate, requests=n, value=n / (t1s - t0s),
                           unit="solves/s", p50_ms=float(np.percentile(lat, 50)),
                           p99_ms=float(np.percentile(lat, 99)), max_ms=float(lat.max()),
                           p50_queue_ms=float(np.percentile(qw, 50)),
                           p99_queue_ms=float(np.percentile(qw, 99)),
                           batches=int(st1["batches"] - st0["batches"]),
                           status_hist=np.bincount(stat, minlength=6).tolist())
                ent["mean_batch"] = n / max(ent["batches"], 1)
                if ref is not None and chk:
                    rr = np.array([pos[int(sel[k])] for k in chk])
                    ent["max_rel_err_u"] = float(rel_err(cu, ref["u"][rr]).max())
                    ent["max_rel_err_p"] = float(rel_err(cp, ref["p"][rr]).max())
                served[f"{int(rate)}"] = ent
                log(f"[bench] served at {rate:.3g} req/s: {ent['value']:.4g} solves/s, "
                    f"p50 {ent['p50_ms']:.3f} ms, p99 {ent['p99_ms']:.3f} ms")
        finally:
            srv.stop()
        extra["served"] = served

    # ---- CPU baseline: the oracle as it stands, bounded sample of the same workload --------
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(ts, mu_h, cfg, args)

    res = {
        "metric": (f"reduced NS solves/sec at N={N} (batched, velocity Newton + pressure "
                   f"recovery{', Q=%d, Qc=%d' % (ts.Q, ts.Qc) if args.workload != 'batched_n50' else ''})"),
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
