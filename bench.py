"""Benchmark: balanced-partition KRR (BKRR2) on one MI355X.

Workload (one "step" = the whole hot path once): n = 65,536 training points,
d = 90, x = s * z with z ~ N(0, I) and s_k ~ U[0.5, 2], y = random two-layer
tanh network + 0.05 noise; K-balance into p = 16 partitions of 4,096
(k-means++ + 20 Lloyd passes + the capacity pass); the 6 settings
sigma in {0.5, 1, 2} x lambda in {1e-4, 1e-2} fitted as one batch of 96
systems; selection of the best setting on a hold-out set of 6,554 points;
prediction of 8,192 test points with the chosen model (nearest-centre route).

Prints one JSON line.  `value` is fits per second of the batched path in the
requested precision (default: mixed, BF16 trailing updates + FP64 diagonal
blocks + FP64-residual refinement to 1e-6).  Extra fields report the plain
per-partition FP64 sequence, the batched FP64 / FP32 fits, phase times, the
roofline of the dominant kernel and the oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

# The serving leg runs four worker streams beside the main one; with HIP's
# default of four hardware queues per process they share queues and a
# predict launch can wait behind a whole fit kernel.  At least eight queues
# give every stream its own (set before the HIP runtime starts; a larger
# value in the environment is kept).
try:
    _hwq = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
except ValueError:
    _hwq = 4
if _hwq < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

P_PARTS = 16
SIGMAS = (0.5, 1.0, 2.0)
LAMBDAS = (1e-4, 1e-2)
LLOYD = 20
SEED = 2
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}   # dense TFLOP/s, MI355X
HBM_PEAK = 8000.0  # GB/s

# HBM traffic per launch of the roofline kernel, from two rocprofv3 counter
# runs of this benchmark (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch,
# averaged over the kernel's dispatches), each scaled by what the same counter
# reads for a plain 1 GiB device copy (FETCH_SIZE reads 512 MiB: x2.0;
# WRITE_SIZE reads 1 GiB: x1.0).  Valid only for the source they were taken
# on: the sha256 of the kernel's whole source file must match, else the figure
# is reported as null.
TRAFFIC = {
    "chol_column_bf16": {
        "kernel": "k_panel_col",
        "source": "paper_1805_00569_amd/csrc/cholesky.hip",
        "sha256": "a75a9d35cd55ecaa37e06a7a2a8ba64045018d7cd4d7da2887fb98b2f6d30ba0",
        "fetch_kib": 118856.3, "write_kib": 79706.3, "fetch_scale": 2.0, "write_scale": 1.0,
    },
}


def _traffic_bytes(cls):
    import hashlib
    t = TRAFFIC.get(cls)
    if t is None:
        return None
    try:
        with open(os.path.join(ROOT, t["source"]), "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if digest != t["sha256"]:
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


def fit_flops(m, d):
    m = float(m)
    return m ** 3 / 3.0 + m * m * d + m * m / 2.0 + 2.0 * m * m


def predict_flops(m, d):
    return 2.0 * m * d + 3.0 * m


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="mixed", choices=["mixed", "fp64", "fp32"])
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--no-baselines", action="store_true", help="skip the plain/batched comparisons")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing on the host")
    ap.add_argument("--cpu-fits", type=int, default=2, help="oracle fits timed for the CPU baseline")
    ap.add_argument("--panel", type=int, default=0, help="Cholesky panel width in 64-wide tiles (0: library default)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-rates", default="100,500,2000", help="Poisson arrival rates (requests/s)")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="length of each rate's arrival trace")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a design note, "
                                   "not an implemented path", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1805_00569_amd import datagen, krr

    dev = torch.device("cuda:0")
    t0 = time.time()
    w = datagen.balanced(seed=SEED, n=args.n, p=P_PARTS, sigmas=SIGMAS, lambdas=LAMBDAS)
    X = torch.from_numpy(w.X).to(dev)
    y = torch.from_numpy(w.y.astype(np.float32)).to(dev)
    Xv = torch.from_numpy(w.Xv).to(dev)
    yv = torch.from_numpy(w.yv.astype(np.float32)).to(dev)
    Xt = torch.from_numpy(w.Xt).to(dev)
    print(f"# data ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    ctx = krr.Context(0)
    if args.panel:
        ctx.set_option(krr.OPT_PANEL_TILES, args.panel)

    def settings(prec):
        return [krr.Params(sigma=s, lam=l, prec=prec, refine_tol=1e-6, max_refine=30)
                for l in LAMBDAS for s in SIGMAS]   # lambda outer, sigma inner (Algorithm 5 loop)

    params = settings(args.prec)
    n_fits = len(params) * P_PARTS
    state = {}

    def step(prec_params=params, phases=None):
        sync = torch.cuda.synchronize
        ta = time.perf_counter()
        C, a, sz = ctx.partition(X, P_PARTS, "kbalance", lloyd_iters=LLOYD, seed=SEED)
        if phases is not None:
            sync()
            tb = time.perf_counter()
        models, info, st = ctx.fit(X, y, a, C, P_PARTS, prec_params)
        if phases is not None:
            tc = time.perf_counter()
        mse, best = ctx.select(models, Xv, yv)
        if phases is not None:
            td = time.perf_counter()
        yhat = ctx.predict(models[best], Xt)
        if phases is not None:
            sync()
            te = time.perf_counter()
            phases.update(partition=tb - ta, fit=tc - tb, select=td - tc, predict=te - td)
        state.update(info=info, status=st, mse=mse, best=best, sizes=sz, assign=a, C=C)
        for m in models:
            m.free()
        return yhat

    for i in range(args.warmup):
        step()
        print(f"# warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    # HIP events around the matrix-core factorisation updates during the timed
    # steps (the library records them on the stream the kernels run on)
    ctx.set_option(krr.OPT_TIMING, 1)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    timed_kernels = ctx.timing_report()
    ctx.set_option(krr.OPT_TIMING, 0)
    ms = 1e3 * t_total / args.steps
    print(f"# timed {args.steps} steps: {ms:.2f} ms/step", file=sys.stderr, flush=True)

    info = state["info"]
    m_sizes = [r["m"] for r in info]
    d = w.d
    k_val, k_test = w.Xv.shape[0], w.Xt.shape[0]
    flops_fit = sum(fit_flops(m, d) for m in m_sizes)
    m_avg = float(np.mean(m_sizes[:P_PARTS]))
    flops_pred = (len(params) * k_val + k_test) * predict_flops(m_avg, d)
    step_s = ms / 1e3
    out = {
        "metric": "KRR fits/s + TFLOP/s (batched vs plain) at 1e-6 rel err; p50/p99 predict ms",
        "value": n_fits / step_s,
        "unit": "fits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "bf16/f32 updates + f64 panels and residual", "fp64": "f64", "fp32": "f32"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "BKRR2 balanced partitioning: n=65536 train (d=90, x=s*z, s~U[0.5,2]), "
                               "p=16 K-balance partitions of 4096, 3 sigma x 2 lambda = 96 fits per step, "
                               "select on 6554 held-out, predict 8192 test (nearest centre)",
                   "n": args.n, "d": d, "p": P_PARTS, "fits_per_step": n_fits, "precision": args.prec,
                   "sigmas": SIGMAS, "lambdas": LAMBDAS, "lloyd_iters": LLOYD},
        "tflops": (flops_fit + flops_pred) / step_s / 1e12,
        "fit_status": state["status"],
        "max_refine_iters": max(r["refine_iters"] for r in info),
        "fallbacks": sum(r["fallback"] for r in info),
        "max_rel_residual": max(r["rel_residual"] for r in info),
        "best_setting": {"index": state["best"], "sigma": params[state["best"]].sigma,
                         "lambda": params[state["best"]].lam, "val_mse": state["mse"][state["best"]]},
    }

    out["roofline"] = roofline(timed_kernels, args.steps)

    phases = {}
    ctx.set_option(krr.OPT_TIMING, 2)
    step(phases=phases)
    kern = ctx.timing_report()
    ctx.set_option(krr.OPT_TIMING, 0)
    out["phase_ms"] = {k: round(v * 1e3, 3) for k, v in phases.items()}
    out["kernel_ms_per_step"] = {k: round(v["ms"], 3) for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["ms"])}

    # batched vs plain comparisons (fit phase only, same partitions)
    if not args.no_baselines:
        C, a = state["C"], state["assign"]
        comp = {}

        def time_fit(prec, serial, reps=1):
            ctx.set_option(krr.OPT_SERIAL_FIT, 1 if serial else 0)
            try:
                models, info2, st2 = ctx.fit(X, y, a, C, P_PARTS, settings(prec))   # warm
                for m in models:
                    m.free()
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(reps):
                    models, info2, st2 = ctx.fit(X, y, a, C, P_PARTS, settings(prec))
                    for m in models:
                        m.free()
                torch.cuda.synchronize()
                return (time.perf_counter() - t) / reps, info2
            finally:
                ctx.set_option(krr.OPT_SERIAL_FIT, 0)

        for name, prec, serial, reps in (("batched_" + args.prec, args.prec, False, 3),
                                         ("batched_fp64", "fp64", False, 1),
                                         ("batched_fp32", "fp32", False, 1),
                                         ("plain_fp64_per_partition", "fp64", True, 1)):
            if name in comp:
                continue
            tt, inf = time_fit(prec, serial, reps)
            comp[name] = {"fit_ms": round(tt * 1e3, 3), "fits_per_s": n_fits / tt,
                          "tflops": flops_fit / tt / 1e12}
            print(f"# {name}: {tt * 1e3:.1f} ms", file=sys.stderr, flush=True)
        base = comp["plain_fp64_per_partition"]["fit_ms"]
        for k, v in comp.items():
            v["speedup_vs_plain_fp64"] = base / v["fit_ms"]
        out["fit_comparison"] = comp

    # oracle on the host: a bounded sample of the same fits
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, state, ctx, params, args.cpu_fits)

    if not args.no_serve:
        del X, y, Xv, yv, Xt
        torch.cuda.empty_cache()
        out["serving"] = serving_leg([float(r) for r in args.serve_rates.split(",") if r], args.serve_seconds)
        top = out["serving"]["rates"][-1]
        out["p50_predict_ms"] = top["predict_p50_ms"]
        out["p99_predict_ms"] = top["predict_p99_ms"]

    print(json.dumps(out))


def serving_leg(rates, seconds, seed=5):
    """Request loop over a resident BKRR2 model: n=262,144 points (d=90,
    64-component Gaussian mixture) K-balanced into 64 partitions of 4,096 and
    fitted in FP32 (sigma=2, lambda=1e-2).  For each rate, a seeded Poisson
    stream of `seconds` mixes 10% fit requests (m uniform in [256, 8192],
    d in {8, 32, 90}, FP32, same setting) and 90% predict requests (1..1024
    points routed to the nearest of the 64 models), submitted open-loop at
    their arrival times.  Latency = submit to completion, measured by the
    server."""
    import torch
    from paper_1805_00569_amd import datagen, krr
    dev = torch.device("cuda:0")
    t0 = time.time()
    pools = datagen.serving_pools(seed=seed)
    w = pools.resident
    X = torch.from_numpy(w.X).to(dev)
    y = torch.from_numpy(w.y.astype(np.float32)).to(dev)
    ctx = krr.Context(0)
    setting = krr.Params(sigma=2.0, lam=1e-2, prec="fp32")
    C, a, sz = ctx.partition(X, 64, "kbalance", lloyd_iters=LLOYD, seed=seed)
    torch.cuda.synchronize()
    tf = time.perf_counter()
    models, info, st = ctx.fit(X, y, a, C, 64, [setting])
    fit_s = time.perf_counter() - tf
    print(f"# serving: resident model ready ({time.time() - t0:.1f}s, fit {fit_s * 1e3:.1f} ms, status {st})",
          file=sys.stderr, flush=True)
    del X, y
    srv = krr.Server(ctx, models[0], predict_workers=2, fit_workers=2, max_batch_fits=16, max_batch_points=16384,
                     hbm_budget=64 << 30)
    res = {"resident": {"n": w.n, "d": w.d, "p": 64, "partition_size_range": [int(sz.min().item()), int(sz.max().item())], "precision": "fp32",
                        "sigma": 2.0, "lambda": 1e-2, "fit_ms": round(fit_s * 1e3, 3), "fit_status": st},
           "workers": {"predict": 2, "fit": 2, "max_batch_fits": 16, "max_batch_points": 16384},
           "rates": []}
    try:
        # warm the workers' workspaces with one request of each kind and size class
        for fd in (8, 32, 90):
            srv.wait(srv.submit_fit(datagen.take_rows(pools.fit_X[fd], 0, 8192),
                                    datagen.take_rows(pools.fit_y[fd][:, None], 0, 8192)[:, 0], setting))
        for _ in range(4):
            srv.wait(srv.submit_predict(datagen.take_rows(pools.queries, 0, 1024)))
        srv.stats(reset=True)
        for rate in rates:
            trace = datagen.serving_trace(seed=seed, rate=rate, seconds=seconds)
            tickets = []
            start = time.perf_counter()
            for r in trace:
                while time.perf_counter() - start < r.t:
                    pass
                if r.kind == "predict":
                    tickets.append(srv.submit_predict(datagen.take_rows(pools.queries, r.offset, r.rows)))
                else:
                    tickets.append(srv.submit_fit(datagen.take_rows(pools.fit_X[r.d], r.offset, r.rows),
                                                  datagen.take_rows(pools.fit_y[r.d][:, None], r.offset, r.rows)[:, 0],
                                                  setting))
            submit_s = time.perf_counter() - start
            bad = 0
            for tk in tickets:
                try:
                    srv.wait(tk)
                except krr.KrrError:
                    bad += 1
            s = srv.stats(reset=True)
            span = max(s["span_ms"], 1e-9) / 1e3
            n_fit = sum(r.kind == "fit" for r in trace)
            row = {"rate": rate, "requests": len(trace), "fit_requests": n_fit,
                   "achieved_rate": len(trace) / max(submit_s, 1e-9),
                   "predict_p50_ms": s["predict_p50_ms"], "predict_p99_ms": s["predict_p99_ms"],
                   "fit_p50_ms": s["fit_p50_ms"], "fit_p99_ms": s["fit_p99_ms"],
                   "fits_per_s": s["fit_requests"] / span, "predictions_per_s": s["points"] / span,
                   "mean_predict_batch": s["predict_requests"] / max(s["predict_batches"], 1),
                   "mean_fit_batch": s["fit_requests"] / max(s["fit_batches"], 1),
                   "failed": s["failed"] + bad, "max_inflight_bytes": s["max_inflight_bytes"]}
            res["rates"].append(row)
            print(f"# serving rate {rate:g}/s: {len(trace)} requests, predict p50 {row['predict_p50_ms']:.2f} ms "
                  f"p99 {row['predict_p99_ms']:.2f} ms, fit p50 {row['fit_p50_ms']:.1f} ms",
                  file=sys.stderr, flush=True)
    finally:
        srv.close()
        models[0].free()
        ctx.close()
    return res


def roofline(timed, steps):
    """Roofline entry of the kernel class with the most event time in the
    timed steps.  The bound is the one its algorithmic intensity (flops per
    algorithmic HBM byte) puts it under: HBM below the ridge point of the
    class's matrix-core peak, the matrix cores above it.  achieved =
    algorithmic bytes (or flops) of its launches / their summed duration."""
    if not timed:
        return None
    name, rec = max(timed.items(), key=lambda kv: kv[1]["ms"])
    prec = "bf16" if name.endswith("bf16") else ("fp64" if name.endswith("f64") else "fp32")
    sec = rec["ms"] * 1e-3
    flops, byts, cnt = rec["flops"], rec.get("bytes", 0.0), max(rec["count"], 1)
    ridge = PEAK[prec] * 1e12 / (HBM_PEAK * 1e9)
    out = {"kernel": name, "launches_per_step": rec["count"] / steps, "ms_per_step": rec["ms"] / steps,
           "avg_launch_us": 1e3 * rec["ms"] / cnt, "algorithmic_flops_per_launch": flops / cnt,
           "algorithmic_bytes_per_launch": byts / cnt if byts > 0 else None,
           "intensity_flop_per_byte": flops / byts if byts > 0 else None,
           "ridge_flop_per_byte": ridge, "mfma_peak_tflops": PEAK[prec],
           "achieved_tflops": flops / sec / 1e12 if sec > 0 else 0.0}
    if byts > 0 and flops / byts < ridge:
        achieved = byts / sec / 1e9 if sec > 0 else 0.0
        out.update(bound="hbm", achieved=achieved, peak=HBM_PEAK, unit="GB/s", frac=achieved / HBM_PEAK)
    else:
        achieved = flops / sec / 1e12 if sec > 0 else 0.0
        out.update(bound="mfma", achieved=achieved, peak=PEAK[prec], unit="TFLOP/s", frac=achieved / PEAK[prec])
    out["traffic"] = _traffic_bytes(name)
    out["other_timed_classes_ms_per_step"] = {k: v["ms"] / steps for k, v in timed.items() if k != name}
    return {k: out[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")} | \
        {k: v for k, v in out.items() if k not in ("bound", "achieved", "peak", "unit", "frac", "traffic")}


def cpu_baseline(w, state, ctx, params, n_fits):
    import threadpoolctl
    import torch
    import oracle as O
    a = state["assign"].cpu().numpy()
    C = state["C"].cpu().numpy()
    yo = w.y.astype(np.float32).astype(np.float64)
    idx = np.nonzero(a == 0)[0]
    Xj = w.X[idx]
    yj = yo[idx]
    info = threadpoolctl.threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    t = time.perf_counter()
    alphas = []
    for q in range(n_fits):
        r = O.fit_one(Xj, yj, params[q].sigma, params[q].lam)
        alphas.append(r["alpha"])
    dt = time.perf_counter() - t
    m = Xj.shape[0]
    return {"value": n_fits / dt, "unit": "fits/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_fits} fits of partition 0 (m={m}, d={w.d}): direct-difference FP64 kernel "
                      f"+ LAPACK Cholesky, settings {[(params[q].sigma, params[q].lam) for q in range(n_fits)]}",
            "seconds": dt, "cpu": _cpu_name(), "os_cpu_count": os.cpu_count()}


def _cpu_name():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
