#!/usr/bin/env python3
"""Benchmark: QMC least-squares American pricing throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2] [--dtype fp32]

A step is one full pricing call (Sobol -> inverse normal -> bridge -> GBM
paths -> backward induction -> discounted mean) on the configuration's inputs,
enqueued through the C-ABI on one stream with a torch-owned workspace.  Inputs
(paths) are produced on the device by the call itself; nothing crosses PCIe in
the timed region except the 16-byte result of the last step.  Prints one JSON
line.

Default workload: the single American put S0=K=100, r=0.05, sigma=0.3, T=1,
100 dates, 2^20 Sobol paths, weighted Laguerre degree 3, FP32 bulk with FP64
solve (the FP64 run of the same workload is reported beside it).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E, GB/s
CSRC = os.path.join(ROOT, "paper_1205_0106_amd", "csrc")
KERNEL_SOURCES = ("amq_internal.h", "amq_math.h", "amq_sync.h", "amq_sweep.h", "amq_kernels.hip",
                  "amq_sweep_f32_mono.hip", "amq_sweep_f32_lag.hip", "amq_sweep_f64_mono.hip",
                  "amq_sweep_f64_lag.hip")


def kernel_source_hash() -> str:
    """sha256 over the kernel sources: counter figures taken on other sources
    are not reported."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(config: int, dtype: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    runs (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None when
    those runs were taken on other kernel sources, dtype or workload."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if dtype != "fp32" or not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("source_hash") != kernel_source_hash():
        return None
    k = t["kernels"].get(f"cfg{config}:{'sweep_kernel' if kernel == 'sweep' else 'gen_kernel'}")
    return None if k is None else k["traffic_bytes"]


PEAK_VALU_LANE_PER_S = 256 * 4 * 16 * 2.4e9   # 1024 SIMDs x 16 lanes x 2.4 GHz (binary64 FMA at full rate)


def measured_valu(config: int, dtype: str, kernel: str):
    """Wave-level vector instructions per launch of `kernel` from the committed
    rocprofv3 counter runs (SQ_INSTS_VALU), or None when those runs were taken
    on other kernel sources, dtype or workload."""
    path = os.path.join(ROOT, "profiles", "valu.json")
    if dtype != "fp32" or not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("source_hash") != kernel_source_hash():
        return None
    k = t["kernels"].get(f"cfg{config}:{'sweep_kernel' if kernel == 'sweep' else 'gen_kernel'}")
    return None if k is None else k["valu_wave_instr"]


def valu_issue(config: int, dtype: str, phase_ms: dict):
    """Vector-instruction issue rate of both kernels against the SIMDs' peak:
    counted instructions (profiles) over the launch times measured here."""
    out = {}
    for kernel in ("generate", "sweep"):
        n = measured_valu(config, dtype, kernel)
        if n is None:
            continue
        achieved = n * 64 / (phase_ms[kernel] * 1e-3)
        out[kernel] = {"bound": "alu", "achieved": round(achieved / 1e12, 3),
                       "peak": round(PEAK_VALU_LANE_PER_S / 1e12, 3), "unit": "T lane-instr/s",
                       "frac": round(achieved / PEAK_VALU_LANE_PER_S, 4), "valu_wave_instr_per_launch": n}
    return out or None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 4])
    ap.add_argument("--dtype", default=None, choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-side", action="store_true")
    ap.add_argument("--serve", type=float, default=0.0, metavar="SECONDS",
                    help="serving mode: replay Poisson arrivals (200 req/s) for SECONDS")
    ap.add_argument("--batch", type=int, default=0, metavar="N",
                    help="batch mode: price N options of the seeded batch workload in one call")
    ap.add_argument("--paper-estimator", action="store_true",
                    help="the paper's eqs. (10)-(11) estimator on the workload's paths and dates")
    ap.add_argument("--rqmc", type=int, default=0, metavar="R",
                    help="randomised QMC: R digitally shifted replicates of N/R paths each")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (counter calibration)")
    return ap.parse_args()


def copy_calibration(mib, steps):
    """Plain device copies of a known size: the reference for scaling the
    FETCH_SIZE / WRITE_SIZE counters of the pricing kernels."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"copy_calibration_bytes_read_per_copy": n * 4,
                      "bytes_written_per_copy": n * 4, "copies": steps + 2,
                      "GBps": 2 * n * 4 * steps / dt / 1e9}), flush=True)


def time_steps(amq, pricer, p, b, w, dtype, steps, warmup):
    import torch
    n_bytes = amq.am_workspace_bytes(w.n_paths, w.n_dates, b, dtype)
    ws = pricer.workspace(n_bytes)
    for _ in range(warmup):
        amq.am_price_american_ex(p, w.n_paths, w.n_dates, b, dtype, ws, pricer.stream, wait=False)
    torch.cuda.synchronize()
    amq.am_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        amq.am_price_american_ex(p, w.n_paths, w.n_dates, b, dtype, ws, pricer.stream, wait=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gen_ms, sweep_ms, calls = amq.am_profile_read()
    amq.am_profile_enable(False)
    res = pricer.views(w.n_paths, w.n_dates, b, dtype)["result"].cpu().numpy()
    return dict(seconds=t1 - t0, gen_ms=gen_ms / calls, sweep_ms=sweep_ms / calls,
                price=float(res[0]), std_err=float(res[1]))


def serve(seconds, dtype):
    """Open-loop replay of seeded Poisson arrivals (200 req/s); each request is
    one option drawn as in the batch workload with 2^12-2^20 paths and 12-365
    dates; latency = completion - scheduled arrival (no coordinated omission)."""
    import numpy as np
    import paper_1205_0106_amd as amq
    from paper_1205_0106_amd.workloads import batch_options, poisson_arrivals
    arr = poisson_arrivals(200.0, seconds)
    specs = batch_options(len(arr), seed=0x12050107, log2_paths=(12.0, 20.0), dates=(12, 365))
    opts = amq.make_options(specs)
    b = amq.make_basis("monomial", 2)
    res = {}
    with amq.Server(64 << 30, b, dtype, n_streams=2, max_batch_requests=64,
                    max_batch_path_steps=4e9) as srv:
        # warm-up (kernel loading, schedules) outside the measured window
        for i in range(4):
            srv.submit(opts[i], 10**9 + i)
        while len(res) < 4:
            for r in srv.poll():
                res[r["id"]] = r
        res.clear()
        t0 = srv.now() + 0.05
        i = 0
        while i < len(arr) or len(res) < len(arr):
            now = srv.now()
            while i < len(arr) and t0 + arr[i] <= now:
                srv.submit(opts[i], i, t0 + arr[i])
                i += 1
            for r in srv.poll():
                res[r["id"]] = r
            if i < len(arr):
                wait = t0 + arr[i] - srv.now()
                if wait > 0.0005:
                    time.sleep(min(wait, 0.002))
        st = srv.stats()
    lat = np.array([r["t_done"] - r["t_arrival"] for r in res.values()])
    ok = sum(1 for r in res.values() if r["status"] == 0)
    t_end = max(r["t_done"] for r in res.values())
    steps = sum(d["n_paths"] * d["n_dates"] for d in specs)
    return {
        "metric": "p50/p99 solve latency at fixed QPS; served path-steps/s",
        "value": steps / (t_end - t0), "unit": "path-steps/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f64", "storage": "f32" if dtype == "fp32" else "f64",
        "data": "synthetic (seeded Poisson arrivals and option mix)",
        "config": {"workload": f"serving: Poisson 200 req/s for {seconds:g} s, paths 2^12-2^20, "
                               "dates 12-365, HBM admission budget 64 GB", "requests": len(arr),
                   "basis": "monomial degree 2"},
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3), "completed_ok": ok, "batches": st["batches"],
        "offered_path_steps_per_s": steps / seconds,
    }


def batch_run(n, dtype, steps, warmup):
    import torch
    import paper_1205_0106_amd as amq
    from paper_1205_0106_amd.workloads import batch_options
    specs = batch_options(n)
    opts = amq.make_options(specs)
    b = amq.make_basis("monomial", 2)
    pr = amq.Pricer(0)
    for _ in range(warmup):
        pr.price_batch(opts, b, dtype, wait=False)
    torch.cuda.synchronize()
    amq.am_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        pr.price_batch(opts, b, dtype, wait=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gen_ms, sweep_ms, calls = amq.am_profile_read()
    amq.am_profile_enable(False)
    total = sum(d["n_paths"] * d["n_dates"] for d in specs)
    return {"metric": "path-steps/s for QMC-LSM American pricing (batch)",
            "value": total * steps / dt, "unit": "path-steps/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": 1e3 * dt / steps, "higher_is_better": True,
            "dtype": "f64", "storage": "f32" if dtype == "fp32" else "f64", "data": "synthetic (seeded option mix)",
            "config": {"workload": f"batch of {n} options: put/call 50/50, K U(80,120), S0 100, "
                                   "sigma U(0.1,0.5), r U(0,0.08), T U(0.25,2), dates U{16..256}, "
                                   "paths 2^14-2^18 log-uniform", "path_steps": total},
            "phase_ms": {"generate": gen_ms / calls, "sweep": sweep_ms / calls}}


def variant_run(args):
    """The paper's own estimator, or randomised QMC, on the workload's option,
    dates and total path count; whole-call wall time between device syncs."""
    import numpy as np
    import torch
    import paper_1205_0106_amd as amq
    from paper_1205_0106_amd.workloads import CONFIGS
    w = CONFIGS[args.config]
    dtype = args.dtype or ("fp32" if "fp32" in w.dtypes else "fp64")
    p = amq.make_params(**w.params(), is_call=w.is_call, allow_exercise=w.allow_exercise)
    pr = amq.Pricer(0)
    if args.paper_estimator:
        call = lambda wait: pr.price_paper(p, w.n_paths, w.n_dates, dtype, wait=wait)
        n_paths, what = w.n_paths, "the paper's estimator (eqs. (10)-(11)): Black-Scholes last interval, pathwise maximum"
    else:
        R = args.rqmc
        n_paths = w.n_paths // R
        b = amq.make_basis(*w.basis)
        shifts = np.random.default_rng(20120501).integers(0, 2 ** 32, size=(R, w.n_dates), dtype=np.uint32)
        call = lambda wait: pr.price_rqmc(p, n_paths, w.n_dates, b, dtype, shifts)
        what = f"randomised QMC: {R} digitally shifted replicates of {n_paths} paths, {w.basis[0]} degree {w.basis[1]}"
    for _ in range(args.warmup):
        call(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = call(False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = call(True)
    total = (n_paths * (args.rqmc or 1)) * w.n_dates
    return {"metric": "path-steps/s for QMC American pricing (" + ("paper estimator" if args.paper_estimator
                                                                   else "randomised QMC-LSM") + ")",
            "value": total * args.steps / dt, "unit": "path-steps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
            "dtype": "f64", "storage": "f32" if dtype == "fp32" else "f64", "data": "synthetic (on-device Sobol paths)",
            "config": {"workload": w.name, "variant": what, "path_steps": total},
            "price": float(res[0]), "error_bar": float(res[1])}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(w):
    """The FP64 oracle, single-threaded, on the first paths of the workload."""
    import oracle
    oracle.build(force=not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")))
    # bounded sample, about 5-15 s of single-threaded work: the whole
    # workload up to 2^20 paths, the first 2^19 paths of larger ones
    n = min(w.n_paths, 1 << 19) if w.n_paths > (1 << 20) else w.n_paths
    kind = oracle.LAGUERRE if w.basis[0] == "laguerre" else oracle.MONOMIAL
    t0 = time.perf_counter()
    r = oracle.price_american(**w.params(), N=n, M=w.n_dates, is_call=w.is_call,
                              allow_exercise=w.allow_exercise, kind=kind, degree=w.basis[1])
    dt = time.perf_counter() - t0
    return dict(value=n * w.n_dates / dt, unit="path-steps/s", cores=1, kind="oracle",
                sample=f"first {n} of {w.n_paths} paths x {w.n_dates} dates of the same workload "
                       f"(FP64, single thread, {dt:.1f} s, {cpu_model()}, nproc {os.cpu_count()})",
                price_on_sample=r.price)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                          "(multi-GPU sharding is a design note, not implemented)"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration, args.steps)
        return
    if args.serve:
        print(json.dumps(serve(args.serve, args.dtype or "fp32")), flush=True)
        return
    if args.batch:
        print(json.dumps(batch_run(args.batch, args.dtype or "fp32", args.steps, args.warmup)), flush=True)
        return
    if args.paper_estimator or args.rqmc:
        print(json.dumps(variant_run(args)), flush=True)
        return
    import torch
    import paper_1205_0106_amd as amq
    from paper_1205_0106_amd.workloads import CONFIGS

    w = CONFIGS[args.config]
    dtype = args.dtype or ("fp32" if "fp32" in w.dtypes else "fp64")
    p = amq.make_params(**w.params(), is_call=w.is_call, allow_exercise=w.allow_exercise)
    b = amq.make_basis(*w.basis)
    pricer = amq.Pricer(0)
    path_steps = w.n_paths * w.n_dates

    m = time_steps(amq, pricer, p, b, w, dtype, args.steps, args.warmup)
    value = path_steps * args.steps / m["seconds"]
    s = 4 if dtype == "fp32" else 8

    # dominant kernel and its roofline (algorithmic bytes: generation writes
    # every path value once, the sweep reads every date's slab once)
    alg_bytes = path_steps * s
    if m["sweep_ms"] >= m["gen_ms"]:
        dom, ms = "sweep", m["sweep_ms"]
    else:
        dom, ms = "generate", m["gen_ms"]
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    roofline = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": measured_traffic(args.config, dtype, dom), "traffic_unit": "HBM bytes per launch",
                "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": round(ms, 4)}

    out = {
        "metric": "path-steps/s for QMC-LSM American pricing",
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * m["seconds"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # arithmetic type of the path: binary64 in both modes (FP32 bulk
        # stores path values and cashflows in binary32, see config.storage)
        "dtype": "f64",
        "data": "synthetic (on-device Sobol paths)",
        "config": {"workload": w.name, "n_paths": w.n_paths, "n_dates": w.n_dates,
                   "basis": f"{w.basis[0]} degree {w.basis[1]}",
                   "storage": "f32" if dtype == "fp32" else "f64",
                   "precision": ("FP32 bulk: binary32 path values and cashflows, binary32 inverse normal, "
                                 "binary64 bridge, exponent, regression, solve and sums")
                   if dtype == "fp32" else "FP64 throughout",
                   "S0": w.S0, "K": w.K, "r": w.r, "sigma": w.sigma, "T": w.T},
        "roofline": roofline,
        "valu_issue": valu_issue(args.config, dtype, {"generate": m["gen_ms"], "sweep": m["sweep_ms"]}),
        "phase_ms": {"generate": round(m["gen_ms"], 4), "sweep": round(m["sweep_ms"], 4)},
        "price": m["price"],
        "std_err": m["std_err"],
    }
    gold = os.path.join(ROOT, "tests", "golden", f"oracle_config{args.config}.json")
    if os.path.exists(gold):
        g = json.load(open(gold))
        out["oracle_price"] = g["price"]
        out["abs_err_vs_oracle"] = abs(m["price"] - g["price"])
    if dtype == "fp32" and "fp64" in w.dtypes and not args.no_fp64_side:
        m64 = time_steps(amq, pricer, p, b, w, "fp64", max(3, args.steps // 4), 1)
        out["fp64_side"] = {"value": path_steps * max(3, args.steps // 4) / m64["seconds"],
                            "price": m64["price"], "phase_ms": {"generate": round(m64["gen_ms"], 4),
                                                               "sweep": round(m64["sweep_ms"], 4)}}
        if "oracle_price" in out:
            out["fp64_side"]["abs_err_vs_oracle"] = abs(m64["price"] - out["oracle_price"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    out["gpu"] = torch.cuda.get_device_name(0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
