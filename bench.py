#!/usr/bin/env python3
"""Benchmark: QMC least-squares American pricing throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 4] [--dtype fp32]

A step is one full pricing call (Sobol -> inverse normal -> bridge -> GBM
paths -> backward induction -> discounted mean) on the configuration's inputs,
enqueued through the C-ABI on one stream with a torch-owned workspace.  Inputs
(paths) are produced on the device by the call itself; nothing crosses PCIe in
the timed region except the 16-byte result of the last step.  Prints one JSON
line.

Default workload: the large single American put S0=100, K=110, r=0.03,
sigma=0.25, T=2, 252 dates, 2^24 Sobol paths, monomials of degree 4, FP32 bulk
with FP64 solve (the largest single-GPU configuration).  Beside it, as extra
keys: the 2^20-path, 100-date weighted-Laguerre put in FP32 bulk and FP64; the
1024-option batch in FP32 bulk against the plain FP64 single-option path over
the same options; a short serving replay (p50/p99).
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
    ap.add_argument("--config", type=int, default=4, choices=[1, 2, 4])
    ap.add_argument("--dtype", default=None, choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-side", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the main workload only (no second workload, batch or serving keys)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the serving replay reported beside the main line "
                         "(the serving workload's own 60 s by default; 0 skips it)")
    ap.add_argument("--paper-table2", action="store_true",
                    help="the paper's Table 2 shape: ten exercise points, 10 .. 10^6 paths, GPU and oracle")
    ap.add_argument("--serve", type=float, default=0.0, metavar="SECONDS",
                    help="serving mode: replay Poisson arrivals (200 req/s) for SECONDS")
    ap.add_argument("--serve-rate", type=float, default=200.0, metavar="REQ_PER_S",
                    help="arrival rate of the serving replay (--serve)")
    ap.add_argument("--serve-large-tile", action="store_true",
                    help="serve with the larger batch tile (--serve)")
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


def serve(seconds, dtype, rate=200.0, large_tile=False):
    """Open-loop replay of seeded Poisson arrivals (`rate` req/s); each request
    is one option drawn as in the batch workload with 2^12-2^20 paths and
    12-365 dates; latency = completion - scheduled arrival (no coordinated
    omission)."""
    import numpy as np
    import paper_1205_0106_amd as amq
    from paper_1205_0106_amd.workloads import batch_options, poisson_arrivals
    arr = poisson_arrivals(rate, seconds)
    specs = batch_options(len(arr), seed=0x12050107, log2_paths=(12.0, 20.0), dates=(12, 365))
    opts = amq.make_options(specs)
    b = amq.make_basis("monomial", 2)
    res = {}
    with amq.Server(64 << 30, b, dtype, n_streams=2, max_batch_requests=64,
                    max_batch_path_steps=4e9, large_tile=large_tile) as srv:
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
        "config": {"workload": f"serving: Poisson {rate:g} req/s for {seconds:g} s, paths 2^12-2^20, "
                               "dates 12-365, HBM admission budget 64 GB", "requests": len(arr),
                   "basis": "monomial degree 2",
                   "batch_tile": "larger (64 paths per thread)" if large_tile else "smaller (16 paths per thread)"},
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
    out = {"metric": "path-steps/s for QMC American pricing (" + ("paper estimator" if args.paper_estimator
                                                                  else "randomised QMC-LSM") + ")",
           "value": total * args.steps / dt, "unit": "path-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
           "dtype": "f64", "storage": "f32" if dtype == "fp32" else "f64", "data": "synthetic (on-device Sobol paths)",
           "config": {"workload": w.name, "variant": what, "path_steps": total},
           "price": float(res[0]), "error_bar": float(res[1])}
    if args.rqmc:
        # the replicates one after another, for comparison with the batch form above
        serial = lambda: pr.price_rqmc(p, n_paths, w.n_dates, b, dtype, shifts, fused=False)
        for _ in range(args.warmup):
            serial()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rs = serial()
        torch.cuda.synchronize()
        ds = time.perf_counter() - t0
        out["replicates_one_after_another"] = {"value": total * args.steps / ds, "ms_per_step": 1e3 * ds / args.steps,
                                               "price": float(rs[0]), "error_bar": float(rs[1])}
    return out


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


def single_run(amq, pricer, w, dtype, steps, warmup):
    """Time `steps` pricing calls of workload w; price and its distance from
    the committed oracle value of the same workload (FP32 bulk: the oracle on
    binary32-stored paths, and the all-binary64 oracle beside it)."""
    p = amq.make_params(**w.params(), is_call=w.is_call, allow_exercise=w.allow_exercise)
    b = amq.make_basis(*w.basis)
    m = time_steps(amq, pricer, p, b, w, dtype, steps, warmup)
    m["value"] = w.n_paths * w.n_dates * steps / m["seconds"]
    gold = os.path.join(ROOT, "tests", "golden", f"oracle_{w.name.split('_')[0]}.json")
    if os.path.exists(gold):
        g = json.load(open(gold))
        ref = g
        if dtype == "fp32" and w.n_paths >= amq.AM_FP32_MIN_PATHS and "store32" in g:
            ref = g["store32"]
            m["abs_err_vs_binary64_oracle"] = abs(m["price"] - g["price"])
        m["oracle_price"] = ref["price"]
        m["abs_err_vs_oracle"] = abs(m["price"] - ref["price"])
    return m


def batch_vs_single(n, steps, warmup):
    """The batched FP32-bulk form against the plain FP64 single-option path on
    the same n options: path-steps/s of each (back-to-back calls on one
    stream between device syncs), and the largest price difference between
    the two (the FP64 single-option prices match the FP64 oracle to 1e-4; the
    difference is the binary32 storage, which moves a few ill-conditioned
    options by more than 2e-3)."""
    import numpy as np
    import torch
    import paper_1205_0106_amd as amq
    from paper_1205_0106_amd.workloads import batch_options
    specs = batch_options(n)
    opts = amq.make_options(specs)
    b = amq.make_basis("monomial", 2)
    total = sum(d["n_paths"] * d["n_dates"] for d in specs)
    pr = amq.Pricer(0)
    for _ in range(warmup):
        pr.price_batch(opts, b, "fp32", wait=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pr.price_batch(opts, b, "fp32", wait=False)
    torch.cuda.synchronize()
    dt32 = (time.perf_counter() - t0) / steps
    p32 = pr.price_batch(opts, b, "fp32")
    pr.ws = None
    torch.cuda.empty_cache()
    one = amq.Pricer(0)
    params = [amq.make_params(d["S0"], d["K"], d["r"], d["sigma"], d["T"], d["is_call"]) for d in specs]
    one.workspace(max(amq.am_workspace_bytes(d["n_paths"], d["n_dates"], b, "fp64") for d in specs))
    for i in range(min(n, 8)):
        one.price(params[i], specs[i]["n_paths"], specs[i]["n_dates"], b, "fp64", wait=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, d in enumerate(specs):
        one.price(params[i], d["n_paths"], d["n_dates"], b, "fp64", wait=False)
    torch.cuda.synchronize()
    dt64 = time.perf_counter() - t0
    p64 = np.array([one.price(params[i], d["n_paths"], d["n_dates"], b, "fp64") for i, d in enumerate(specs)])
    one.ws = None
    torch.cuda.empty_cache()
    diff = np.abs(p32[:, 0] - p64[:, 0])
    return {"workload": f"batch of {n} options: put/call 50/50, K U(80,120), S0 100, sigma U(0.1,0.5), "
                        "r U(0,0.08), T U(0.25,2), dates U{16..256}, paths 2^14-2^18 log-uniform, "
                        "monomials degree 2",
            "path_steps": total,
            "batch_fp32_bulk": {"value": total / dt32, "ms_per_batch": 1e3 * dt32},
            "single_option_fp64": {"value": total / dt64, "ms_for_all": 1e3 * dt64},
            "speedup": dt64 / dt32,
            "max_abs_price_diff": float(diff.max()), "median_abs_price_diff": float(np.median(diff)),
            "n_price_diff_over_2e-3": int((diff > 2e-3).sum()),
            "median_naive_std_err": float(np.median(p64[:, 1])),
            "unit": "path-steps/s"}


def paper_table2(steps):
    """The paper's Table 2 shape (ten exercise points, 10 .. 10^6 paths) on
    config 1's option: GPU (FP64, whole call between device syncs) and the
    oracle (one thread), milliseconds per pricing at each path count."""
    import torch
    import oracle
    import paper_1205_0106_amd as amq
    from paper_1205_0106_amd.workloads import CONFIG1, PAPER_TABLE2_PATHS
    oracle.build(force=not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")))
    w = CONFIG1
    M = 10
    p = amq.make_params(**w.params())
    b = amq.make_basis(*w.basis)
    pr = amq.Pricer(0)
    # the oracle's one-time set-up (direction numbers) outside its timings
    oracle.price_american(**w.params(), N=16, M=M, kind=oracle.MONOMIAL, degree=w.basis[1])
    rows = []
    for N in PAPER_TABLE2_PATHS:
        for _ in range(2):
            pr.price(p, N, M, b, "fp64", wait=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            pr.price(p, N, M, b, "fp64", wait=False)
        torch.cuda.synchronize()
        gpu_ms = 1e3 * (time.perf_counter() - t0) / steps
        price = pr.price(p, N, M, b, "fp64")[0]
        t0 = time.perf_counter()
        r = oracle.price_american(**w.params(), N=N, M=M, kind=oracle.MONOMIAL, degree=w.basis[1])
        cpu_ms = 1e3 * (time.perf_counter() - t0)
        rows.append({"paths": N, "gpu_ms": round(gpu_ms, 4), "oracle_ms": round(cpu_ms, 3),
                     "gpu_price": price, "oracle_price": r.price, "abs_diff": abs(price - r.price)})
    return {"metric": "milliseconds per pricing (the paper's Table 2 shape)",
            "config": {"workload": "put S0 36, K 40, r 0.06, sigma 0.2, T 1, ten exercise dates, "
                                   "monomials degree 2, FP64"},
            "oracle": f"single thread, {cpu_model()}", "rows": rows}


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
        print(json.dumps(serve(args.serve, args.dtype or "fp32", args.serve_rate, args.serve_large_tile)),
              flush=True)
        return
    if args.batch:
        print(json.dumps(batch_run(args.batch, args.dtype or "fp32", args.steps, args.warmup)), flush=True)
        return
    if args.paper_estimator or args.rqmc:
        print(json.dumps(variant_run(args)), flush=True)
        return
    if args.paper_table2:
        print(json.dumps(paper_table2(max(3, args.steps // 4))), flush=True)
        return
    import torch
    import paper_1205_0106_amd as amq
    from paper_1205_0106_amd.workloads import CONFIG2, CONFIGS

    w = CONFIGS[args.config]
    dtype = args.dtype or ("fp32" if "fp32" in w.dtypes else "fp64")
    pricer = amq.Pricer(0)
    path_steps = w.n_paths * w.n_dates
    m = single_run(amq, pricer, w, dtype, args.steps, args.warmup)
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
    # the other kernel against the same roofline
    other = "generate" if dom == "sweep" else "sweep"
    oms = m["gen_ms"] if other == "generate" else m["sweep_ms"]
    roofline_other = {"kernel": other, "bound": "hbm", "achieved": round(alg_bytes / (oms * 1e-3) / 1e9, 1),
                      "peak": PEAK_HBM_GBS, "unit": "GB/s",
                      "frac": round(alg_bytes / (oms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                      "traffic": measured_traffic(args.config, dtype, other), "avg_launch_ms": round(oms, 4)}

    out = {
        "metric": "path-steps/s for QMC-LSM American pricing",
        "value": m["value"],
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * m["seconds"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # arithmetic of the path: FP32 bulk computes in binary64 and stores
        # path values and cashflows in binary32 (each rounded once); FP64 is
        # binary64 throughout
        "dtype": "f64",
        "data": "synthetic (on-device Sobol paths)",
        "config": {"workload": w.name, "n_paths": w.n_paths, "n_dates": w.n_dates,
                   "basis": f"{w.basis[0]} degree {w.basis[1]}",
                   "storage": "f32" if dtype == "fp32" else "f64",
                   "precision": ("FP32 bulk: binary32 storage of path values and cashflows (each rounded "
                                 "once from binary64); binary64 inverse normal, bridge, exponent, "
                                 "regression, solve and sums")
                   if dtype == "fp32" else "FP64 throughout",
                   "S0": w.S0, "K": w.K, "r": w.r, "sigma": w.sigma, "T": w.T},
        "roofline": roofline,
        "roofline_other_kernel": roofline_other,
        "valu_issue": valu_issue(args.config, dtype, {"generate": m["gen_ms"], "sweep": m["sweep_ms"]}),
        "phase_ms": {"generate": round(m["gen_ms"], 4), "sweep": round(m["sweep_ms"], 4)},
        "price": m["price"],
        "std_err": m["std_err"],
    }
    for k in ("oracle_price", "abs_err_vs_oracle", "abs_err_vs_binary64_oracle"):
        if k in m:
            out[k] = m[k]
    if dtype == "fp32" and "fp64" in w.dtypes and not args.no_fp64_side:
        n64 = max(3, args.steps // 4)
        m64 = single_run(amq, pricer, w, "fp64", n64, 1)
        out["fp64_side"] = {"value": m64["value"], "price": m64["price"],
                            "phase_ms": {"generate": round(m64["gen_ms"], 4), "sweep": round(m64["sweep_ms"], 4)},
                            "abs_err_vs_oracle": m64.get("abs_err_vs_oracle")}
    pricer.ws = None
    torch.cuda.empty_cache()
    if not args.no_extras:
        if w is not CONFIG2:
            w2 = CONFIG2
            extra = {"workload": w2.name}
            for d2 in ("fp32", "fp64"):
                m2 = single_run(amq, pricer, w2, d2, args.steps, args.warmup)
                extra[d2] = {"value": m2["value"], "ms_per_step": 1e3 * m2["seconds"] / args.steps,
                             "phase_ms": {"generate": round(m2["gen_ms"], 4), "sweep": round(m2["sweep_ms"], 4)},
                             "price": m2["price"], "abs_err_vs_oracle": m2.get("abs_err_vs_oracle"),
                             "abs_err_vs_binary64_oracle": m2.get("abs_err_vs_binary64_oracle")}
            out["config2"] = extra
            pricer.ws = None
            torch.cuda.empty_cache()
        out["batch_fp32_vs_single_fp64"] = batch_vs_single(1024, max(3, args.steps // 4), 1)
        if args.serve_seconds > 0:
            sv = serve(args.serve_seconds, "fp32")
            out["serving"] = {k: sv[k] for k in ("value", "unit", "p50_ms", "p99_ms", "mean_ms", "completed_ok",
                                                 "batches", "offered_path_steps_per_s")}
            out["serving"]["workload"] = sv["config"]["workload"]
            out["serving"]["requests"] = sv["config"]["requests"]
            # the same mix at ten times the rate for a shorter window: the
            # dispatcher merges waiting requests into batches under load
            hv = serve(min(10.0, max(2.0, args.serve_seconds / 3)), "fp32", rate=2000.0)
            out["serving_2000rps"] = {k: hv[k] for k in ("value", "unit", "p50_ms", "p99_ms", "mean_ms",
                                                         "completed_ok", "batches", "offered_path_steps_per_s")}
            out["serving_2000rps"]["requests"] = hv["config"]["requests"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    out["gpu"] = torch.cuda.get_device_name(0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
