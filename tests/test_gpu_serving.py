"""Serving (continuous batching): requests that arrive while others run are
admitted as streams and pool memory free up; every result equals the same
request priced alone (bitwise) and matches the oracle."""
import sys
import time

import numpy as np
import pytest

from paper_1205_0106_amd.workloads import batch_options

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def amq():
    import torch
    import paper_1205_0106_amd as amq
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    amq.lib()
    return amq


def _collect(srv, n, timeout=120.0):
    got = {}
    t0 = time.time()
    while len(got) < n:
        for r in srv.poll():
            got[r["id"]] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"only {len(got)} of {n} results")
        time.sleep(0.001)
    return got


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_serving_mix_equals_alone_and_oracle(amq, orc, dtype):
    # FP32 at the workload's 2^14 path floor and above (a single flipped
    # exercise decision is worth up to (largest payoff)/N)
    lo = 10.0 if dtype == "fp64" else 14.0
    specs = batch_options(40, seed=21, log2_paths=(lo, 15.0), dates=(12, 60))
    b = amq.make_basis("monomial", 2)
    opts = amq.make_options(specs)
    # a small pool forces admission to wait for memory; two streams overlap
    with amq.Server(256 << 20, b, dtype, n_streams=2, max_batch_requests=8) as srv:
        for i in range(len(specs)):
            srv.submit(opts[i], i)
            if i % 5 == 4:
                time.sleep(0.002)          # arrivals while earlier batches run
        mix = _collect(srv, len(specs))
        st = srv.stats()
        log(f"  {dtype}: {st['batches']:.0f} batches for {st['requests']:.0f} requests")
        assert st["batches"] > 1
        for i in (0, 7, 19, 39):
            srv.submit(opts[i], 1000 + i)
        alone = _collect(srv, 4)
    for i in (0, 7, 19, 39):
        assert alone[1000 + i]["price"] == mix[i]["price"], i
    tol = 1e-4 if dtype == "fp64" else 2e-3
    for i in range(0, 40, 3):
        d = specs[i]
        want = orc.price_american(d["S0"], d["K"], d["r"], d["sigma"], d["T"], N=d["n_paths"],
                                  M=d["n_dates"], is_call=d["is_call"], kind=orc.MONOMIAL, degree=2,
                                  store32=dtype == "fp32" and d["n_paths"] >= amq.AM_FP32_MIN_PATHS)
        assert mix[i]["status"] == 0
        assert abs(mix[i]["price"] - want.price) <= tol, (i, mix[i]["price"], want.price)
    lat = np.array([r["t_done"] - r["t_arrival"] for r in mix.values()])
    log(f"  latency p50 {np.percentile(lat, 50) * 1e3:.2f} ms p99 {np.percentile(lat, 99) * 1e3:.2f} ms")


def test_serving_refuses_request_larger_than_budget(amq):
    b = amq.make_basis("monomial", 2)
    big = amq.make_options([dict(S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, n_paths=1 << 20,
                                 n_dates=200)])
    with amq.Server(64 << 20, b, "fp32") as srv:
        srv.submit(big[0], 7)
        r = _collect(srv, 1)[7]
    assert r["status"] == amq.AM_ENOMEM


def test_serving_fp32_small_paths(amq, orc):
    # the served workload's lower path range, FP32 bulk: requests below
    # AM_FP32_MIN_PATHS paths run in a binary64 part of their batch; every
    # result within the FP32-bulk tolerance of the oracle on the same storage
    specs = batch_options(24, seed=31, log2_paths=(12.0, 14.6), dates=(12, 40))
    assert any(d["n_paths"] < amq.AM_FP32_MIN_PATHS for d in specs)
    b = amq.make_basis("monomial", 2)
    opts = amq.make_options(specs)
    with amq.Server(256 << 20, b, "fp32", n_streams=2, max_batch_requests=6) as srv:
        for i in range(len(specs)):
            srv.submit(opts[i], i)
        got = _collect(srv, len(specs))
    worst = 0.0
    for i, d in enumerate(specs):
        want = orc.price_american(d["S0"], d["K"], d["r"], d["sigma"], d["T"], N=d["n_paths"],
                                  M=d["n_dates"], is_call=d["is_call"], kind=orc.MONOMIAL, degree=2,
                                  store32=d["n_paths"] >= amq.AM_FP32_MIN_PATHS)
        assert got[i]["status"] == 0
        err = abs(got[i]["price"] - want.price)
        worst = max(worst, err)
        assert err <= 2e-3, (i, d, got[i]["price"], want.price)
    log(f"  worst |served - oracle| = {worst:.3e}")


@pytest.mark.parametrize("large_tile", [False, True])
@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_serving_request_larger_than_a_stream_share(amq, dtype, large_tile):
    # eight streams: a 2^20-path request needs more sweep groups than one
    # stream's share of the device, so it runs alone on the whole device;
    # the smaller requests around it are served as usual, and every result is
    # the batch result of the request alone (same tile: the server's smaller
    # or larger one)
    b = amq.make_basis("monomial", 2)
    specs = batch_options(6, seed=37, log2_paths=(14.0, 15.0), dates=(12, 30))
    big = dict(S0=100.0, K=105.0, r=0.03, sigma=0.25, T=1.0, is_call=False, n_paths=1 << 20, n_dates=24)
    specs = specs[:2] + [big] + specs[2:4] + [dict(big, K=95.0, is_call=True)] + specs[4:]
    opts = amq.make_options(specs)
    with amq.Server(8 << 30, b, dtype, n_streams=8, max_batch_requests=4, large_tile=large_tile) as srv:
        for i in range(len(specs)):
            srv.submit(opts[i], i)
        got = _collect(srv, len(specs))
    pr = amq.Pricer(0)
    amq.am_debug_set_batch_ppt((64 if large_tile else 16) if dtype == "fp32" else (32 if large_tile else 8))
    try:
        for i, d in enumerate(specs):
            assert got[i]["status"] == 0, (i, got[i])
            alone = pr.price_batch(amq.make_options([d]), b, dtype)
            assert got[i]["price"] == alone[0, 0], (i, got[i]["price"], alone[0, 0])
    finally:
        amq.am_debug_set_batch_ppt(0)



@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_serving_burst_is_merged(amq, dtype):
    # a burst of requests arriving together: the dispatcher merges waiting
    # requests into batches (far fewer batches than requests), and every
    # result is still the request's result alone (batch tiles are per option)
    lo = 12.0 if dtype == "fp64" else 14.0
    specs = batch_options(64, seed=41, log2_paths=(lo, 15.0), dates=(12, 40))
    b = amq.make_basis("monomial", 2)
    opts = amq.make_options(specs)
    with amq.Server(1 << 30, b, dtype, n_streams=2, max_batch_requests=32) as srv:
        for i in range(len(specs)):
            srv.submit(opts[i], i)
        got = _collect(srv, len(specs))
        st = srv.stats()
    log(f"  {dtype}: {st['batches']:.0f} batches for {st['requests']:.0f} requests")
    assert st["requests"] == len(specs) and st["batches"] <= len(specs) // 4
    for i in range(0, 64, 9):
        with amq.Server(1 << 30, b, dtype, n_streams=1, max_batch_requests=1) as one:
            one.submit(opts[i], 0)
            alone = _collect(one, 1)[0]
        assert got[i]["status"] == 0 and got[i]["price"] == alone["price"], (i, got[i], alone)
