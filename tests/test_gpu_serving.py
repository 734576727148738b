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
                                  M=d["n_dates"], is_call=d["is_call"], kind=orc.MONOMIAL, degree=2)
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
