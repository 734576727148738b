"""GPU parity of the batched path: many options with uneven path and date
counts in one generation launch and one persistent sweep.  Each option must
match the oracle to the single-option tolerance (FP32-bulk options that store
binary32 paths: the oracle on binary32-rounded paths), and be bitwise the same
priced alone (a batch of one) and in the mix."""
import sys

import numpy as np
import pytest

from paper_1205_0106_amd.workloads import batch_options

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-4, "fp32": 2e-3}


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


@pytest.fixture(scope="module")
def pricer(amq):
    return amq.Pricer(0)


def _small_mix(n=24, seed=7, dtype="fp64"):
    # The batch workload's distribution with fewer dates so the oracle is
    # quick.  FP64 runs also take path counts below the workload's 2^14 floor;
    # FP32 runs stay at 2^14-2^15 (binary32 storage).
    lo, hi = (9.0, 13.0) if dtype == "fp64" else (14.0, 15.0)
    return batch_options(n, seed=seed, log2_paths=(lo, hi), dates=(3, 40))


def _want(amq, orc, d, dtype, degree=2, store32=None):
    """The oracle's price for one option of a batch priced in `dtype`."""
    if store32 is None:
        store32 = dtype == "fp32" and d["n_paths"] >= amq.AM_FP32_MIN_PATHS
    return orc.price_american(d["S0"], d["K"], d["r"], d["sigma"], d["T"], N=d["n_paths"],
                              M=d["n_dates"], is_call=d["is_call"], kind=orc.MONOMIAL, degree=degree,
                              store32=store32)


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_batch_matches_oracle(amq, orc, pricer, dtype):
    specs = _small_mix(dtype=dtype)
    opts = amq.make_options(specs)
    b = amq.make_basis("monomial", 2)
    log(f"  batch of {len(specs)} ({dtype})")
    got = pricer.price_batch(opts, b, dtype)
    worst = 0.0
    for i, d in enumerate(specs):
        want = _want(amq, orc, d, dtype)
        err = abs(got[i, 0] - want.price)
        worst = max(worst, err)
        assert err <= TOL[dtype], (i, d, got[i], want.price)
    log(f"    worst |gpu - oracle| = {worst:.3e}")


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_batch_alone_equals_in_mix(amq, pricer, dtype):
    specs = _small_mix(16, seed=11, dtype=dtype)
    b = amq.make_basis("laguerre", 3)
    mix = pricer.price_batch(amq.make_options(specs), b, dtype)
    for i in (0, 5, 15):
        alone = pricer.price_batch(amq.make_options([specs[i]]), b, dtype)
        assert alone[0, 0] == mix[i, 0] and alone[0, 1] == mix[i, 1]
    # and close to the single-option entry point (different tile shape)
    p = amq.make_params(specs[3]["S0"], specs[3]["K"], specs[3]["r"], specs[3]["sigma"], specs[3]["T"],
                        specs[3]["is_call"])
    single = pricer.price(p, specs[3]["n_paths"], specs[3]["n_dates"], b, dtype)
    assert abs(single[0] - mix[3, 0]) <= TOL[dtype]


def test_batch_deterministic_and_tile_choice(amq, pricer):
    specs = _small_mix(12, seed=3, dtype="fp32")
    opts = amq.make_options(specs)
    b = amq.make_basis("monomial", 3)
    a = pricer.price_batch(opts, b, "fp32")
    assert np.array_equal(a, pricer.price_batch(opts, b, "fp32"))
    amq.am_debug_set_batch_ppt(16)
    try:
        c = pricer.price_batch(opts, b, "fp32")
    finally:
        amq.am_debug_set_batch_ppt(0)
    assert np.abs(a - c)[:, 0].max() <= TOL["fp32"]


def test_batch_full_distribution_sample(amq, orc, pricer):
    # the batch workload's real size range on a seeded sample of 64 options
    specs = batch_options(64)
    opts = amq.make_options(specs)
    b = amq.make_basis("monomial", 2)
    got = pricer.price_batch(opts, b, "fp32")
    for i in (0, 17, 63):
        d = specs[i]
        want = _want(amq, orc, d, "fp32")
        log(f"    opt {i}: N={d['n_paths']} M={d['n_dates']} gpu {got[i, 0]:.6f} oracle {want.price:.6f}")
        assert abs(got[i, 0] - want.price) <= TOL["fp32"]


def test_batch_autotune_and_graph_replay(amq, orc, pricer):
    import torch
    specs = _small_mix(20, seed=13, dtype="fp32")
    opts = amq.make_options(specs)
    b = amq.make_basis("monomial", 2)
    ref = pricer.price_batch(opts, b, "fp32")
    ws = pricer.workspace(amq.am_batch_workspace_bytes(opts, b, "fp32"))
    best, ms = amq.am_batch_autotune(opts, b, "fp32", ws, pricer.stream)
    log(f"  autotune: best ppt {best}, ms {ms}")
    assert best in (16, 64) and all(m > 0 for m in ms)
    tuned = pricer.price_batch(opts, b, "fp32")
    # each tile shape is an FP32 result within tolerance of the oracle
    for i, d in enumerate(specs):
        want = _want(amq, orc, d, "fp32")
        assert abs(ref[i, 0] - want.price) <= TOL["fp32"], (i, ref[i, 0], want.price)
        assert abs(tuned[i, 0] - want.price) <= TOL["fp32"], (i, tuned[i, 0], want.price)
    amq.am_debug_set_batch_ppt(64)
    try:
        g = amq.BatchGraph(opts, b, "fp32", ws)
        eager = pricer.price_batch(opts, b, "fp32")
        for _ in range(3):
            g.launch(pricer.stream)
            got = g.results()
            assert np.array_equal(got, eager)
            torch.cuda.synchronize()
            x = torch.ones(1 << 20, device="cuda").sum().item()   # eager work between replays
            assert x == float(1 << 20)
        g.close()
    finally:
        amq.am_debug_set_batch_ppt(0)


def test_batch_fp32_small_paths(amq, orc, pricer):
    # the served workload's lower path range (2^12 and up): options below
    # AM_FP32_MIN_PATHS paths form a sub-batch stored in binary64.  Every
    # option meets the FP32-bulk tolerance, and each small option is bitwise
    # its result in an FP64 batch
    specs = batch_options(24, seed=29, log2_paths=(12.0, 14.6), dates=(3, 40))
    small = [i for i, d in enumerate(specs) if d["n_paths"] < amq.AM_FP32_MIN_PATHS]
    log(f"  {len(small)} of {len(specs)} options below {amq.AM_FP32_MIN_PATHS} paths")
    assert 0 < len(small) < len(specs)
    b = amq.make_basis("monomial", 2)
    got = pricer.price_batch(amq.make_options(specs), b, "fp32")
    worst = 0.0
    for i, d in enumerate(specs):
        want = _want(amq, orc, d, "fp32")
        err = abs(got[i, 0] - want.price)
        worst = max(worst, err)
        assert err <= TOL["fp32"], (i, d, got[i], want.price)
    log(f"    worst |gpu - oracle| = {worst:.3e}")
    g64 = pricer.price_batch(amq.make_options([specs[i] for i in small]), b, "fp64")
    for j, i in enumerate(small):
        assert got[i, 0] == g64[j, 0] and got[i, 1] == g64[j, 1], i


def test_batch_fp32_many_dates_ill_conditioned(amq, orc, pricer):
    # options of the batch workload with 134-255 dates whose exercise
    # decisions react to single-ulp changes of the binary32 path values
    # (price moves of up to 7e-2 from a binary32 inverse normal).  Each must
    # meet the oracle on binary32-stored paths; two of them sit farther than
    # the tolerance from the all-binary64 oracle, which is the storage
    # precision itself, not the kernels
    full = batch_options(1024)
    pick = [813, 105, 732, 18, 749]
    specs = [full[i] for i in pick]
    b = amq.make_basis("monomial", 2)
    got = pricer.price_batch(amq.make_options(specs), b, "fp32")
    for j, d in enumerate(specs):
        want = _want(amq, orc, d, "fp32")
        log(f"    opt {pick[j]}: N={d['n_paths']} M={d['n_dates']} gpu {got[j, 0]:.8f} "
            f"oracle(binary32 paths) {want.price:.8f} |err| {abs(got[j, 0] - want.price):.2e}")
        assert abs(got[j, 0] - want.price) <= TOL["fp32"], (pick[j], got[j], want.price)
    # the same options on the single-option entry point
    for j in (0, 3):
        d = specs[j]
        p = amq.make_params(d["S0"], d["K"], d["r"], d["sigma"], d["T"], d["is_call"])
        single = pricer.price(p, d["n_paths"], d["n_dates"], b, "fp32")[0]
        want = _want(amq, orc, d, "fp32")
        assert abs(single - want.price) <= TOL["fp32"], (pick[j], single, want.price)


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_batch_long_date_counts(amq, orc, pricer, dtype):
    # options up to the engine's date limit in one batch with a short one:
    # the generator's LDS then holds the longest option's lane tables, block
    # words and schedule (compact tail staging, fewer groups per CU); every
    # option still meets the oracle, and the short one prices as it does alone.
    # (r = sigma^2 / 2 with S0 = K would put paths exactly at the strike:
    # test_gpu_parity.py::test_zero_drift_at_the_money_ties covers that case.)
    n = 1 << 14
    mmax = amq.am_max_dates()
    specs = [dict(S0=100.0, K=105.0, r=0.03, sigma=0.25, T=1.0, is_call=False, n_paths=n, n_dates=mmax),
             dict(S0=100.0, K=95.0, r=0.05, sigma=0.3, T=2.0, is_call=True, n_paths=n, n_dates=400),
             dict(S0=100.0, K=100.0, r=0.03, sigma=0.2, T=0.5, is_call=False, n_paths=2 * n, n_dates=300),
             dict(S0=100.0, K=110.0, r=0.04, sigma=0.35, T=1.5, is_call=False, n_paths=n, n_dates=12)]
    b = amq.make_basis("monomial", 2)
    log(f"  batch with {mmax}, 400, 300 and 12 dates ({dtype})")
    got = pricer.price_batch(amq.make_options(specs), b, dtype)
    for i, d in enumerate(specs):
        want = _want(amq, orc, d, dtype)
        log(f"    opt {i}: N={d['n_paths']} M={d['n_dates']} gpu {got[i, 0]:.8f} oracle {want.price:.8f}")
        assert abs(got[i, 0] - want.price) <= TOL[dtype], (i, got[i], want.price)
    alone = pricer.price_batch(amq.make_options([specs[3]]), b, dtype)
    assert alone[0, 0] == got[3, 0] and alone[0, 1] == got[3, 1]
