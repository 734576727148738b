"""GPU parity: the HIP path against the CPU oracle on identical points.

Every call goes through the C-ABI (paper_1205_0106_amd binding).  Integer
work (Sobol points, in-the-money counts) must match bit for bit; prices within
1e-4 absolute in FP64 mode and 2e-3 in FP32-bulk mode; per-path values to the
tolerance their arithmetic allows.  FP32-bulk requests that store binary32
paths are checked against the oracle on the same storage (its path values
rounded to binary32, everything else binary64); their distance from the
all-binary64 oracle is logged beside it.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_1205_0106_amd import AM_FP32_MIN_PATHS
from paper_1205_0106_amd.workloads import CONFIG1, CONFIG2, CONFIG4

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
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


def _kind(orc, name):
    return orc.LAGUERRE if name == "laguerre" else orc.MONOMIAL


def gpu_price(amq, pricer, w=None, *, N=None, M=None, dtype="fp64", basis=None, is_call=None,
              allow_exercise=None, **over):
    kw = dict(w.params()) if w is not None else {}
    kw.update(over)
    N = N if N is not None else w.n_paths
    M = M if M is not None else w.n_dates
    basis = basis if basis is not None else w.basis
    is_call = is_call if is_call is not None else (w.is_call if w is not None else False)
    allow_exercise = allow_exercise if allow_exercise is not None else \
        (w.allow_exercise if w is not None else True)
    p = amq.make_params(kw["S0"], kw["K"], kw["r"], kw["sigma"], kw["T"], is_call, allow_exercise)
    b = amq.make_basis(*basis)
    log(f"  gpu: N={N} M={M} dtype={dtype} basis={basis} call={is_call} ex={allow_exercise} {kw}")
    price, se = pricer.price(p, N, M, b, dtype)
    v = pricer.views(N, M, b, dtype)
    return price, se, v


def stores32(dtype, N):
    """Whether a request of this precision and path count stores binary32."""
    return dtype == "fp32" and N >= AM_FP32_MIN_PATHS


def oracle_price(orc, w=None, *, N=None, M=None, basis=None, is_call=None, allow_exercise=None,
                 dtype="fp64", **over):
    kw = dict(w.params()) if w is not None else {}
    kw.update(over)
    N = N if N is not None else w.n_paths
    M = M if M is not None else w.n_dates
    basis = basis if basis is not None else w.basis
    is_call = is_call if is_call is not None else (w.is_call if w is not None else False)
    allow_exercise = allow_exercise if allow_exercise is not None else \
        (w.allow_exercise if w is not None else True)
    return orc.price_american(**kw, N=N, M=M, is_call=is_call, allow_exercise=allow_exercise,
                              kind=_kind(orc, basis[0]), degree=basis[1], detail=True,
                              store32=stores32(dtype, N))


def ulps32(got, want):
    """Distance in binary32 ulps between stored binary32 values and the
    binary64 values rounded to binary32 (positive values)."""
    g = np.asarray(got, dtype=np.float32).view(np.int32).astype(np.int64)
    w = np.asarray(want, dtype=np.float64).astype(np.float32).view(np.int32).astype(np.int64)
    return np.abs(g - w)


def check_stored32(got, want, what):
    # each binary32 value is the binary64 path value rounded once: equal to the
    # oracle's value rounded to binary32 except where the two binary64 values
    # straddle a rounding boundary (one ulp)
    u = ulps32(got, want)
    log(f"  {what}: binary32 values off by one ulp: {int((u != 0).sum())} of {u.size}")
    assert u.max() <= 1
    assert (u != 0).mean() <= 1e-4


# --------------------------------------------------------------------------
# Generation: Sobol integers, inverse normal, paths
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dims,N", [(1, 100), (50, 16384), (100, 4097), (252, 3000), (365, 1000),
                                    (7, 64 * 33 + 5)])
def test_sobol_integers_bit_exact(amq, orc, dims, N):
    log(f"sobol dims={dims} N={N}")
    got = amq.am_debug_generate(1, None, N, dims, "fp32")
    want = orc.sobol_block(dims, 1, N).T          # path i uses index i + 1
    assert np.array_equal(got, want)


def test_sobol_integers_large_index(amq, orc):
    # enough paths that waves walk many 64-point blocks (Gray-code carries)
    N, dims = 1 << 18, 3
    got = amq.am_debug_generate(1, None, N, dims, "fp32")
    for first in (0, 4095, 65535, 131071, N - 300):
        want = orc.sobol_block(dims, first + 1, 300).T
        assert np.array_equal(got[:, first:first + 300], want)


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_inverse_normal(amq, orc, dtype):
    # binary64 normals for both storage precisions
    N, dims = 4096, 20
    z = amq.am_debug_generate(2, None, N, dims, dtype)
    x = orc.sobol_block(dims, 1, N).T
    want = np.vectorize(orc.inv_normal_u32)(x)
    err = np.abs(z - want)
    log(f"  max |z - oracle| ({dtype}) = {err.max():.3e}")
    assert err.max() <= 1e-13 * np.abs(want).max()


# binary32 paths are the binary64 normal, bridge and exponent rounded once
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("M", [1, 2, 3, 17, 50, 252])
def test_paths_match_oracle(amq, orc, dtype, M):
    N = 4000
    p = amq.make_params(36.0, 40.0, 0.06, 0.2, 1.0)
    got = amq.am_debug_generate(0, p, N, M, dtype)
    want = orc.paths(36.0, 40.0, 0.06, 0.2, 1.0, N, M)
    if dtype == "fp32":
        check_stored32(got, want, f"paths M={M}")
    else:
        rel = np.abs(got - want) / want
        log(f"  paths M={M} {dtype}: max rel err {rel.max():.3e}")
        assert rel.max() <= 1e-12


# --------------------------------------------------------------------------
# Prices on the configurations
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_config1_price_and_paths(amq, orc, pricer, dtype):
    w = CONFIG1
    price, se, v = gpu_price(amq, pricer, w, dtype=dtype)
    ores, od = oracle_price(orc, w, dtype=dtype)
    err = abs(price - ores.price)
    log(f"config1 {dtype}: gpu {price:.10f} oracle {ores.price:.10f} |err| {err:.3e} se {se:.4e}")
    if dtype == "fp32":
        log(f"  vs the all-binary64 oracle: |err| {abs(price - oracle_price(orc, w)[0].price):.3e}")
    assert err <= TOL[dtype]
    assert abs(se - ores.std_err) <= 0.02 * ores.std_err
    want = orc.paths(**w.params(), N=w.n_paths, M=w.n_dates)
    if dtype == "fp32":
        check_stored32(v["S"].cpu().numpy(), want, "config1 paths")
    else:
        S = v["S"].cpu().numpy()
        assert np.abs(S - want).max() / want.max() <= 1e-12
    rec = v["rec"].cpu().numpy()
    nitm = rec[1:w.n_dates, 9].astype(np.int64)
    diff = np.abs(nitm - od["nitm"][1:w.n_dates])
    assert diff.max() <= (0 if dtype == "fp64" else 1)
    # per-path cashflows: binary32 storage holds each discounted payoff
    # rounded once
    pv = v["PV"].cpu().numpy().astype(np.float64)
    bad = np.abs(pv - od["pv"]) > (1e-10 if dtype == "fp64" else 1e-7) * np.maximum(1.0, od["pv"])
    log(f"  per-path PV mismatches: {bad.sum()} of {w.n_paths}")
    assert bad.mean() <= 1e-3


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_zero_drift_at_the_money_ties(amq, orc, pricer, dtype):
    # S0 = K and r = sigma^2 / 2: the log-price drift is zero, so every path
    # whose bridge noise is zero at a date (Sobol coordinates exactly 1/2)
    # sits exactly at the strike there, and its in-the-money test (h > 0
    # strictly) is decided by the last ulp of the exponential, which differs
    # between the kernel's and the C library's.  Such a tie moves the
    # regression of its date and, through it, decisions of other paths, so
    # the parity that is unique here is: the paths agree to rounding, and the
    # backward induction on the kernel's own paths is the oracle's.
    N, M = 1 << 15, 40
    prm = dict(S0=100.0, K=100.0, r=0.02, sigma=0.2, T=0.5)
    p = amq.make_params(**prm)
    b = amq.make_basis("monomial", 2)
    price = pricer.price(p, N, M, b, dtype)[0]
    v = pricer.views(N, M, b, dtype)
    S = v["S"].cpu().numpy().astype(np.float64)
    want = orc.paths(**prm, N=N, M=M)
    if dtype == "fp32":
        check_stored32(S, want, "zero-drift paths")
    else:
        assert (np.abs(S - want) / want).max() <= 1e-12
    ties = int((np.abs(want - prm["K"]) <= 1e-12 * prm["K"]).sum())
    same = orc.lsm_on_paths(S, **prm, kind=orc.MONOMIAL, degree=2, store32=(dtype == "fp32"))
    own = orc.price_american(**prm, N=N, M=M, kind=orc.MONOMIAL, degree=2, store32=(dtype == "fp32"))
    log(f"  {dtype}: {ties} path-dates at the strike; gpu {price:.10f}, oracle on the gpu's paths "
        f"{same.price:.10f}, oracle on its own paths {own.price:.10f}")
    assert ties > 0
    assert abs(price - same.price) <= (1e-10 if dtype == "fp64" else 1e-7)


def golden(cid, dtype):
    """Stored oracle results for a full-size configuration (written by
    tests/golden/make_oracle_goldens.py, which calls only the oracle): the
    all-binary64 result, and under "store32" the result on binary32-stored
    paths."""
    path = os.path.join(GOLDEN, f"oracle_config{cid}.json")
    if not os.path.exists(path):
        pytest.skip(f"oracle_config{cid}.json not generated (tests/golden/make_oracle_goldens.py {cid})")
    g = json.load(open(path))
    if dtype == "fp32":
        assert "store32" in g, f"oracle_config{cid}.json lacks the binary32-storage result"
        return g, g["store32"]
    return g, g


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_config2_full_size(amq, orc, pricer, dtype):
    w = CONFIG2
    g64, g = golden(2, dtype)
    price, se, v = gpu_price(amq, pricer, w, dtype=dtype)
    err = abs(price - g["price"])
    log(f"config2 {dtype}: gpu {price:.10f} oracle {g['price']:.10f} |err| {err:.3e} "
        f"(all-binary64 oracle {abs(price - g64['price']):.3e})")
    assert err <= TOL[dtype]
    rec = v["rec"].cpu().numpy()
    nitm = rec[1:w.n_dates, 9].astype(np.int64)
    diff = np.abs(nitm - np.array(g["n_itm"][1:w.n_dates]))
    assert diff.max() <= (0 if dtype == "fp64" else 1)
    # sampled paths, computed one by one by the oracle
    S = v["S"]
    for first in (0, 123457, w.n_paths - 257):
        want = orc.paths_range(**w.params(), first=first, count=257, M=w.n_dates)
        got = S[:, first:first + 257].cpu().numpy()
        if dtype == "fp32":
            check_stored32(got, want, f"config2 paths from {first}")
        else:
            assert np.abs(got - want).max() / want.max() <= 1e-12


def test_config4_full_size_fp32(amq, orc, pricer):
    g64, g = golden(4, "fp32")
    w = CONFIG4
    price, se, v = gpu_price(amq, pricer, w, dtype="fp32")
    err = abs(price - g["price"])
    log(f"config4 fp32: gpu {price:.10f} oracle {g['price']:.10f} |err| {err:.3e} "
        f"(all-binary64 oracle {abs(price - g64['price']):.3e})")
    assert err <= TOL["fp32"]
    S = v["S"]
    for first in (0, (1 << 23) + 77, w.n_paths - 129):
        want = orc.paths_range(**w.params(), first=first, count=129, M=w.n_dates)
        check_stored32(S[:, first:first + 129].cpu().numpy(), want, f"config4 paths from {first}")
    # per-date in-the-money counts: the same binary32 values on both sides
    nitm = v["rec"].cpu().numpy()[1:w.n_dates, 9].astype(np.int64)
    diff = np.abs(nitm - np.array(g["n_itm"][1:w.n_dates], dtype=np.int64))
    log(f"  config4 itm counts: max |gpu - oracle| = {diff.max()} (of up to {max(g['n_itm'])})")
    assert diff.max() <= 1


# --------------------------------------------------------------------------
# Edge cases
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N,M", [(4, 3), (10, 1), (63, 2), (64, 5), (65, 7), (1000, 17),
                                 (4097, 12), (33001, 9), (70000, 3)])
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_ragged_sizes(amq, orc, pricer, N, M, dtype):
    kw = dict(S0=100.0, K=105.0, r=0.04, sigma=0.25, T=0.75)
    price, se, v = gpu_price(amq, pricer, None, N=N, M=M, dtype=dtype, basis=("monomial", 2), **kw)
    ores, od = oracle_price(orc, None, N=N, M=M, basis=("monomial", 2), dtype=dtype, **kw)
    log(f"  N={N} M={M} {dtype}: gpu {price:.10f} oracle {ores.price:.10f}")
    # FP32-bulk requests below AM_FP32_MIN_PATHS paths are stored in binary64
    want_storage = amq.AM_FP64 if (dtype == "fp64" or N < amq.AM_FP32_MIN_PATHS) else amq.AM_FP32_BULK
    assert amq.am_storage_dtype(N, dtype) == want_storage
    assert v["S"].element_size() == (8 if want_storage == amq.AM_FP64 else 4)
    assert abs(price - ores.price) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("M", [365, "max"])
def test_many_dates_up_to_the_maximum(amq, orc, pricer, dtype, M):
    # the serving workload's longest schedules and the engine's date limit:
    # bridge depth, Sobol dimensions and on-chip lane tables at their largest
    M = amq.am_max_dates() if M == "max" else M
    N = 20000
    kw = dict(S0=100.0, K=100.0, r=0.04, sigma=0.3, T=2.0)
    price, se, v = gpu_price(amq, pricer, None, N=N, M=M, dtype=dtype, basis=("monomial", 2), **kw)
    ores, od = oracle_price(orc, None, N=N, M=M, basis=("monomial", 2), dtype=dtype, **kw)
    log(f"  M={M} {dtype}: gpu {price:.10f} oracle {ores.price:.10f}")
    assert abs(price - ores.price) <= TOL[dtype]
    nitm = v["rec"].cpu().numpy()[1:M, 9].astype(np.int64)
    assert np.abs(nitm - od["nitm"][1:M]).max() <= (0 if dtype == "fp64" else 1)
    want = orc.paths_range(**kw, first=N - 100, count=100, M=M)
    got = v["S"][:, N - 100:N].cpu().numpy()
    if dtype == "fp32":
        check_stored32(got, want, f"last paths at M={M}")
    else:
        assert np.abs(got - want).max() / want.max() <= 1e-12


@pytest.mark.parametrize("N,M", [(4, 3), (1000, 17), (4097, 12), (16383, 5)])
def test_fp32_below_path_floor_is_the_fp64_result(amq, pricer, N, M):
    # the storage rule: such an FP32-bulk request is the FP64 request, bitwise
    kw = dict(S0=100.0, K=105.0, r=0.04, sigma=0.25, T=0.75)
    p32 = gpu_price(amq, pricer, None, N=N, M=M, dtype="fp32", basis=("monomial", 2), **kw)[:2]
    p64 = gpu_price(amq, pricer, None, N=N, M=M, dtype="fp64", basis=("monomial", 2), **kw)[:2]
    assert p32 == p64


@pytest.mark.parametrize("N,M,basis,dtype", [(33001, 9, ("laguerre", 3), "fp64"), (4097, 12, ("laguerre", 2), "fp64"),
                                             (70000, 17, ("monomial", 2), "fp32"),
                                             (1 << 18, 20, ("laguerre", 3), "fp32"),
                                             ((1 << 18) + 999, 6, ("monomial", 3), "fp64"),
                                             ((1 << 23) - 5, 5, ("monomial", 3), "fp32"),
                                             ((1 << 23) + 4097, 4, ("laguerre", 2), "fp32")])
def test_group_size_forms_agree(amq, orc, pricer, N, M, basis, dtype):
    # tiles run in 256- or 512-thread groups (register-resident tiles, and
    # binary32 streamed tiles of 2^23 paths and more): both forms must meet
    # the oracle, with identical in-the-money counts (those depend on the
    # path values only)
    kw = dict(S0=100.0, K=104.0, r=0.045, sigma=0.28, T=1.25)
    ores, od = oracle_price(orc, None, N=N, M=M, basis=basis, dtype=dtype, **kw)
    out = []
    try:
        for wide in (False, True):
            amq.am_debug_set_sweep_wide(wide)
            price, se, v = gpu_price(amq, pricer, None, N=N, M=M, dtype=dtype, basis=basis, **kw)
            nitm = v["rec"].cpu().numpy()[1:M, 9].astype(np.int64)
            out.append((price, nitm))
            log(f"  wide={wide}: gpu {price:.10f} oracle {ores.price:.10f}")
            assert abs(price - ores.price) <= TOL[dtype]
    finally:
        amq.am_debug_set_sweep_wide(True)
    assert np.array_equal(out[0][1], out[1][1])
    assert np.abs(out[0][1] - od["nitm"][1:M]).max() <= (0 if dtype == "fp64" else 1)


@pytest.mark.parametrize("ppt,N,M,degree,call,K", [
    (128, 3 * 65536 - 1234, 24, 4, False, 110.0), (128, 3 * 65536 - 1234, 24, 4, True, 95.0),
    (128, 2 * 65536 - 5, 13, 6, False, 104.0), (128, 2 * 65536 - 5, 9, 1, True, 100.0),
    (128, 65536, 7, 0, False, 100.0),
    (64, 100001, 17, 2, False, 100.3), (64, 100001, 17, 3, True, 97.0), (64, 40000, 30, 5, False, 120.0),
    (64, 50000, 10, 4, True, 150.0)])
def test_slab_resident_tiles(amq, orc, pricer, ppt, N, M, degree, call, K):
    # binary32 monomial tiles of 512 threads x 64 or 128 paths keep each
    # date's slab on chip between the moment pass and the update (LDS,
    # registers, and for 128 paths a part read again); forced here at sizes
    # the oracle prices quickly, puts and calls (separately compiled), all
    # degrees, dates where too few paths are in the money to fit
    kw = dict(S0=100.0, K=K, r=0.04, sigma=0.3, T=1.5)
    ores, od = oracle_price(orc, None, N=N, M=M, basis=("monomial", degree), is_call=call, dtype="fp32",
                            **kw)
    try:
        amq.am_debug_set_sweep_tile(512, ppt)
        price, se, v = gpu_price(amq, pricer, None, N=N, M=M, dtype="fp32", basis=("monomial", degree),
                                 is_call=call, **kw)
    finally:
        amq.am_debug_set_sweep_tile(0, 0)
    rec = v["rec"].cpu().numpy()
    nitm = rec[1:M, 9].astype(np.int64)
    solved = rec[1:M, 8]
    log(f"  ppt={ppt} N={N} M={M} d={degree} call={call}: gpu {price:.10f} oracle {ores.price:.10f} "
        f"skipped {int((solved == 0).sum())}")
    assert abs(price - ores.price) <= TOL["fp32"]
    assert np.abs(nitm - od["nitm"][1:M]).max() <= 1
    assert abs(se - ores.std_err) <= 0.02 * ores.std_err


def test_team_level_device_sum(amq, orc, pricer):
    # more than 256 workgroups: teams sum first; 500 groups of 64 paths per
    # thread leaves a last team of 4 (teams of 16)
    N, M = 500 * 256 * 64 - 7, 4
    kw = dict(S0=100.0, K=105.0, r=0.04, sigma=0.25, T=0.75)
    price, se, v = gpu_price(amq, pricer, None, N=N, M=M, dtype="fp64", basis=("monomial", 2), **kw)
    ores, od = oracle_price(orc, None, N=N, M=M, basis=("monomial", 2), **kw)
    nitm = v["rec"].cpu().numpy()[1:M, 9].astype(np.int64)
    log(f"  N={N}: gpu {price:.10f} oracle {ores.price:.10f}; itm {nitm} vs {od['nitm'][1:M]}")
    assert np.array_equal(nitm, od["nitm"][1:M])
    assert abs(price - ores.price) <= TOL["fp64"]
    assert abs(se - ores.std_err) <= 1e-6 * ores.std_err


@pytest.mark.parametrize("call,K", [(False, 100.59555281085481), (True, 80.14936968208303),
                                    (False, 97.3), (True, 113.1)])
def test_fp32_padding_stays_out_of_the_money(amq, orc, pricer, call, K):
    # strikes that binary32 cannot hold exactly, and a row mostly made of
    # padding (N far below the tile multiple): padded paths must never count
    # as in the money, so the per-date counts match the oracle's
    kw = dict(S0=100.0, K=K, r=0.05, sigma=0.3, T=1.0)
    N, M = 16385, 6   # binary32 storage from 2^14 paths; the row's other half is padding
    price, se, v = gpu_price(amq, pricer, None, N=N, M=M, dtype="fp32", basis=("monomial", 2),
                             is_call=call, **kw)
    ores, od = oracle_price(orc, None, N=N, M=M, basis=("monomial", 2), is_call=call, dtype="fp32", **kw)
    nitm = v["rec"].cpu().numpy()[1:M, 9].astype(np.int64)
    log(f"  K={K} call={call}: itm {nitm} oracle {od['nitm'][1:M]}; gpu {price:.8f} oracle {ores.price:.8f}")
    assert np.abs(nitm - od["nitm"][1:M]).max() <= 1
    assert abs(price - ores.price) <= TOL["fp32"]


@pytest.mark.parametrize("call", [False, True])
@pytest.mark.parametrize("basis", [("monomial", 1), ("monomial", 3), ("laguerre", 2), ("laguerre", 4),
                                   ("monomial", 6), ("monomial", 0)])
def test_bases_and_calls_fp64(amq, orc, pricer, call, basis):
    kw = dict(S0=100.0, K=100.0, r=0.05, sigma=0.3, T=1.0)
    price, se, v = gpu_price(amq, pricer, None, N=1 << 15, M=20, basis=basis, is_call=call, **kw)
    ores, od = oracle_price(orc, None, N=1 << 15, M=20, basis=basis, is_call=call, **kw)
    log(f"  {basis} call={call}: gpu {price:.10f} oracle {ores.price:.10f}")
    assert abs(price - ores.price) <= TOL["fp64"]


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_european_mode(amq, orc, pricer, dtype):
    for call in (False, True):
        price, se, _ = gpu_price(amq, pricer, CONFIG1, dtype=dtype, is_call=call, allow_exercise=False)
        ores, _ = oracle_price(orc, CONFIG1, is_call=call, allow_exercise=False, dtype=dtype)
        assert abs(price - ores.price) <= TOL[dtype]
        bs = orc.bs_price(**CONFIG1.params(), is_call=call)
        assert abs(price - bs) < 0.01


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_standard_error_with_tiny_variance(amq, orc, pricer, dtype):
    # deep in the money, sigma 1e-6: cashflows of about 100 with a standard
    # deviation near 1e-4, so sums of squares taken about zero would lose the
    # variance to cancellation (relative 1e-16 * 100^2 / 1e-8)
    kw = dict(S0=100.0, K=200.0, r=0.0, sigma=1e-6, T=1.0)
    N, M = 1 << 15, 6
    price, se, _ = gpu_price(amq, pricer, None, N=N, M=M, dtype=dtype, basis=("monomial", 2),
                             allow_exercise=False, **kw)
    ores, _ = oracle_price(orc, None, N=N, M=M, basis=("monomial", 2), allow_exercise=False, dtype=dtype,
                           **kw)
    log(f"  {dtype}: se gpu {se:.6e} oracle {ores.std_err:.6e}; price {price!r} {ores.price!r}")
    assert ores.std_err > 0.0
    # binary32 storage: K - S is exact in binary32 for these values, so both
    # sides hold the same cashflows
    assert abs(se - ores.std_err) <= 1e-6 * ores.std_err
    p = amq.make_params(200.0, 100.0, 0.0, 1e-6, 1.0, is_call=True)
    pse = pricer.price_paper(p, N, 4, "fp64")[1]
    want = orc.paper_estimator(200.0, 100.0, 0.0, 1e-6, 1.0, N=N, m=4, is_call=True)
    log(f"  paper estimator se gpu {pse:.6e} oracle {want.std_err:.6e}")
    assert want.std_err > 0.0 and abs(pse - want.std_err) <= 1e-6 * want.std_err


def test_t0_exercise_wins(amq, orc, pricer):
    kw = dict(S0=40.0, K=100.0, r=0.08, sigma=0.1, T=1.0)
    price, se, v = gpu_price(amq, pricer, None, N=4096, M=10, basis=("monomial", 2), **kw)
    ores, _ = oracle_price(orc, None, N=4096, M=10, basis=("monomial", 2), **kw)
    assert ores.t0_exercise and price == 60.0 and se == 0.0
    assert v["result"].cpu().numpy()[3] == 1.0


def test_degenerate_dates_skip_exercise(amq, orc, pricer):
    # deep out of the money: most dates have fewer in-the-money paths than p
    kw = dict(S0=100.0, K=40.0, r=0.03, sigma=0.15, T=1.0)
    price, se, v = gpu_price(amq, pricer, None, N=2048, M=30, basis=("monomial", 3), **kw)
    ores, od = oracle_price(orc, None, N=2048, M=30, basis=("monomial", 3), **kw)
    res = v["result"].cpu().numpy()
    log(f"  skipped gpu {res[4]} oracle {ores.n_skipped}; price {price} vs {ores.price}")
    assert res[4] == ores.n_skipped
    assert abs(price - ores.price) <= TOL["fp64"]


def test_deterministic_repeats(amq, pricer):
    w = CONFIG1
    ref = gpu_price(amq, pricer, w, dtype="fp64")[0]
    for _ in range(10):
        assert gpu_price(amq, pricer, w, dtype="fp64")[0] == ref
    ref32 = gpu_price(amq, pricer, w, dtype="fp32")[0]
    for _ in range(5):
        assert gpu_price(amq, pricer, w, dtype="fp32")[0] == ref32


def test_sync_entry_point_matches_async(amq, pricer):
    w = CONFIG1
    p = amq.make_params(**w.params())
    b = amq.make_basis(*w.basis)
    a = amq.am_price_american(p, w.n_paths, w.n_dates, b, "fp64")
    c = pricer.price(p, w.n_paths, w.n_dates, b, "fp64")
    assert a == c


def test_bounded_wait_reports_timeout(amq, orc, pricer):
    # force the device-side barrier waits to give up almost at once; every
    # workgroup must still exit and the call must report AM_ETIMEOUT (or, if
    # no wait ever had to poll twice, succeed) -- then work normally again
    w = CONFIG1
    p = amq.make_params(**w.params())
    b = amq.make_basis(*w.basis)
    amq.am_debug_set_spin_limit(1)
    try:
        try:
            pricer.price(p, w.n_paths, w.n_dates, b, "fp64")
            outcome = "ok"
        except amq.AmError as e:
            assert e.code == amq.AM_ETIMEOUT
            outcome = "timeout"
    finally:
        amq.am_debug_set_spin_limit(0)
    log(f"  tiny spin limit -> {outcome}")
    ref = gpu_price(amq, pricer, w, dtype="fp64")[0]
    ores, _ = oracle_price(orc, w)
    assert abs(ref - ores.price) <= TOL["fp64"]


def test_too_many_paths_rejected(amq):
    mx = amq.am_max_paths("fp32")
    assert mx >= 1 << 24
    p = amq.make_params(100.0, 100.0, 0.05, 0.3, 1.0)
    with pytest.raises(amq.AmError) as e:
        amq.am_price_american(p, mx * 4, 4, amq.make_basis("monomial", 2), "fp32")
    assert e.value.code in (amq.AM_EDIM, amq.AM_ENOMEM)


# --------------------------------------------------------------------------
# The paper's own estimator (Section V, eqs. (10)-(11))
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("m,N,call", [(10, 1 << 16, True), (10, 1 << 16, False), (1, 1000, True),
                                      (50, 4097, False), (3, 10, True)])
def test_paper_estimator_matches_oracle(amq, orc, pricer, dtype, m, N, call):
    kw = CONFIG1.params()
    p = amq.make_params(**kw, is_call=call)
    log(f"  paper estimator m={m} N={N} call={call} {dtype}")
    price, se = pricer.price_paper(p, N, m, dtype)
    want = orc.paper_estimator(**kw, N=N, m=m, is_call=call)
    log(f"    gpu {price:.10f} oracle {want.price:.10f}")
    assert abs(price - want.price) <= TOL[dtype]
    if N >= 1 << 16:   # perfect foresight exceeds the European value (in expectation)
        assert price >= orc.bs_price(**kw, is_call=call) - TOL[dtype]


# --------------------------------------------------------------------------
# Randomised QMC (digital shifts): replicate prices and the error bar
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_rqmc_matches_oracle(amq, orc, pricer, dtype):
    w = CONFIG1
    R, N, M = 8, 1 << 12, 50
    rng = np.random.default_rng(0x12050108)
    sh = rng.integers(0, 2 ** 32, size=(R, M), dtype=np.uint64).astype(np.uint32)
    p = amq.make_params(**w.params())
    b = amq.make_basis(*w.basis)
    log(f"  rqmc R={R} N={N} M={M} {dtype}")
    mean, se, reps = pricer.price_rqmc(p, N, M, b, dtype, sh)
    omean, ose, oreps = orc.price_american_rqmc(**w.params(), N=N, M=M, shifts=sh,
                                                kind=orc.MONOMIAL, degree=2)
    log(f"    gpu {mean:.8f} +- {se:.2e}  oracle {omean:.8f} +- {ose:.2e}")
    assert np.abs(reps - oreps).max() <= TOL[dtype]
    assert abs(mean - omean) <= TOL[dtype]
    assert abs(se - ose) <= 0.05 * ose + TOL[dtype] / 10


@pytest.mark.parametrize("dtype,N,R", [("fp64", 1 << 12, 8), ("fp32", 1 << 15, 5), ("fp64", 3000, 1),
                                       ("fp32", 20000, 16)])
def test_rqmc_fused_equals_serial_and_oracle(amq, orc, pricer, dtype, N, R):
    # all replicates at once (a batch of shifted options) against one after
    # another: the same replicate prices to rounding, both against the oracle
    # on the same storage
    w = CONFIG1
    M = 20
    rng = np.random.default_rng(0x5EED + R)
    sh = rng.integers(0, 2 ** 32, size=(R, M), dtype=np.uint64).astype(np.uint32)
    p = amq.make_params(**w.params())
    b = amq.make_basis(*w.basis)
    log(f"  rqmc fused vs serial {dtype} N={N} R={R}")
    fm, fse, freps = pricer.price_rqmc(p, N, M, b, dtype, sh, fused=True)
    sm, sse, sreps = pricer.price_rqmc(p, N, M, b, dtype, sh, fused=False)
    omean, ose, oreps = orc.price_american_rqmc(**w.params(), N=N, M=M, shifts=sh, kind=orc.MONOMIAL,
                                                degree=2, store32=stores32(dtype, N))
    log(f"    fused {fm:.10f} serial {sm:.10f} oracle {omean:.10f}")
    assert np.abs(freps - sreps).max() <= 1e-9
    assert np.abs(freps - oreps).max() <= TOL[dtype]
    assert abs(fm - omean) <= TOL[dtype]
    if R > 1:
        assert abs(fse - sse) <= 1e-9 and abs(fse - ose) <= 0.05 * ose + TOL[dtype] / 10
    else:
        assert fse == 0.0 and sse == 0.0
