"""Why FP32 bulk stores binary32 but computes the induction in binary64 (CPU).

The least-squares induction (Section V, eqs. (10)-(11) in regression form)
feeds every exercise decision back into the cashflows that later dates
regress on.  For some options of the batch workload's distribution the
exercise value and the fitted continuation run nearly parallel over the
in-the-money paths, so a shift of the fit by a relative 1e-7 flips many
decisions at once.  This test reproduces that on the oracle's paths:

- binary32 *storage* of the path values and cashflows (each rounded once),
  with binary64 arithmetic, moves the price by rounding-level amounts (the
  oracle's binary32-storage mode);
- the same formulation as the GPU kernels (standardised monomial basis,
  normal equations solved in binary64, cashflows discounted to t0 and stored
  in binary32), emulated here in numpy with binary64 arithmetic, agrees with
  that oracle;
- the same emulation with the exercise update (continuation value and
  exercise value) in binary32 arithmetic misses the oracle by more than the
  2e-3 FP32-bulk tolerance.

Storage alone is not always harmless either: two options of the batch
workload (seed 0) move by more than 2e-3 between binary64 and binary32
storage, one through the rounding of its path values and one through the
rounding of its cashflows.  That is why FP32-bulk results are checked
against the oracle on binary32 storage.
"""
import numpy as np
import pytest

from paper_1205_0106_amd.workloads import batch_options

FP32_TOL = 2e-3


def _option(i):
    # the batch workload's distribution with 2^14-2^15 paths and 3-40 dates
    # (the FP32 batch parity mix); option 6 is a deep in-the-money call
    return batch_options(48, seed=7, log2_paths=(14.0, 15.0), dates=(3, 40))[i]


def lsm_emulated(S, S0, K, r, T, is_call, degree, f32_update):
    """Least squares in the kernels' formulation: cashflows discounted to t0
    and stored in binary32; per date the abscissa x = S/K standardised over the
    in-the-money paths, monomials of it, normal equations solved in binary64;
    exercise where the discounted payoff exceeds max(fit, 0).  f32_update:
    the fit and the discounted payoff in binary32 arithmetic."""
    M, N = S.shape
    dt = T / M
    sg = 1.0 if is_call else -1.0
    disc = np.exp(-r * dt * np.arange(M + 1))
    pv = np.float64(np.float32(disc[M] * np.maximum(sg * (S[M - 1] - K), 0.0)))
    pv = np.asarray(pv, dtype=np.float64)
    for k in range(M - 1, 0, -1):
        hk = sg * (S[k - 1] - K)
        itm = hk > 0
        if itm.sum() <= degree:
            continue
        x = S[k - 1] / K
        mu, sd = x[itm].mean(), x[itm].std()
        xs = (x - mu) / sd
        V = np.vander(xs[itm], degree + 1, increasing=True)
        beta = np.linalg.solve(V.T @ V, V.T @ pv[itm])
        if f32_update:
            xs32, b32 = xs.astype(np.float32), beta.astype(np.float32)
            cont = np.zeros(N, np.float32)
            for q in range(degree, -1, -1):
                cont = cont * xs32 + b32[q]
            ex = np.float32(disc[k]) * hk.astype(np.float32)
            dec = itm & (ex > np.maximum(cont, np.float32(0.0)))
        else:
            cont = np.zeros(N)
            for q in range(degree, -1, -1):
                cont = cont * xs + beta[q]
            ex = disc[k] * hk
            dec = itm & (ex > np.maximum(cont, 0.0))
        pv = np.where(dec, np.float32(disc[k] * hk).astype(np.float64), pv)
    h0 = max(sg * (S0 - K), 0.0)
    return max(h0, float(pv.mean()))


@pytest.fixture(scope="module")
def case(orc):
    d = _option(6)
    assert d["is_call"] and d["K"] < 85.0          # deep in the money at S0 = 100
    S = orc.paths(d["S0"], d["K"], d["r"], d["sigma"], d["T"], d["n_paths"], d["n_dates"])
    ref = orc.price_american(d["S0"], d["K"], d["r"], d["sigma"], d["T"], N=d["n_paths"], M=d["n_dates"],
                             is_call=True, kind=orc.MONOMIAL, degree=2).price
    S32 = S.astype(np.float32).astype(np.float64)
    return d, S32, ref


def test_binary32_storage_moves_price_at_rounding_level(orc, case):
    d, S32, ref = case
    stored = orc.lsm_on_paths(S32, d["S0"], d["K"], d["r"], d["sigma"], d["T"], is_call=True, degree=2,
                              store32=True).price
    assert abs(stored - ref) <= 1e-6, (stored, ref)


def test_emulation_with_binary64_arithmetic_matches_oracle(orc, case):
    d, S32, ref = case
    got = lsm_emulated(S32, d["S0"], d["K"], d["r"], d["T"], True, 2, f32_update=False)
    stored = orc.lsm_on_paths(S32, d["S0"], d["K"], d["r"], d["sigma"], d["T"], is_call=True, degree=2,
                              store32=True).price
    assert abs(got - stored) <= 1e-9, (got, stored)


def test_binary32_update_arithmetic_exceeds_fp32_tolerance(case):
    d, S32, ref = case
    got = lsm_emulated(S32, d["S0"], d["K"], d["r"], d["T"], True, 2, f32_update=True)
    assert abs(got - ref) > FP32_TOL, (got, ref)


def test_well_conditioned_options_tolerate_either(orc):
    # most options do not care: an at-the-money put of the same mix
    d = _option(14)
    assert not d["is_call"]
    S = orc.paths(d["S0"], d["K"], d["r"], d["sigma"], d["T"], d["n_paths"], d["n_dates"])
    ref = orc.price_american(d["S0"], d["K"], d["r"], d["sigma"], d["T"], N=d["n_paths"], M=d["n_dates"],
                             kind=orc.MONOMIAL, degree=2).price
    S32 = S.astype(np.float32).astype(np.float64)
    for f32 in (False, True):
        got = lsm_emulated(S32, d["S0"], d["K"], d["r"], d["T"], False, 2, f32_update=f32)
        assert abs(got - ref) <= 1e-6


@pytest.mark.parametrize("idx,cause", [(842, "paths"), (302, "cashflows")])
def test_storage_alone_moves_ill_conditioned_options(orc, idx, cause):
    d = batch_options(1024)[idx]
    kw = dict(is_call=d["is_call"], degree=2)
    prm = (d["S0"], d["K"], d["r"], d["sigma"], d["T"])
    S = orc.paths(*prm, d["n_paths"], d["n_dates"])
    S32 = S.astype(np.float32).astype(np.float64)
    full = orc.lsm_on_paths(S, *prm, **kw).price
    paths32 = orc.lsm_on_paths(S32, *prm, **kw).price          # rounded paths, binary64 cashflows
    both32 = orc.lsm_on_paths(S, *prm, store32=True, **kw).price
    assert abs(both32 - full) > FP32_TOL
    if cause == "paths":
        assert abs(paths32 - full) > FP32_TOL and abs(both32 - paths32) < 1e-6
    else:
        assert abs(paths32 - full) < 1e-6 and abs(both32 - paths32) > FP32_TOL
    # the kernels' formulation on the same storage lands on the storage result
    emu = lsm_emulated(S32, d["S0"], d["K"], d["r"], d["T"], d["is_call"], 2, f32_update=False)
    assert abs(emu - both32) <= 1e-9, (emu, both32)
