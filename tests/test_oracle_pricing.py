"""Pins for the oracle's pricing: closed forms, lattices, a published worked
example, exact special cases and invariants of the least-squares induction."""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

CONFIG1 = dict(S0=36.0, K=40.0, r=0.06, sigma=0.2, T=1.0)
CONFIG2 = dict(S0=100.0, K=100.0, r=0.05, sigma=0.3, T=1.0)
CONFIG4 = dict(S0=100.0, K=110.0, r=0.03, sigma=0.25, T=2.0)


# --------------------------------------------------------------------------
# Black–Scholes closed form and the CRR tree
# --------------------------------------------------------------------------
def test_bs_put_call_parity(orc):
    for S0, K, r, s, T in [(36, 40, .06, .2, 1), (100, 110, .03, .25, 2), (100, 100, 0, .3, .5)]:
        c = orc.bs_price(S0, K, r, s, T, True)
        p = orc.bs_price(S0, K, r, s, T, False)
        assert abs((c - p) - (S0 - K * math.exp(-r * T))) < 1e-12


def test_bs_textbook_value(orc):
    # Hull, "Options, Futures and Other Derivatives": S0=42, K=40, r=10%,
    # sigma=20%, T=0.5 gives c = 4.76 and p = 0.81 (printed to cents)
    assert round(orc.bs_price(42, 40, .1, .2, .5, True), 2) == 4.76
    assert round(orc.bs_price(42, 40, .1, .2, .5, False), 2) == 0.81


def test_bs_limits(orc):
    # deep in the money: value tends to the discounted forward payoff
    assert abs(orc.bs_price(1000, 1, .05, .2, 1, True) - (1000 - math.exp(-.05))) < 1e-9
    assert orc.bs_price(1, 1000, .05, .2, 1, True) < 1e-12


@pytest.mark.parametrize("cfg", [CONFIG1, CONFIG2, CONFIG4])
def test_crr_european_converges_to_bs(orc, cfg):
    for call in (False, True):
        crr = orc.crr_price(**cfg, is_call=call, n=5000, style=orc.EUROPEAN)
        assert abs(crr - orc.bs_price(**cfg, is_call=call)) < 1e-3


@pytest.mark.parametrize("cfg", [CONFIG1, CONFIG2])
def test_crr_american_call_equals_european_without_dividends(orc, cfg):
    a = orc.crr_price(**cfg, is_call=True, n=2000, style=orc.AMERICAN)
    e = orc.crr_price(**cfg, is_call=True, n=2000, style=orc.EUROPEAN)
    assert abs(a - e) < 1e-10


def test_crr_ordering_and_bermudan_monotone(orc):
    am = orc.crr_price(**CONFIG1, n=4000, style=orc.AMERICAN)
    eu = orc.crr_price(**CONFIG1, n=4000, style=orc.EUROPEAN)
    prev = eu
    for M in (5, 10, 20, 40, 80):
        b = orc.crr_price(**CONFIG1, n=4000, style=orc.BERMUDAN, M=M)
        assert prev - 1e-12 <= b <= am + 1e-12
        prev = b
    assert am > eu + 0.5


def test_crr_bermudan_limits(orc):
    # exercisable at every step: the Bermudan tree is the American tree
    n = 1200
    am = orc.crr_price(**CONFIG1, n=n, style=orc.AMERICAN)
    assert orc.crr_price(**CONFIG1, n=n, style=orc.BERMUDAN, M=n) == am
    # exercisable only at t0 (and expiry): max(h(S0), European value)
    eu = orc.crr_price(**CONFIG1, n=n, style=orc.EUROPEAN)
    b1 = orc.crr_price(**CONFIG1, n=n, style=orc.BERMUDAN, M=1)
    assert b1 == max(CONFIG1["K"] - CONFIG1["S0"], eu)


# --------------------------------------------------------------------------
# The published worked example of the least-squares method (reference [12])
# --------------------------------------------------------------------------
def test_longstaff_schwartz_worked_example(orc):
    g = json.load(open(os.path.join(GOLDEN, "longstaff_schwartz_2001_example.json")))
    S = np.array(g["paths_t1_t2_t3"]).T.copy()
    res, d = orc.lsm_on_paths(S, g["S0"], g["K"], g["r"], 0.2, g["T"], is_call=False,
                              kind=orc.MONOMIAL, degree=2, detail=True)
    K = g["K"]
    for k, key in ((2, "regression_t2"), (1, "regression_t1")):
        b = d["beta"][k]
        assert b[8] == 1.0
        in_stock_units = [b[0], b[1] / K, b[2] / K ** 2]   # oracle regresses on x = S/K
        # printed to 3 decimals: agree within one unit of the last printed digit
        assert np.abs(np.array(in_stock_units) - g[key]).max() <= 1.0e-3
    assert d["nitm"][2] == g["in_the_money_t2"] and d["nitm"][1] == g["in_the_money_t1"]
    assert d["tau"].tolist() == g["stopping_date_per_path"]
    cf = d["pv"] * np.exp(g["r"] * d["tau"])
    assert np.allclose(np.round(cf, 2), g["cashflow_at_stop"], atol=1e-12)
    assert round(res.price, 4) == g["price"]
    assert not res.t0_exercise


# --------------------------------------------------------------------------
# Exact special cases of the induction
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind,degree", [(0, 1), (0, 2), (1, 2), (1, 3)])
def test_interpolating_regression_is_perfect_foresight(orc, kind, degree):
    # With exactly p in-the-money paths the least-squares fit interpolates the
    # realised cashflows, so every path stops at the best of its own dates.
    p = degree + 1
    S0, K, r, sig, T, M = 40.0, 100.0, 0.05, 0.3, 1.0, 6
    # seeded lognormal paths with distinct abscissae at every date (the first
    # few Sobol points coincide at some dates, which makes those fits singular)
    rng = np.random.default_rng(11)
    S = S0 * np.exp(np.cumsum(0.2 * rng.standard_normal((M, p)), axis=0))
    assert (S < K).all()
    res, d = orc.lsm_on_paths(S, S0, K, r, sig, T, kind=kind, degree=degree, detail=True)
    assert res.n_skipped == 0
    t = np.arange(1, M + 1) * T / M
    disc_payoff = (K - S) * np.exp(-r * t)[:, None]
    assert np.allclose(d["pv"], disc_payoff.max(axis=0), rtol=1e-12, atol=0)
    assert d["tau"].tolist() == (disc_payoff.argmax(axis=0) + 1).tolist()


def test_hand_computed_two_path_case(orc):
    # Two paths, two dates, basis {1} (degree 0): the fit at t1 is the mean of
    # the in-the-money targets.  Put K=1, r=0, T=2 (t1=1, t2=2).
    S = np.array([[0.5, 0.8],      # t1: payoffs 0.5, 0.2
                  [0.9, 0.2]])     # t2: payoffs 0.1, 0.8
    res, d = orc.lsm_on_paths(S, 1.0, 1.0, 0.0, 0.2, 2.0, kind=orc.MONOMIAL, degree=0, detail=True)
    # fit at t1 = (0.1 + 0.8)/2 = 0.45: path 0 exercises (0.5 > 0.45), path 1 does not
    assert d["tau"].tolist() == [1, 2]
    assert abs(d["beta"][1][0] - 0.45) < 1e-15
    assert abs(res.mean_pv - (0.5 + 0.8) / 2) < 1e-15
    # naive standard error: sample sd sqrt(2 * 0.15^2 / 1) over sqrt(2) = 0.15
    assert abs(res.std_err - 0.15) < 1e-15


def test_single_date_equals_exercise_off(orc):
    kw = dict(S0=36.0, K=40.0, r=0.06, sigma=0.2, T=1.0)
    a = orc.price_american(**kw, N=4096, M=1, allow_exercise=True)
    e = orc.price_american(**kw, N=4096, M=1, allow_exercise=False)
    assert a.mean_pv == e.mean_pv
    assert a.price == max(4.0, e.price)


def test_fewer_paths_than_basis_skips_every_date(orc):
    a = orc.price_american(**CONFIG1, N=3, M=10, kind=orc.MONOMIAL, degree=3)
    e = orc.price_american(**CONFIG1, N=3, M=10, allow_exercise=False)
    assert a.n_skipped == 9 and a.mean_pv == e.mean_pv


@pytest.mark.parametrize("call", [False, True])
@pytest.mark.parametrize("kind,degree", [(0, 2), (1, 3)])
def test_homogeneity_is_bitwise(orc, call, kind, degree):
    base = dict(r=0.05, sigma=0.3, T=1.0, N=2048, M=16, is_call=call, kind=kind, degree=degree)
    a = orc.price_american(S0=100.0, K=95.0, **base)
    b = orc.price_american(S0=200.0, K=190.0, **base)
    assert b.price == 2.0 * a.price and b.std_err == 2.0 * a.std_err


# --------------------------------------------------------------------------
# Binary32 storage: the induction on the path values rounded to binary32
# --------------------------------------------------------------------------
@pytest.mark.parametrize("call,kind,degree", [(False, 0, 2), (True, 0, 4), (False, 1, 3)])
def test_store32_rounds_paths_and_cashflows_to_nearest(orc, call, kind, degree):
    kw = dict(S0=100.0, K=104.0, r=0.06, sigma=0.3, T=1.0)
    N, M = 3000, 12
    S = orc.paths(**kw, N=N, M=M)
    S32 = S.astype(np.float32).astype(np.float64)          # numpy's round to nearest
    assert np.any(S32 != S)
    # the full oracle in binary32 storage reads the paths rounded to nearest
    got, gd = orc.price_american(**kw, N=N, M=M, is_call=call, kind=kind, degree=degree, store32=True,
                                 detail=True)
    on32, od = orc.lsm_on_paths(S32, **kw, is_call=call, kind=kind, degree=degree, store32=True, detail=True)
    assert got.price == on32.price and np.array_equal(gd["pv"], od["pv"])
    # every cashflow is its binary64 value discounted to t0, rounded to
    # nearest: on the same (binary32) paths and the same stopping dates, the
    # binary64-storage cashflow rounds to the binary32-storage one
    full, fd = orc.lsm_on_paths(S32, **kw, is_call=call, kind=kind, degree=degree, detail=True)
    same = od["tau"] == fd["tau"]
    assert same.mean() >= 0.99
    assert np.array_equal(od["pv"][same], fd["pv"][same].astype(np.float32).astype(np.float64))
    # and the price moves at rounding level only
    assert full.price != got.price and abs(full.price - got.price) < 1e-5


def test_store32_exact_when_storage_is_exact(orc):
    # r = 0 (no discounting) and path values already binary32 within [K/2, 2K]:
    # every cashflow K - S is exact in binary32, so storage changes nothing
    kw = dict(S0=100.0, K=104.0, r=0.0, sigma=0.1, T=1.0)
    S = orc.paths(**kw, N=2000, M=9).astype(np.float32).astype(np.float64)
    assert S.min() > 52.0 and S.max() < 208.0
    a, ad = orc.lsm_on_paths(S, **kw, detail=True)
    b, bd = orc.lsm_on_paths(S, **kw, detail=True, store32=True)
    assert a.price == b.price and a.std_err == b.std_err and np.array_equal(ad["pv"], bd["pv"])
    # sigma = 0 and r = 0: every path value is S0
    c = orc.price_american(**dict(kw, sigma=0.0), N=500, M=7, allow_exercise=False, store32=True)
    assert c.price == 4.0


def test_store32_rqmc_replicates(orc):
    kw = dict(S0=36.0, K=40.0, r=0.06, sigma=0.2, T=1.0)
    sh = np.random.default_rng(5).integers(0, 2 ** 32, size=(2, 9), dtype=np.uint64).astype(np.uint32)
    _, _, reps = orc.price_american_rqmc(**kw, N=2048, M=9, shifts=sh, store32=True)
    for j in range(2):
        one = orc.price_american_rqmc(**kw, N=2048, M=9, shifts=sh[j:j + 1], store32=True)[2][0]
        assert one == reps[j]
    _, _, reps64 = orc.price_american_rqmc(**kw, N=2048, M=9, shifts=sh)
    assert np.all(reps != reps64) and np.abs(reps - reps64).max() < 1e-5


# --------------------------------------------------------------------------
# Levels: closed form without exercise, lattice with exercise
# --------------------------------------------------------------------------
@pytest.mark.parametrize("cfg,N", [(CONFIG1, 1 << 14), (CONFIG4, 1 << 14), (CONFIG2, 1 << 12)])
def test_exercise_off_matches_black_scholes(orc, cfg, N):
    # With the bridge S_T depends on the first Sobol dimension only: a 1-D
    # quadrature on a near-uniform grid.  For the put (monotone, bounded by K)
    # Koksma–Hlawka bounds the error by K/N.  The call is unbounded; its error
    # is the upper tail beyond the largest point, u = 1 - O(1/N), z ~ sqrt(2 ln N).
    put = orc.price_american(**cfg, N=N, M=8, is_call=False, allow_exercise=False)
    assert abs(put.price - orc.bs_price(**cfg, is_call=False)) < cfg["K"] / N
    call = orc.price_american(**cfg, N=N, M=8, is_call=True, allow_exercise=False)
    tail = cfg["S0"] * math.exp(cfg["sigma"] * math.sqrt(cfg["T"]) * math.sqrt(2 * math.log(N))) / N
    assert abs(call.price - orc.bs_price(**cfg, is_call=True)) < tail + cfg["K"] / N


def test_config1_lsm_close_to_bermudan_tree(orc):
    r = orc.price_american(**CONFIG1, N=1 << 14, M=50, kind=orc.MONOMIAL, degree=2)
    berm = orc.crr_price(**CONFIG1, n=5000, style=orc.BERMUDAN, M=50)
    assert abs(r.price - berm) < 0.03
    assert r.price > orc.bs_price(**CONFIG1) + 0.5


def test_config2_lsm_close_to_bermudan_tree(orc):
    r = orc.price_american(**CONFIG2, N=1 << 16, M=100, kind=orc.LAGUERRE, degree=3)
    berm = orc.crr_price(**CONFIG2, n=5000, style=orc.BERMUDAN, M=100)
    assert abs(r.price - berm) < 0.03


def test_zero_rate_put_has_no_early_exercise_premium(orc):
    cfg = dict(S0=100.0, K=100.0, r=0.0, sigma=0.3, T=1.0)
    r = orc.price_american(**cfg, N=1 << 14, M=20, kind=orc.MONOMIAL, degree=2)
    bs = orc.bs_price(**cfg)
    assert abs(r.price - bs) < 0.005 * bs


@pytest.mark.parametrize("kind,degree,band", [(0, 2, 0.015), (0, 3, 0.002), (0, 4, 0.005), (1, 3, 0.015)])
def test_american_call_close_to_european(orc, kind, degree, band):
    # Without dividends early exercise of a call never pays (the CRR tree shows
    # it exactly, above); least squares can only lose value through spurious
    # exercise, by a basis-dependent amount.  The bands are that bias level.
    cfg = dict(S0=100.0, K=100.0, r=0.05, sigma=0.3, T=1.0)
    r = orc.price_american(**cfg, N=1 << 14, M=50, is_call=True, kind=kind, degree=degree)
    bs = orc.bs_price(**cfg, is_call=True)
    assert abs(r.price - bs) < band * bs


def test_laguerre_basis_matches_scipy(orc):
    from scipy.special import eval_laguerre
    for x in [0.0, 0.3, 0.9, 1.0, 1.7, 4.2]:
        psi = orc.basis_eval(orc.LAGUERRE, 5, x)
        want = [math.exp(-x / 2) * eval_laguerre(n, x) for n in range(6)]
        assert np.allclose(psi, want, rtol=1e-14, atol=1e-15)
        mono = orc.basis_eval(orc.MONOMIAL, 4, x)
        assert np.allclose(mono, [x ** a for a in range(5)], rtol=1e-15, atol=0)


# --------------------------------------------------------------------------
# The paper's own estimator (eqs. (10)-(11))
# --------------------------------------------------------------------------
def test_paper_estimator_no_dates_is_black_scholes(orc):
    r = orc.paper_estimator(**CONFIG2, N=64, m=0, is_call=True)
    assert r.price == orc.bs_price(**CONFIG2, is_call=True)


def test_paper_estimator_is_an_upper_bound(orc):
    # Section V: perfect foresight over the dates gives an upper bound; it must
    # exceed both the European value and the least-squares (lower) estimate
    for call in (False, True):
        up = orc.paper_estimator(**CONFIG1, N=4096, m=10, is_call=call)
        eu = orc.bs_price(**CONFIG1, is_call=call)
        assert up.price >= eu
    up = orc.paper_estimator(**CONFIG1, N=4096, m=10, is_call=False)
    lsm = orc.price_american(**CONFIG1, N=4096, M=11, kind=orc.MONOMIAL, degree=2)
    assert up.price > lsm.price


@pytest.mark.parametrize("m", [1, 3, 10])
def test_paper_estimator_deterministic_paths(orc, m):
    # sigma -> 0 makes every path deterministic, S_t = S0 e^{rt}, and eq. (10)'s
    # Black-Scholes value over the last interval dt = T/(m+1) becomes
    # max(S - K e^{-r dt}, 0) for a call, max(K e^{-r dt} - S, 0) for a put.
    # In-the-money call (r > 0): holding beats exercise at every point
    # (S_i - K < e^{-r dt} c_{i+1} = S_i - K e^{-r(m-i+1)dt}), so the value
    # discounted to t0 is S0 - K e^{-rT}.  In-the-money put: exercise at t_1
    # wins (K - S_1 > K e^{-r dt} - S_1), worth K e^{-r dt} - S0 at t0.  A
    # dropped discount in eq. (11) or in the final step, or the last interval
    # taken over T, moves both values by far more than the tolerance.
    r, T = 0.05, 1.0
    dt = T / (m + 1)
    call = orc.paper_estimator(S0=120.0, K=100.0, r=r, sigma=1e-9, T=T, N=1024, m=m, is_call=True)
    assert abs(call.price - (120.0 - 100.0 * math.exp(-r * T))) < 1e-8
    put = orc.paper_estimator(S0=80.0, K=100.0, r=r, sigma=1e-9, T=T, N=1024, m=m, is_call=False)
    assert abs(put.price - (100.0 * math.exp(-r * dt) - 80.0)) < 1e-8


@pytest.mark.parametrize("cfg", [CONFIG1, CONFIG2, CONFIG4])
def test_paper_estimator_one_point_call_is_black_scholes(orc, cfg):
    # m = 1: one point at t_1 = T/2 with dt = T/2.  For a call with r >= 0 the
    # Black-Scholes value over dt is at least S - K e^{-r dt} >= h(S), so the
    # pathwise maximum of eq. (10) is the Black-Scholes value itself, and by the
    # tower property e^{-r dt} E[BS(S_dt, dt)] = BS(S0, 2 dt) = BS(S0, T).  The
    # quasi-random mean over Sobol dimension 1 is a 1-D quadrature of a smooth
    # function, within 2K/N of the integral at N = 2^14 (measured about 0.8K/N).
    N = 1 << 14
    got = orc.paper_estimator(**cfg, N=N, m=1, is_call=True)
    assert abs(got.price - orc.bs_price(**cfg, is_call=True)) < 2.0 * cfg["K"] / N


# --------------------------------------------------------------------------
# Randomised QMC (digital shifts, midpoint mapping)
# --------------------------------------------------------------------------
def _shifts(R, M, seed=0x12050108):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2 ** 32, size=(R, M), dtype=np.uint64).astype(np.uint32)


def test_midpoint_inverse_normal(orc):
    from scipy.special import ndtri
    rng = np.random.default_rng(9)
    xs = [0, 1, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 1] + [int(v) for v in rng.integers(0, 2 ** 32, 3000, dtype=np.uint64)]
    for x in xs:
        z = orc.inv_normal_mid_u32(x)
        assert abs(z - ndtri((x + 0.5) / 2.0 ** 32)) < 3.2e-9
        # exact odd symmetry: cell x and cell 2^32-1-x mirror about 1/2
        assert orc.inv_normal_mid_u32((1 << 32) - 1 - x) == -z


def test_rqmc_exercise_off_covers_black_scholes(orc):
    mean, se, prices = orc.price_american_rqmc(**CONFIG1, N=1 << 12, M=16, shifts=_shifts(16, 16),
                                               allow_exercise=False)
    bs = orc.bs_price(**CONFIG1)
    assert se > 0 and len(set(prices.tolist())) == 16
    assert abs(mean - bs) < 4 * se


def test_rqmc_lsm_close_to_bermudan_tree(orc):
    mean, se, _ = orc.price_american_rqmc(**CONFIG1, N=1 << 12, M=50, shifts=_shifts(8, 50))
    berm = orc.crr_price(**CONFIG1, n=5000, style=orc.BERMUDAN, M=50)
    assert abs(mean - berm) < 0.03 + 3 * se
