"""Planted-mistake checks for the oracle's pins (CPU only).

Each case edits a copy of the oracle's C source to introduce one plausible
mistake (a dropped term, a wrong sign, a wrong index, swapped operands),
compiles it, routes the oracle through that build and runs the pin suite.  At
least one pin must fail for every mutant; otherwise that part of the oracle
would be unpinned.
"""
import os

import numpy as np
import pytest

import tests.test_oracle_pricing as P
import tests.test_oracle_sobol_normal_bridge as B

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "amq_oracle.c")

# (name, exact text in the source, replacement)
MUTANTS = [
    ("gray code dropped", "uint64_t g = n ^ (n >> 1);", "uint64_t g = n;"),
    ("recurrence loses m_{k-s}", "uint64_t v = m[k - s] ^ (m[k - s] << s);",
     "uint64_t v = (m[k - s] << s);"),
    ("recurrence shift off by one", "if (ai) v ^= m[k - i] << i;", "if (ai) v ^= m[k - i] << (i + 1);"),
    ("direction bit misplaced", "(uint32_t)(m[b + 1] << (31 - b));", "(uint32_t)(m[b + 1] << (32 - b - 1 - (b > 3)));"),
    ("central coefficient typo", "41.39119773534", "41.93119773534"),
    ("tail coefficient sign", "0.1607979714918209", "-0.1607979714918209"),
    ("tail uses wrong side", "return bsm_tail((4294967296.0 - (double)x) * s);",
     "return bsm_tail((double)x * s);"),
    ("central/tail threshold", "if (fabs(y) < 0.42) return bsm_central(y);\n    if (y < 0.0) return -bsm_tail((double)x * s);",
     "if (fabs(y) < 0.46) return bsm_central(y);\n    if (y < 0.0) return -bsm_tail((double)x * s);"),
    ("bridge weights swapped", "double mean = ((tr - tm) * W[nl[q]] + (tm - tl) * W[nr[q]]) / (tr - tl);",
     "double mean = ((tm - tl) * W[nl[q]] + (tr - tm) * W[nr[q]]) / (tr - tl);"),
    ("bridge sd without sqrt", "double sd = sqrt((tm - tl) * (tr - tm) / (tr - tl));",
     "double sd = (tm - tl) * (tr - tm) / (tr - tl);"),
    ("bridge root scale", "W[M] = sqrt(T) * z[0];", "W[M] = T * z[0];"),
    ("bridge midpoint rounding", "int m = (l + r) / 2;\n        m_out[q] = m;", "int m = (l + r + 1) / 2;\n        m_out[q] = m;"),
    ("drift sign", "double drift = p->r - 0.5 * p->sigma * p->sigma;\n    for (int64_t c = 0; c < count; ++c) {",
     "double drift = p->r + 0.5 * p->sigma * p->sigma;\n    for (int64_t c = 0; c < count; ++c) {"),
    ("origin not skipped", "uint64_t n = (uint64_t)(first + c) + 1u;       /* skip the origin */",
     "uint64_t n = (uint64_t)(first + c);"),
    ("target not discounted", ": CF[i] * exp(-p->r * (t[tau[i]] - t[k]));", ": CF[i];"),
    ("target discounted to t0", ": CF[i] * exp(-p->r * (t[tau[i]] - t[k]));",
     ": CF[i] * exp(-p->r * t[tau[i]]);"),
    ("out-of-the-money rows regressed", "if (!(h > 0.0)) continue;\n                or_basis_eval(kind, degree, s / p->K, psi);\n                double y",
     "or_basis_eval(kind, degree, s / p->K, psi);\n                double y"),
    ("exercise test reversed", "if (h > cont) {\n                    CF[i] = h;", "if (h < cont) {\n                    CF[i] = h;"),
    ("first date never visited", "for (int k = M - 1; k >= 1; --k) {", "for (int k = M - 1; k >= 2; --k) {"),
    ("pv discounted at maturity", ": CF[i] * exp(-p->r * t[tau[i]]);", ": CF[i] * exp(-p->r * p->T);"),
    ("store32 paths not rounded", "#define SV(x) (store32 ? rd32(x) : (x))", "#define SV(x) (x)"),
    ("store32 cashflow not rounded", "if (store32) PV32[i] = rd32(h * exp(-p->r * t[k]));",
     "if (store32) PV32[i] = h * exp(-p->r * t[k]);"),
    ("store32 rounds before discounting", "if (store32) PV32[i] = rd32(h * exp(-p->r * t[k]));",
     "if (store32) PV32[i] = rd32(h) * exp(-p->r * t[k]);"),
    ("store32 terminal cashflow not rounded", "if (store32) PV32[i] = rd32(CF[i] * exp(-p->r * t[M]));",
     "if (store32) PV32[i] = CF[i] * exp(-p->r * t[M]);"),
    ("store32 target left at t0", "double y = store32 ? PV32[i] * exp(p->r * t[k])", "double y = store32 ? PV32[i]"),
    ("store32 rounds toward zero", "static double rd32(double v) { return (double)(float)v; }",
     "static double rd32(double v) { float f = (float)v; if (fabs((double)f) > fabs(v)) f = nextafterf(f, 0.0f); return (double)f; }"),
    ("givens rotation sign", "psi[l] = -s * t1 + c * t2;", "psi[l] = s * t1 + c * t2;"),
    ("back substitution index", "for (int l = j + 1; l < np; ++l) v -= R[j][l] * beta[l];",
     "for (int l = j + 1; l < np; ++l) v -= R[l][j] * beta[l];"),
    ("laguerre recurrence", "double l1 = ((2.0 * n + 1.0 - x) * l0 - (double)n * lm1) / (double)(n + 1);",
     "double l1 = ((2.0 * n + 1.0 - x) * l0 + (double)n * lm1) / (double)(n + 1);"),
    ("laguerre weight", "double w = exp(-0.5 * x);", "double w = exp(-x);"),
    ("t0 exercise dropped", "if (h0 > mean) { res->price = h0;", "if (0) { res->price = h0;"),
    ("variance divisor", "double var = N > 1 ? ks_val(&ss) / (double)(N - 1) : 0.0;\n    double se = sqrt(var) / sqrt((double)N);",
     "double var = N > 1 ? ks_val(&ss) / (double)(N) : 0.0;\n    double se = sqrt(var) / sqrt((double)N);"),
    ("bs d2 sign", "double d2 = d1 - sq;", "double d2 = d1 + sq;"),
    ("crr probability", "double q = (exp(r * dt) - d) / (u - d);", "double q = (exp(r * dt) - d) / (u + d);"),
    ("digital shift ignored", "z[q] = shift ? or_inv_normal_mid_u32(or_sobol_int(V, q, n) ^ shift[q])",
     "z[q] = shift ? or_inv_normal_mid_u32(or_sobol_int(V, q, n))"),
    ("midpoint offset dropped", "double y = ((double)x + 0.5 - 2147483648.0) * s;",
     "double y = ((double)x - 2147483648.0) * s;"),
    ("paper final discount dropped", "c[i] = disc * v;", "c[i] = v;"),
    ("paper last interval over T", "or_bs_price(S, p->K, p->r, p->sigma, dt, p->is_call)",
     "or_bs_price(S, p->K, p->r, p->sigma, p->T, p->is_call)"),
    ("paper backward discount dropped", ": disc * v;", ": v;"),
    ("paper grid spacing T/m", "double dt = p->T / (double)(m + 1);", "double dt = p->T / (double)m;"),
    ("paper pathwise maximum dropped", "v = h > cont ? h : cont;", "v = cont;"),
    ("paper horizon is T", "double horizon = dt * (double)m;", "double horizon = p->T;"),
    ("crr bermudan stride", "int ex = (style == OR_AMERICAN) || (style == OR_BERMUDAN && i % stride == 0);",
     "int ex = (style == OR_AMERICAN) || (style == OR_BERMUDAN && i % stride == 1);"),
]


def _pin_suite(orc):
    """Every CPU pin, as zero-argument callables (fast sizes)."""
    c1, c2, c4 = P.CONFIG1, P.CONFIG2, P.CONFIG4
    return [
        lambda: B.test_sobol_matches_scipy_bit_exact(orc, 50, 1025),
        lambda: B.test_sobol_matches_torch_30bit(orc),
        lambda: B.test_sobol_first_dimension_is_van_der_corput_in_gray_order(orc),
        lambda: B.test_inverse_normal_within_moro_bound(orc),
        lambda: B.test_inverse_normal_integer_odd_symmetry(orc),
        lambda: B.test_inverse_normal_monotone(orc),
        lambda: B.test_inverse_normal_u32_matches_real_argument(orc),
        lambda: B.test_bridge_covariance_is_brownian(orc, 7),
        lambda: B.test_bridge_covariance_is_brownian(orc, 50),
        lambda: B.test_bridge_nodes_cover_each_date_once(orc, 50),
        lambda: B.test_bridge_single_date_is_scaled_normal(orc),
        lambda: P.test_bs_put_call_parity(orc),
        lambda: P.test_bs_textbook_value(orc),
        lambda: P.test_crr_european_converges_to_bs(orc, c1),
        lambda: P.test_crr_ordering_and_bermudan_monotone(orc),
        lambda: P.test_crr_bermudan_limits(orc),
        lambda: P.test_longstaff_schwartz_worked_example(orc),
        lambda: P.test_interpolating_regression_is_perfect_foresight(orc, 0, 2),
        lambda: P.test_interpolating_regression_is_perfect_foresight(orc, 1, 3),
        lambda: P.test_hand_computed_two_path_case(orc),
        lambda: P.test_single_date_equals_exercise_off(orc),
        lambda: P.test_store32_rounds_paths_and_cashflows_to_nearest(orc, False, 0, 2),
        lambda: P.test_store32_exact_when_storage_is_exact(orc),
        lambda: P.test_exercise_off_matches_black_scholes(orc, c1, 1 << 12),
        lambda: P.test_exercise_off_matches_black_scholes(orc, c4, 1 << 12),
        lambda: P.test_laguerre_basis_matches_scipy(orc),
        lambda: P.test_config1_lsm_close_to_bermudan_tree(orc),
        lambda: P.test_midpoint_inverse_normal(orc),
        lambda: P.test_rqmc_exercise_off_covers_black_scholes(orc),
        lambda: P.test_paper_estimator_no_dates_is_black_scholes(orc),
        lambda: P.test_paper_estimator_deterministic_paths(orc, 3),
        lambda: P.test_paper_estimator_one_point_call_is_black_scholes(orc, P.CONFIG2),
    ]


def _fails(fn):
    try:
        with np.errstate(all="ignore"):
            fn()
    except Exception:
        return True
    return False


def test_mutants_are_killed(orc, tmp_path):
    src = open(SRC).read()
    survivors = []
    for i, (name, old, new) in enumerate(MUTANTS):
        assert src.count(old) == 1, f"mutation anchor not unique/found: {name}"
        so = orc.compile_variant(src.replace(old, new), str(tmp_path / f"mut{i}.so"))
        with orc.swapped_library(so):
            killed = any(_fails(fn) for fn in _pin_suite(orc))
        if not killed:
            survivors.append(name)
    assert not survivors, f"mutants not caught by any pin: {survivors}"


def test_unmutated_source_passes_the_suite(orc, tmp_path):
    so = orc.compile_variant(open(SRC).read(), str(tmp_path / "clean.so"))
    with orc.swapped_library(so):
        failed = [i for i, fn in enumerate(_pin_suite(orc)) if _fails(fn)]
    assert not failed
