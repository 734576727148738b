"""FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

This package wraps ``liboracle.so`` (plain C, binary64, single-threaded) with
ctypes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it.  The product path (the HIP library and its
binding in ``paper_1205_0106_amd``) never imports, links or calls anything
here, and this package never imports the product.

The Sobol direction numbers are derived here from the published Joe–Kuo
primitive polynomials and initial values (read from SciPy's data file with
``allow_pickle=False``) by the oracle's own recurrence.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "amq_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MONOMIAL = 0
LAGUERRE = 1
EUROPEAN, AMERICAN, BERMUDAN = 0, 1, 2
BETA_STRIDE = 16


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc: -O2, no fast-math, no FMA contraction."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("S0", ctypes.c_double), ("K", ctypes.c_double), ("r", ctypes.c_double),
                ("sigma", ctypes.c_double), ("T", ctypes.c_double),
                ("is_call", ctypes.c_int32), ("allow_exercise", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("price", ctypes.c_double), ("std_err", ctypes.c_double),
                ("mean_pv", ctypes.c_double), ("t0_exercise", ctypes.c_int32),
                ("n_skipped", ctypes.c_int32)]


@dataclass
class OracleResult:
    price: float
    std_err: float
    mean_pv: float
    t0_exercise: bool
    n_skipped: int


_lib = None


def compile_variant(src_text: str, out_path: str) -> str:
    """Compile an edited copy of the oracle source (used by the mutation
    tests, which plant mistakes to show that the pins catch them)."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                    "-I", _HERE, "-o", out_path, src, "-lm"], check=True)
    return out_path


class swapped_library:
    """Context manager: route every oracle call through another build."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _configure(ctypes.CDLL(self.path))
        _JK_CACHE.clear()
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        _JK_CACHE.clear()
        return False


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def _configure(L):
    """Declare the C signatures on a loaded oracle library."""
    P = ctypes.POINTER
    L.or_sobol_directions.argtypes = [ctypes.c_int, P(ctypes.c_int64), P(ctypes.c_int64),
                                      ctypes.c_int, P(ctypes.c_uint32)]
    L.or_sobol_int.argtypes = [P(ctypes.c_uint32), ctypes.c_int, ctypes.c_uint64]
    L.or_sobol_int.restype = ctypes.c_uint32
    L.or_sobol_block.argtypes = [P(ctypes.c_uint32), ctypes.c_int, ctypes.c_uint64,
                                 ctypes.c_int64, P(ctypes.c_uint32)]
    L.or_inv_normal.argtypes = [ctypes.c_double]
    L.or_inv_normal.restype = ctypes.c_double
    L.or_inv_normal_u32.argtypes = [ctypes.c_uint32]
    L.or_inv_normal_u32.restype = ctypes.c_double
    L.or_bridge_nodes.argtypes = [ctypes.c_int, P(ctypes.c_int32), P(ctypes.c_int32),
                                  P(ctypes.c_int32)]
    L.or_bridge_apply.argtypes = [ctypes.c_int, ctypes.c_double, P(ctypes.c_double),
                                  P(ctypes.c_double)]
    L.or_paths.argtypes = [P(_Params), P(ctypes.c_uint32), ctypes.c_int64, ctypes.c_int,
                           P(ctypes.c_double)]
    L.or_inv_normal_mid_u32.argtypes = [ctypes.c_uint32]
    L.or_inv_normal_mid_u32.restype = ctypes.c_double
    L.or_price_american_shifted.argtypes = [P(_Params), P(ctypes.c_uint32), ctypes.c_int64,
                                            ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            P(ctypes.c_uint32), P(_Result), P(ctypes.c_double),
                                            P(ctypes.c_int32), P(ctypes.c_double)]
    L.or_price_american_stored.argtypes = [P(_Params), P(ctypes.c_uint32), ctypes.c_int64,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           P(ctypes.c_uint32), ctypes.c_int, P(_Result),
                                           P(ctypes.c_double), P(ctypes.c_int32),
                                           P(ctypes.c_double)]
    L.or_paths_range_shifted.argtypes = [P(_Params), P(ctypes.c_uint32), ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_int, P(ctypes.c_uint32),
                                         P(ctypes.c_double)]
    L.or_paths_range.argtypes = [P(_Params), P(ctypes.c_uint32), ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_int, P(ctypes.c_double)]
    L.or_basis_eval.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                P(ctypes.c_double)]
    L.or_lsm_on_paths_stored.argtypes = [P(ctypes.c_double), ctypes.c_int64, ctypes.c_int,
                                         P(_Params), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         P(_Result), P(ctypes.c_double), P(ctypes.c_int32),
                                         P(ctypes.c_int32), P(ctypes.c_double)]
    L.or_lsm_on_paths.argtypes = [P(ctypes.c_double), ctypes.c_int64, ctypes.c_int,
                                  P(_Params), ctypes.c_int, ctypes.c_int, P(_Result),
                                  P(ctypes.c_double), P(ctypes.c_int32),
                                  P(ctypes.c_int32), P(ctypes.c_double)]
    L.or_price_american.argtypes = [P(_Params), P(ctypes.c_uint32), ctypes.c_int64,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, P(_Result),
                                    P(ctypes.c_double), P(ctypes.c_int32),
                                    P(ctypes.c_double)]
    L.or_paper_estimator.argtypes = [P(_Params), P(ctypes.c_uint32), ctypes.c_int64,
                                     ctypes.c_int, P(_Result)]
    L.or_bs_price.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int]
    L.or_bs_price.restype = ctypes.c_double
    L.or_crr_price.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int] * 4
    L.or_crr_price.restype = ctypes.c_double
    return L


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# --------------------------------------------------------------------------
# Sobol direction numbers (Joe–Kuo), derived by the oracle's own recurrence.
# --------------------------------------------------------------------------
_JK_CACHE: dict[int, np.ndarray] = {}


def joe_kuo_data():
    """Primitive polynomials and initial direction values (Joe & Kuo 2008).

    Read from the data file SciPy ships (plain arrays, no pickle)."""
    import scipy.stats
    path = os.path.join(os.path.dirname(scipy.stats.__file__), "_sobol_direction_numbers.npz")
    with np.load(path, allow_pickle=False) as d:
        return np.ascontiguousarray(d["poly"], dtype=np.int64), \
            np.ascontiguousarray(d["vinit"], dtype=np.int64)


def directions(ndim: int) -> np.ndarray:
    """uint32 [ndim][32]: V[j][b] is the direction number of bit b, dim j."""
    if ndim not in _JK_CACHE:
        poly, vinit = joe_kuo_data()
        if ndim > poly.shape[0]:
            raise ValueError("dimension beyond the Joe–Kuo table")
        V = np.zeros((ndim, 32), dtype=np.uint32)
        rc = lib().or_sobol_directions(ndim, _ptr(poly, ctypes.c_int64),
                                       _ptr(vinit, ctypes.c_int64), vinit.shape[1],
                                       _ptr(V, ctypes.c_uint32))
        if rc != 0:
            raise RuntimeError("or_sobol_directions failed")
        _JK_CACHE[ndim] = V
    return _JK_CACHE[ndim]


def sobol_block(ndim: int, first: int, count: int) -> np.ndarray:
    """uint32 [count][ndim] Sobol integers for indices first..first+count-1."""
    V = directions(ndim)
    out = np.zeros((count, ndim), dtype=np.uint32)
    lib().or_sobol_block(_ptr(V, ctypes.c_uint32), ndim, first, count,
                         _ptr(out, ctypes.c_uint32))
    return out


def inv_normal(u: float) -> float:
    return lib().or_inv_normal(float(u))


def inv_normal_u32(x: int) -> float:
    return lib().or_inv_normal_u32(int(x))


def bridge_nodes(M: int):
    m = np.zeros(M, dtype=np.int32)
    left = np.zeros(M, dtype=np.int32)
    right = np.zeros(M, dtype=np.int32)
    rc = lib().or_bridge_nodes(M, _ptr(m, ctypes.c_int32), _ptr(left, ctypes.c_int32),
                               _ptr(right, ctypes.c_int32))
    if rc != 0:
        raise RuntimeError("or_bridge_nodes failed")
    return m, left, right


def bridge_apply(M: int, T: float, z: np.ndarray) -> np.ndarray:
    z = np.ascontiguousarray(z, dtype=np.float64)
    W = np.zeros(M + 1, dtype=np.float64)
    lib().or_bridge_apply(M, T, _ptr(z, ctypes.c_double), _ptr(W, ctypes.c_double))
    return W


def _params(S0, K, r, sigma, T, is_call, allow_exercise) -> _Params:
    return _Params(float(S0), float(K), float(r), float(sigma), float(T),
                   int(bool(is_call)), int(bool(allow_exercise)))


def paths(S0, K, r, sigma, T, N: int, M: int, is_call=False) -> np.ndarray:
    """float64 [M][N]: row k-1 is S at t_k = kT/M for every path."""
    p = _params(S0, K, r, sigma, T, is_call, True)
    V = directions(M)
    S = np.zeros((M, N), dtype=np.float64)
    rc = lib().or_paths(ctypes.byref(p), _ptr(V, ctypes.c_uint32), N, M, _ptr(S, ctypes.c_double))
    if rc != 0:
        raise RuntimeError("or_paths failed")
    return S


def paths_range(S0, K, r, sigma, T, first: int, count: int, M: int) -> np.ndarray:
    """float64 [M][count]: paths first..first+count-1 (same points as paths())."""
    p = _params(S0, K, r, sigma, T, False, True)
    V = directions(M)
    S = np.zeros((M, count), dtype=np.float64)
    rc = lib().or_paths_range(ctypes.byref(p), _ptr(V, ctypes.c_uint32), first, count, M,
                              _ptr(S, ctypes.c_double))
    if rc != 0:
        raise RuntimeError("or_paths_range failed")
    return S


def basis_eval(kind: int, degree: int, x: float) -> np.ndarray:
    psi = np.zeros(8, dtype=np.float64)
    n = lib().or_basis_eval(kind, degree, float(x), _ptr(psi, ctypes.c_double))
    return psi[:n].copy()


def lsm_on_paths(S: np.ndarray, S0, K, r, sigma, T, *, is_call=False, allow_exercise=True,
                 kind=MONOMIAL, degree=2, detail=False, store32=False):
    """Least-squares backward induction on a given path matrix S[M][N].
    store32: binary32 storage (path values read rounded to binary32, cashflows
    held discounted to t0 and rounded to binary32), binary64 arithmetic."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    M, N = S.shape
    p = _params(S0, K, r, sigma, T, is_call, allow_exercise)
    res = _Result()
    beta = np.zeros((M + 1, BETA_STRIDE), dtype=np.float64)
    nitm = np.zeros(M + 1, dtype=np.int32)
    tau = np.zeros(N, dtype=np.int32)
    pv = np.zeros(N, dtype=np.float64)
    rc = lib().or_lsm_on_paths_stored(_ptr(S, ctypes.c_double), N, M, ctypes.byref(p), kind, degree,
                                      int(bool(store32)), ctypes.byref(res), _ptr(beta, ctypes.c_double),
                                      _ptr(nitm, ctypes.c_int32), _ptr(tau, ctypes.c_int32),
                                      _ptr(pv, ctypes.c_double))
    if rc != 0:
        raise RuntimeError(f"or_lsm_on_paths failed ({rc})")
    out = OracleResult(res.price, res.std_err, res.mean_pv, bool(res.t0_exercise), res.n_skipped)
    if detail:
        return out, dict(beta=beta, nitm=nitm, tau=tau, pv=pv)
    return out


def price_american(S0, K, r, sigma, T, N: int, M: int, *, is_call=False, allow_exercise=True,
                   kind=MONOMIAL, degree=2, detail=False, store32=False):
    """The full oracle on Sobol points: returns OracleResult (and details).
    store32: binary32 storage of the path values and cashflows (the FP32-bulk
    reading; see lsm_on_paths), binary64 arithmetic."""
    p = _params(S0, K, r, sigma, T, is_call, allow_exercise)
    V = directions(M)
    res = _Result()
    beta = np.zeros((M + 1, BETA_STRIDE), dtype=np.float64)
    nitm = np.zeros(M + 1, dtype=np.int32)
    pv = np.zeros(N, dtype=np.float64) if detail else None
    rc = lib().or_price_american_stored(ctypes.byref(p), _ptr(V, ctypes.c_uint32), N, M, kind,
                                        degree, None, int(bool(store32)), ctypes.byref(res),
                                        _ptr(beta, ctypes.c_double), _ptr(nitm, ctypes.c_int32),
                                        _ptr(pv, ctypes.c_double) if pv is not None else None)
    if rc != 0:
        raise RuntimeError(f"or_price_american failed ({rc})")
    out = OracleResult(res.price, res.std_err, res.mean_pv, bool(res.t0_exercise), res.n_skipped)
    if detail:
        return out, dict(beta=beta, nitm=nitm, pv=pv)
    return out


def inv_normal_mid_u32(x: int) -> float:
    return lib().or_inv_normal_mid_u32(int(x))


def price_american_rqmc(S0, K, r, sigma, T, N: int, M: int, shifts: np.ndarray, *, is_call=False,
                        allow_exercise=True, kind=MONOMIAL, degree=2, store32=False):
    """Randomised QMC: one price per digital-shift replicate (shifts: uint32
    [R][M]).  Returns (mean, sd/sqrt(R), per-replicate prices)."""
    p = _params(S0, K, r, sigma, T, is_call, allow_exercise)
    V = directions(M)
    shifts = np.ascontiguousarray(shifts, dtype=np.uint32)
    prices = []
    for row in shifts:
        res = _Result()
        row = np.ascontiguousarray(row)
        rc = lib().or_price_american_stored(ctypes.byref(p), _ptr(V, ctypes.c_uint32), N, M, kind,
                                            degree, _ptr(row, ctypes.c_uint32), int(bool(store32)),
                                            ctypes.byref(res), None, None, None)
        if rc != 0:
            raise RuntimeError("or_price_american_stored failed")
        prices.append(res.price)
    prices = np.array(prices)
    R = len(prices)
    se = prices.std(ddof=1) / np.sqrt(R) if R > 1 else 0.0
    return float(prices.mean()), float(se), prices


def paper_estimator(S0, K, r, sigma, T, N: int, m: int, *, is_call=True) -> OracleResult:
    p = _params(S0, K, r, sigma, T, is_call, True)
    V = directions(max(m, 1))
    res = _Result()
    rc = lib().or_paper_estimator(ctypes.byref(p), _ptr(V, ctypes.c_uint32), N, m, ctypes.byref(res))
    if rc != 0:
        raise RuntimeError("or_paper_estimator failed")
    return OracleResult(res.price, res.std_err, res.mean_pv, bool(res.t0_exercise), res.n_skipped)


def bs_price(S0, K, r, sigma, T, is_call=False) -> float:
    return lib().or_bs_price(S0, K, r, sigma, T, int(bool(is_call)))


def crr_price(S0, K, r, sigma, T, *, is_call=False, n=5000, style=AMERICAN, M=0) -> float:
    return lib().or_crr_price(S0, K, r, sigma, T, int(bool(is_call)), n, style, M)
