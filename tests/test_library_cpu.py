"""CPU checks of the HIP library's host side: it loads, exports every symbol
the header declares, lays out workspaces sanely, rejects bad arguments before
touching a device, and builds a bridge schedule with Brownian covariance."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amqmc.h")


@pytest.fixture(scope="module")
def amq():
    import paper_1205_0106_amd as amq
    if not os.path.exists(amq.LIB_PATH):
        pytest.skip("libamqmc.so not built")
    amq.lib()
    return amq


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(am_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_exports_every_declared_symbol(amq):
    names = _declared_functions()
    assert len(names) >= 10
    L = ctypes.CDLL(amq.LIB_PATH)
    for n in names:
        assert hasattr(L, n), f"{n} not exported"


def test_max_dates(amq):
    assert amq.am_max_dates() >= 365


def test_storage_rule(amq):
    # FP32-bulk requests below AM_FP32_MIN_PATHS paths are stored in binary64,
    # and their workspace is the binary64 one
    lo = amq.AM_FP32_MIN_PATHS
    assert lo == 1 << 14
    assert amq.am_storage_dtype(lo - 1, "fp32") == amq.AM_FP64
    assert amq.am_storage_dtype(lo, "fp32") == amq.AM_FP32_BULK
    assert amq.am_storage_dtype(10, "fp64") == amq.AM_FP64
    assert amq.lib().am_storage_dtype(1000, 7) == -1
    b = amq.make_basis("monomial", 2)
    assert amq.am_workspace_bytes(lo - 1, 20, b, "fp32") == amq.am_workspace_bytes(lo - 1, 20, b, "fp64")
    assert amq.am_workspace_bytes(lo, 20, b, "fp32") < amq.am_workspace_bytes(lo, 20, b, "fp64")


def test_shutdown_without_device_work(amq):
    # nothing set up yet on this host: releases nothing, touches no device
    assert amq.lib().am_shutdown() == amq.AM_OK


@pytest.mark.parametrize("N,M,dt", [(16384, 50, "fp64"), (1 << 20, 100, "fp32"), (1000, 3, "fp64")])
def test_workspace_layout(amq, N, M, dt):
    b = amq.make_basis("monomial", 2)
    lay = amq.am_workspace_layout(N, M, b, dt)
    s = 8 if dt == "fp64" else 4
    assert lay.ld >= N and lay.ld % 32768 == 0
    assert lay.off_S == 0 and lay.off_PV >= M * lay.ld * s
    for off in (lay.off_PV, lay.off_rec, lay.off_result):
        assert off % 256 == 0
    assert lay.total == amq.am_workspace_bytes(N, M, b, dt) and lay.total > lay.off_result


@pytest.mark.parametrize("bad", [
    dict(S0=-1.0), dict(K=0.0), dict(sigma=0.0), dict(T=float("nan")), dict(r=float("inf")),
])
def test_invalid_params_rejected_before_device(amq, bad):
    kw = dict(S0=36.0, K=40.0, r=0.06, sigma=0.2, T=1.0)
    kw.update(bad)
    p = amq.make_params(**kw)
    with pytest.raises(amq.AmError) as e:
        amq.am_price_american(p, 4096, 10, amq.make_basis("monomial", 2), "fp64")
    assert e.value.code == amq.AM_EINVAL


@pytest.mark.parametrize("args,code", [
    (dict(n_paths=2, n_dates=10, degree=2), -1),       # fewer paths than p + 1
    (dict(n_paths=4096, n_dates=0, degree=2), -1),
    (dict(n_paths=4096, n_dates=100000, degree=2), -4),
    (dict(n_paths=4096, n_dates=641, degree=2), -4),
    (dict(n_paths=4096, n_dates=10, degree=7), -1),
    (dict(n_paths=1 << 33, n_dates=10, degree=2), -4),
])
def test_invalid_shapes_rejected(amq, args, code):
    p = amq.make_params(36.0, 40.0, 0.06, 0.2, 1.0)
    with pytest.raises(amq.AmError) as e:
        amq.am_price_american(p, args["n_paths"], args["n_dates"],
                              amq.make_basis("monomial", args["degree"]), "fp64")
    assert e.value.code == code


def test_bad_enums_rejected(amq):
    p = amq.make_params(36.0, 40.0, 0.06, 0.2, 1.0)
    with pytest.raises(amq.AmError):
        amq.am_price_american(p, 4096, 10, amq.am_basis(5, 2), "fp64")
    with pytest.raises(amq.AmError):
        amq.am_price_american(p, 4096, 10, amq.make_basis("monomial", 2), 7)


@pytest.mark.parametrize("M", [1, 2, 3, 7, 50, 100, 252, 365, 640])
def test_schedule_gives_brownian_covariance(amq, M):
    # apply the library's depth-first schedule to unit vectors: the map W = Bz
    # must have covariance min(t_i, t_j) (dt = 1 units here)
    sc = amq.am_debug_schedule(M)
    B = np.zeros((M + 1, M))      # row = date 0..M, col = Sobol dim
    for q in range(M):
        m, l, r = sc["m"][q], sc["left"][q], sc["right"][q]
        B[m] = sc["wl"][q] * B[l] + sc["wr"][q] * B[r]
        B[m, sc["dim"][q]] += sc["sd"][q]
    cov = B[1:] @ B[1:].T
    t = np.arange(1, M + 1, dtype=float)
    assert np.abs(cov - np.minimum.outer(t, t)).max() < 1e-9 * M


@pytest.mark.parametrize("M", [1, 2, 7, 100, 252, 640])
def test_schedule_weights_carry_drift(amq, M):
    # the kernels run the schedule on the log-price a + b t + c W(t): below the
    # root the two interpolation weights must sum to 1 and reproduce the
    # linear drift exactly (b m = wl b l + wr b r); the root reads its anchor
    # (log S0 + b M) with weight 1
    sc = amq.am_debug_schedule(M)
    assert sc["wl"][0] == 1.0 and sc["wr"][0] == 0.0 and sc["m"][0] == M
    for q in range(1, M):
        wl, wr = sc["wl"][q], sc["wr"][q]
        l, r, m = sc["left"][q], sc["right"][q], sc["m"][q]
        assert abs(wl + wr - 1.0) <= 2.3e-16
        assert abs(wl * l + wr * r - m) <= 1e-12 * M


@pytest.mark.parametrize("M", [1, 5, 50, 365])
def test_schedule_dimension_numbering_is_breadth_first(amq, orc, M):
    # each date must read the same Sobol dimension as in the breadth-first
    # bisection (the construction order may differ)
    sc = amq.am_debug_schedule(M)
    om, ol, orr = orc.bridge_nodes(M)
    want = {int(m): q for q, m in enumerate(om)}
    for q in range(M):
        assert want[int(sc["m"][q])] == sc["dim"][q]
        if q > 0:
            assert (sc["left"][q], sc["right"][q]) == (ol[sc["dim"][q]], orr[sc["dim"][q]])


def test_binding_raises_when_library_missing(monkeypatch):
    import paper_1205_0106_amd as amq
    monkeypatch.setattr(amq, "_lib", None)
    monkeypatch.setattr(amq, "LIB_PATH", "/nonexistent/libamqmc.so")
    with pytest.raises(ImportError):
        amq.lib()


def test_batch_workspace_sizing(amq):
    from paper_1205_0106_amd.workloads import batch_options
    specs = batch_options(32, seed=5)
    opts = amq.make_options(specs)
    b = amq.make_basis("monomial", 2)
    n32 = amq.am_batch_workspace_bytes(opts, b, "fp32")
    n64 = amq.am_batch_workspace_bytes(opts, b, "fp64")
    need = sum(d["n_paths"] * d["n_dates"] for d in specs)
    assert n32 >= 4 * need and n64 >= 8 * need and n64 > n32
    bad = amq.make_options([dict(specs[0], sigma=-1.0)])
    assert amq.am_batch_workspace_bytes(bad, b, "fp32") == 0


@pytest.mark.parametrize("field, value", [("n_streams", 0), ("n_streams", 9), ("max_batch_requests", 0),
                                          ("dtype", 7), ("large_tile", 2), ("large_tile", -1)])
def test_server_config_rejected_before_device(amq, field, value):
    # the server's configuration is checked on the host, before any device call
    cfg = amq.am_server_config(1 << 30, 2e9, 8, 2, amq.make_basis("monomial", 2), amq.AM_FP32_BULK, 0)
    setattr(cfg, field, value)
    h = ctypes.c_void_p()
    assert amq.lib().am_server_create(ctypes.byref(cfg), ctypes.byref(h)) == amq.AM_EINVAL
    assert field in amq.am_last_error() or field == "dtype"


def test_math_tables_match_their_definitions():
    # the generator's logarithm and exponential tables, recomputed from their
    # definitions at 60 digits and rounded once, equal the constants compiled
    # into the kernels
    import subprocess
    import sys
    script = os.path.join(ROOT, "paper_1205_0106_amd", "csrc", "gen_math_tables.py")
    r = subprocess.run([sys.executable, script, "--check"], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr


def test_header_is_plain_c(tmp_path):
    # the boundary header compiles as ISO C99 (no C++ or HIP types), so any C
    # caller can use it
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use_header.c"
    src.write_text('#include "amqmc.h"\n'
                   "int use(void) { am_server_config c = {0}; am_params p = {0};\n"
                   "  (void)c; (void)p; return am_max_dates(); }\n")
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                        os.path.join(ROOT, "include"), "-c", str(src), "-o", str(tmp_path / "u.o")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
