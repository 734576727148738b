"""MI355X quasi-Monte Carlo American option engine — Python binding.

Thin ctypes layer over ``libamqmc.so`` (C-ABI in ``include/amqmc.h``).  Every
step of the pricing path runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch provides device memory (the workspace) and
streams for the asynchronous entry point.  Importing the binding never falls
back to anything else: if the library is missing the calls raise.

Method: Cvetanoska & Stojanovski, "Using High Performance Computing and Monte
Carlo Simulation for Pricing American Options" (Sections III.D, III.E, V).
"""
from __future__ import annotations

import atexit
import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamqmc.so")

AM_OK, AM_EINVAL, AM_ENOMEM, AM_EDEVICE, AM_EDIM, AM_EWORKSPACE, AM_ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
AM_BASIS_MONOMIAL, AM_BASIS_LAGUERRE = 0, 1
AM_FP64, AM_FP32_BULK = 0, 1
AM_MAX_DEGREE = 6
AM_FP32_MIN_PATHS = 16384   # FP32-bulk requests below this path count are stored in binary64
AM_SCRATCH_BYTES = 134217728   # fixed device workspace of am_price_american_noalloc
REC = 40            # doubles per per-date record in the workspace

_BASIS_NAMES = {"monomial": AM_BASIS_MONOMIAL, "laguerre": AM_BASIS_LAGUERRE}
_DTYPE_NAMES = {"fp64": AM_FP64, "f64": AM_FP64, "fp32": AM_FP32_BULK, "fp32_bulk": AM_FP32_BULK,
                "f32": AM_FP32_BULK}


class AmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class am_params(ctypes.Structure):
    """Option and model parameters (S0, strike K, rate r, volatility sigma, expiry T)."""
    _fields_ = [("S0", ctypes.c_double), ("K", ctypes.c_double), ("r", ctypes.c_double),
                ("sigma", ctypes.c_double), ("T", ctypes.c_double),
                ("is_call", ctypes.c_int32), ("allow_exercise", ctypes.c_int32)]


class am_basis(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("degree", ctypes.c_int32)]


class am_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_batch_path_steps", ctypes.c_double),
                ("max_batch_requests", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("basis", am_basis), ("dtype", ctypes.c_int32), ("large_tile", ctypes.c_int32)]


class am_result(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_uint64), ("price", ctypes.c_double),
                ("std_err", ctypes.c_double), ("t_arrival", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class am_option(ctypes.Structure):
    _fields_ = [("params", am_params), ("n_paths", ctypes.c_int64), ("n_dates", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


def make_params(S0, K, r, sigma, T, is_call=False, allow_exercise=True) -> am_params:
    return am_params(float(S0), float(K), float(r), float(sigma), float(T),
                     int(bool(is_call)), int(bool(allow_exercise)))


def make_basis(kind="monomial", degree=2) -> am_basis:
    if isinstance(kind, str):
        kind = _BASIS_NAMES[kind.lower()]
    return am_basis(int(kind), int(degree))


def _dtype(d) -> int:
    if isinstance(d, str):
        return _DTYPE_NAMES[d.lower()]
    return int(d)


_lib = None


def lib():
    """Load libamqmc.so; raise (never fall back) if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "(or python -m paper_1205_0106_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.am_storage_dtype.argtypes = [ctypes.c_int64, ctypes.c_int32]
        L.am_storage_dtype.restype = ctypes.c_int32
        L.am_shutdown.argtypes = []
        L.am_shutdown.restype = ctypes.c_int
        i64, i32, sz, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t, ctypes.c_double
        L.am_price_american.argtypes = [P(am_params), i64, i32, am_basis, i32, P(dbl), P(dbl)]
        L.am_price_american.restype = ctypes.c_int
        L.am_workspace_bytes.argtypes = [i64, i32, am_basis, i32]
        L.am_workspace_bytes.restype = sz
        L.am_workspace_layout.argtypes = [i64, i32, am_basis, i32, P(sz)]
        L.am_workspace_layout.restype = ctypes.c_int
        L.am_price_american_ex.argtypes = [P(am_params), i64, i32, am_basis, i32, ctypes.c_void_p,
                                           sz, ctypes.c_void_p, P(dbl)]
        L.am_price_american_ex.restype = ctypes.c_int
        L.am_init.argtypes = []
        L.am_init.restype = ctypes.c_int
        L.am_price_american_noalloc.argtypes = [P(am_params), i64, i32, am_basis, i32, ctypes.c_void_p,
                                                P(dbl)]
        L.am_price_american_noalloc.restype = ctypes.c_int
        L.am_price_american_rqmc.argtypes = [P(am_params), i64, i32, am_basis, i32, i32,
                                             P(ctypes.c_uint32), ctypes.c_void_p, sz,
                                             ctypes.c_void_p, P(dbl)]
        L.am_price_american_rqmc.restype = ctypes.c_int
        L.am_price_paper_estimator.argtypes = [P(am_params), i64, i32, i32, ctypes.c_void_p, sz,
                                               ctypes.c_void_p, P(dbl)]
        L.am_price_paper_estimator.restype = ctypes.c_int
        L.am_price_rqmc_batch.argtypes = L.am_price_american_rqmc.argtypes
        L.am_price_rqmc_batch.restype = ctypes.c_int
        L.am_rqmc_workspace_bytes.argtypes = [i64, i32, am_basis, i32, i32]
        L.am_rqmc_workspace_bytes.restype = sz
        L.am_batch_workspace_bytes.argtypes = [P(am_option), i32, am_basis, i32]
        L.am_batch_workspace_bytes.restype = sz
        L.am_price_batch.argtypes = [P(am_option), i32, am_basis, i32, ctypes.c_void_p, sz,
                                     ctypes.c_void_p, P(dbl)]
        L.am_price_batch.restype = ctypes.c_int
        L.am_server_create.argtypes = [P(am_server_config), P(ctypes.c_void_p)]
        L.am_server_create.restype = ctypes.c_int
        L.am_server_submit.argtypes = [ctypes.c_void_p, P(am_option), ctypes.c_uint64, dbl]
        L.am_server_submit.restype = ctypes.c_int
        L.am_server_poll.argtypes = [ctypes.c_void_p, P(am_result), i32, P(i32)]
        L.am_server_poll.restype = ctypes.c_int
        L.am_server_now.argtypes = []
        L.am_server_now.restype = dbl
        L.am_server_stats.argtypes = [ctypes.c_void_p, P(dbl)]
        L.am_server_stats.restype = ctypes.c_int
        L.am_server_destroy.argtypes = [ctypes.c_void_p]
        L.am_server_destroy.restype = ctypes.c_int
        L.am_batch_autotune.argtypes = [P(am_option), i32, am_basis, i32, ctypes.c_void_p, sz,
                                        ctypes.c_void_p, P(i32), P(dbl)]
        L.am_batch_autotune.restype = ctypes.c_int
        L.am_batch_graph_create.argtypes = [P(am_option), i32, am_basis, i32, ctypes.c_void_p, sz,
                                            P(ctypes.c_void_p)]
        L.am_batch_graph_create.restype = ctypes.c_int
        L.am_batch_graph_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.am_batch_graph_launch.restype = ctypes.c_int
        L.am_batch_graph_results.argtypes = [ctypes.c_void_p, P(dbl)]
        L.am_batch_graph_results.restype = ctypes.c_int
        L.am_batch_graph_destroy.argtypes = [ctypes.c_void_p]
        L.am_batch_graph_destroy.restype = ctypes.c_int
        L.am_debug_set_batch_ppt.argtypes = [i32]
        L.am_debug_set_batch_ppt.restype = None
        L.am_debug_set_sweep_wide.argtypes = [i32]
        L.am_debug_set_sweep_wide.restype = None
        L.am_debug_set_sweep_tile.argtypes = [i32, i32]
        L.am_debug_set_sweep_tile.restype = None
        L.am_last_error.argtypes = []
        L.am_last_error.restype = ctypes.c_char_p
        L.am_max_dates.argtypes = []
        L.am_max_dates.restype = ctypes.c_int
        L.am_max_paths.argtypes = [i32]
        L.am_max_paths.restype = i64
        L.am_debug_generate.argtypes = [i32, P(am_params), i64, i32, i32, ctypes.c_void_p]
        L.am_debug_generate.restype = ctypes.c_int
        L.am_debug_schedule.argtypes = [i32, P(i32), P(i32), P(i32), P(i32), P(dbl), P(dbl), P(dbl)]
        L.am_debug_schedule.restype = ctypes.c_int
        L.am_profile_enable.argtypes = [i32]
        L.am_profile_enable.restype = ctypes.c_int
        L.am_profile_read.argtypes = [P(dbl), P(i64)]
        L.am_profile_read.restype = ctypes.c_int
        L.am_debug_set_spin_limit.argtypes = [ctypes.c_uint32]
        L.am_debug_set_spin_limit.restype = None
        _lib = L
        # release the library's process-lifetime HIP objects before the
        # runtime (and any profiler attached to it) finalises
        atexit.register(_shutdown_at_exit)
    return _lib


def _shutdown_at_exit():
    if _lib is not None:
        _lib.am_shutdown()


def am_shutdown() -> None:
    """Release the library's process-lifetime device objects (it sets them up
    again on the next call)."""
    _check(lib().am_shutdown())


def am_storage_dtype(n_paths: int, dtype) -> int:
    """Storage type (AM_FP64 or AM_FP32_BULK) a pricing request gets."""
    return int(lib().am_storage_dtype(int(n_paths), _dtype(dtype)))


def _check(rc: int):
    if rc != AM_OK:
        raise AmError(rc, lib().am_last_error().decode())


# --------------------------------------------------------------------------
# C-ABI entry points, same names
# --------------------------------------------------------------------------
def am_price_american(params: am_params, n_paths: int, n_dates: int, basis: am_basis,
                      dtype) -> Tuple[float, float]:
    """Synchronous pricing with the library-owned workspace and stream."""
    price, se = ctypes.c_double(), ctypes.c_double()
    _check(lib().am_price_american(ctypes.byref(params), int(n_paths), int(n_dates), basis,
                                   _dtype(dtype), ctypes.byref(price), ctypes.byref(se)))
    return price.value, se.value


def am_workspace_bytes(n_paths: int, n_dates: int, basis: am_basis, dtype) -> int:
    return int(lib().am_workspace_bytes(int(n_paths), int(n_dates), basis, _dtype(dtype)))


@dataclass
class Layout:
    off_S: int
    off_PV: int
    off_rec: int
    off_result: int
    ld: int
    total: int


def am_workspace_layout(n_paths: int, n_dates: int, basis: am_basis, dtype) -> Layout:
    out = (ctypes.c_size_t * 6)()
    _check(lib().am_workspace_layout(int(n_paths), int(n_dates), basis, _dtype(dtype), out))
    return Layout(*[int(v) for v in out])


def am_price_american_ex(params: am_params, n_paths: int, n_dates: int, basis: am_basis, dtype,
                         workspace, stream=None, wait: bool = True) -> Optional[Tuple[float, float]]:
    """Asynchronous pricing on a torch CUDA(HIP) stream with a torch workspace.

    ``workspace``: a contiguous uint8 CUDA tensor of >= am_workspace_bytes.
    ``stream``: torch.cuda.Stream or None (current stream).  With wait=True
    returns (price, std_err); otherwise returns None and the result stays in
    the workspace result region."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(workspace.device)
    if workspace.dtype != torch.uint8 or not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 CUDA tensor")
    out = (ctypes.c_double * 2)() if wait else None
    _check(lib().am_price_american_ex(ctypes.byref(params), int(n_paths), int(n_dates), basis,
                                      _dtype(dtype), ctypes.c_void_p(workspace.data_ptr()),
                                      workspace.numel(), ctypes.c_void_p(stream.cuda_stream), out))
    if wait:
        return out[0], out[1]
    return None


def am_init() -> None:
    """Set up the current device (needed before am_price_american_noalloc)."""
    _check(lib().am_init())


def am_price_american_noalloc(params: am_params, n_paths: int, n_dates: int, basis: am_basis, dtype,
                              stream=None) -> Tuple[float, float]:
    """Allocation-free pricing in the library's fixed device workspace, on a
    torch stream (None: the current stream); returns (price, std_err)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    out = (ctypes.c_double * 2)()
    _check(lib().am_price_american_noalloc(ctypes.byref(params), int(n_paths), int(n_dates), basis,
                                           _dtype(dtype), ctypes.c_void_p(stream.cuda_stream), out))
    return out[0], out[1]


def am_price_american_rqmc(params: am_params, n_paths: int, n_dates: int, basis: am_basis, dtype,
                           shifts, workspace, stream=None, _entry="am_price_american_rqmc"):
    """Randomised QMC (digital shifts, uint32 [R][n_dates]), replicates one
    after another; returns (mean, error bar, replicate prices)."""
    import numpy as np
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(workspace.device)
    sh = np.ascontiguousarray(shifts, dtype=np.uint32)
    R = sh.shape[0]
    out = (ctypes.c_double * (R + 2))()
    _check(getattr(lib(), _entry)(ctypes.byref(params), int(n_paths), int(n_dates), basis,
                                  _dtype(dtype), R, sh.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                  ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                  ctypes.c_void_p(stream.cuda_stream), out))
    return out[0], out[1], np.array(out[2:R + 2])


def am_price_rqmc_batch(params: am_params, n_paths: int, n_dates: int, basis: am_basis, dtype,
                        shifts, workspace, stream=None):
    """The same replicates all at once (batch form); returns (mean, error bar,
    replicate prices)."""
    return am_price_american_rqmc(params, n_paths, n_dates, basis, dtype, shifts, workspace, stream,
                                  _entry="am_price_rqmc_batch")


def am_rqmc_workspace_bytes(n_paths: int, n_dates: int, basis: am_basis, dtype, n_rep: int) -> int:
    """Workspace of the all-replicates-at-once randomised QMC form (0: invalid)."""
    return int(lib().am_rqmc_workspace_bytes(int(n_paths), int(n_dates), basis, _dtype(dtype), int(n_rep)))


def am_price_paper_estimator(params: am_params, n_paths: int, n_points: int, dtype, workspace,
                             stream=None, wait: bool = True):
    """The paper's eqs. (10)-(11) estimator on the GPU (torch workspace/stream)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(workspace.device)
    out = (ctypes.c_double * 2)() if wait else None
    _check(lib().am_price_paper_estimator(ctypes.byref(params), int(n_paths), int(n_points),
                                          _dtype(dtype), ctypes.c_void_p(workspace.data_ptr()),
                                          workspace.numel(), ctypes.c_void_p(stream.cuda_stream), out))
    if wait:
        return out[0], out[1]
    return None


def make_options(specs) -> "ctypes.Array":
    """specs: iterable of dicts with S0, K, r, sigma, T, n_paths, n_dates
    (is_call, allow_exercise optional)."""
    specs = list(specs)
    arr = (am_option * len(specs))()
    for i, d in enumerate(specs):
        arr[i].params = make_params(d["S0"], d["K"], d["r"], d["sigma"], d["T"],
                                    d.get("is_call", False), d.get("allow_exercise", True))
        arr[i].n_paths = int(d["n_paths"])
        arr[i].n_dates = int(d["n_dates"])
        arr[i].reserved = 0
    return arr


def am_batch_workspace_bytes(opts, basis: am_basis, dtype) -> int:
    return int(lib().am_batch_workspace_bytes(opts, len(opts), basis, _dtype(dtype)))


def am_price_batch(opts, basis: am_basis, dtype, workspace, stream=None, wait: bool = True):
    """Price a batch (am_option array) in two launches; returns an [n][2]
    numpy array of (price, std_err) or None when wait=False."""
    import numpy as np
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(workspace.device)
    n = len(opts)
    out = (ctypes.c_double * (2 * n))() if wait else None
    _check(lib().am_price_batch(opts, n, basis, _dtype(dtype), ctypes.c_void_p(workspace.data_ptr()),
                                workspace.numel(), ctypes.c_void_p(stream.cuda_stream), out))
    if wait:
        return np.frombuffer(out, dtype=np.float64).reshape(n, 2).copy()
    return None


def am_batch_autotune(opts, basis: am_basis, dtype, workspace, stream=None):
    """Returns (best paths-per-thread, [ms per candidate])."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(workspace.device)
    best = ctypes.c_int32()
    ms = (ctypes.c_double * 2)()
    _check(lib().am_batch_autotune(opts, len(opts), basis, _dtype(dtype),
                                   ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                   ctypes.c_void_p(stream.cuda_stream), ctypes.byref(best), ms))
    return best.value, [ms[0], ms[1]]


class BatchGraph:
    """A batch captured as a HIP graph; launch() replays it, results() waits."""

    def __init__(self, opts, basis: am_basis, dtype, workspace):
        self._opts = opts
        self._ws = workspace
        self._h = ctypes.c_void_p()
        _check(lib().am_batch_graph_create(opts, len(opts), basis, _dtype(dtype),
                                           ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                           ctypes.byref(self._h)))

    def launch(self, stream) -> None:
        _check(lib().am_batch_graph_launch(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def results(self):
        import numpy as np
        n = len(self._opts)
        out = (ctypes.c_double * (2 * n))()
        _check(lib().am_batch_graph_results(self._h, out))
        return np.frombuffer(out, dtype=np.float64).reshape(n, 2).copy()

    def close(self) -> None:
        if self._h:
            lib().am_batch_graph_destroy(self._h)
            self._h = ctypes.c_void_p()


class Server:
    """Continuous-batching pricing server (am_server_* through the C-ABI)."""

    def __init__(self, hbm_budget_bytes: int, basis: am_basis, dtype, *, n_streams: int = 2,
                 max_batch_requests: int = 64, max_batch_path_steps: float = 2e9, large_tile: bool = False):
        cfg = am_server_config(int(hbm_budget_bytes), float(max_batch_path_steps),
                               int(max_batch_requests), int(n_streams), basis, _dtype(dtype), int(large_tile))
        self._h = ctypes.c_void_p()
        _check(lib().am_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._buf = (am_result * 1024)()

    @staticmethod
    def now() -> float:
        return float(lib().am_server_now())

    def submit(self, opt: "am_option", request_id: int, t_arrival: float = -1.0) -> None:
        _check(lib().am_server_submit(self._h, ctypes.byref(opt), int(request_id), float(t_arrival)))

    def poll(self):
        n = ctypes.c_int32()
        _check(lib().am_server_poll(self._h, self._buf, len(self._buf), ctypes.byref(n)))
        return [dict(id=r.request_id, price=r.price, std_err=r.std_err, t_arrival=r.t_arrival,
                     t_launch=r.t_launch, t_done=r.t_done, status=r.status)
                for r in self._buf[:n.value]]

    def stats(self):
        out = (ctypes.c_double * 4)()
        _check(lib().am_server_stats(self._h, out))
        return dict(batches=out[0], requests=out[1], path_steps=out[2], pool_bytes_used=out[3])

    def close(self) -> None:
        if self._h:
            rc = lib().am_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            _check(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False


def am_debug_set_batch_ppt(ppt: int) -> None:
    lib().am_debug_set_batch_ppt(int(ppt))


def am_debug_set_sweep_wide(allow: bool) -> None:
    lib().am_debug_set_sweep_wide(1 if allow else 0)


def am_debug_set_sweep_tile(wg: int, ppt: int) -> None:
    """Force the single-option sweep tile on this thread (wg=0: automatic)."""
    lib().am_debug_set_sweep_tile(int(wg), int(ppt))


def am_last_error() -> str:
    return lib().am_last_error().decode()


def am_max_dates() -> int:
    return int(lib().am_max_dates())


def am_max_paths(dtype) -> int:
    return int(lib().am_max_paths(_dtype(dtype)))


def am_debug_generate(what: int, params: Optional[am_params], n_paths: int, n_dims: int, dtype):
    """Diagnostic generation: what=1 Sobol ints [dims][paths] (uint32),
    what=2 normals, what=0 paths (float64 [dims][paths])."""
    import numpy as np
    dt = np.uint32 if what == 1 else np.float64
    out = np.zeros((n_dims, n_paths), dtype=dt)
    _check(lib().am_debug_generate(int(what), ctypes.byref(params) if params is not None else None,
                                   int(n_paths), int(n_dims), _dtype(dtype),
                                   out.ctypes.data_as(ctypes.c_void_p)))
    return out


def am_debug_schedule(n_dates: int):
    import numpy as np
    m = np.zeros(n_dates, np.int32)
    dim = np.zeros(n_dates, np.int32)
    left = np.zeros(n_dates, np.int32)
    right = np.zeros(n_dates, np.int32)
    wl = np.zeros(n_dates)
    wr = np.zeros(n_dates)
    sd = np.zeros(n_dates)
    P = ctypes.POINTER
    _check(lib().am_debug_schedule(int(n_dates), *[a.ctypes.data_as(P(ctypes.c_int32)) for a in (m, dim, left, right)],
                                   *[a.ctypes.data_as(P(ctypes.c_double)) for a in (wl, wr, sd)]))
    return dict(m=m, dim=dim, left=left, right=right, wl=wl, wr=wr, sd=sd)


def am_profile_enable(on: bool) -> None:
    _check(lib().am_profile_enable(int(bool(on))))


def am_profile_read():
    """Returns (gen_ms_total, sweep_ms_total, calls) since the last read."""
    ms = (ctypes.c_double * 2)()
    n = ctypes.c_int64()
    _check(lib().am_profile_read(ms, ctypes.byref(n)))
    return ms[0], ms[1], n.value


def am_debug_set_spin_limit(spins: int) -> None:
    lib().am_debug_set_spin_limit(int(spins))


# --------------------------------------------------------------------------
# Convenience: price with a torch-owned workspace (cached per size)
# --------------------------------------------------------------------------
class Pricer:
    """Holds a torch workspace and stream; prices options through the C-ABI."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = torch.device("cuda", device)
        self.stream = stream or torch.cuda.Stream(self.device)
        self.ws = None

    def workspace(self, nbytes: int):
        import torch
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = None
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.ws

    def price(self, params: am_params, n_paths: int, n_dates: int, basis: am_basis, dtype,
              wait: bool = True):
        nbytes = am_workspace_bytes(n_paths, n_dates, basis, dtype)
        ws = self.workspace(nbytes)
        return am_price_american_ex(params, n_paths, n_dates, basis, dtype, ws, self.stream, wait)

    def price_rqmc(self, params: am_params, n_paths: int, n_dates: int, basis: am_basis, dtype, shifts,
                   fused: bool = True):
        """fused: every replicate at once (batch form); else one after another."""
        if fused:
            nbytes = am_rqmc_workspace_bytes(n_paths, n_dates, basis, dtype, len(shifts))
            if nbytes == 0:
                raise AmError(AM_EINVAL, am_last_error())
            return am_price_rqmc_batch(params, n_paths, n_dates, basis, dtype, shifts, self.workspace(nbytes),
                                       self.stream)
        nbytes = am_workspace_bytes(n_paths, n_dates, basis, dtype)
        return am_price_american_rqmc(params, n_paths, n_dates, basis, dtype, shifts, self.workspace(nbytes),
                                      self.stream)

    def price_batch(self, opts, basis: am_basis, dtype, wait: bool = True):
        nbytes = am_batch_workspace_bytes(opts, basis, dtype)
        if nbytes == 0:
            raise AmError(AM_EINVAL, am_last_error())
        ws = self.workspace(nbytes)
        return am_price_batch(opts, basis, dtype, ws, self.stream, wait)

    def price_paper(self, params: am_params, n_paths: int, n_points: int, dtype, wait: bool = True):
        nbytes = am_workspace_bytes(n_paths, n_points, make_basis("monomial", 0), dtype)
        ws = self.workspace(nbytes)
        return am_price_paper_estimator(params, n_paths, n_points, dtype, ws, self.stream, wait)

    def views(self, n_paths: int, n_dates: int, basis: am_basis, dtype):
        """Torch views of the last call's paths, PV, per-date records, result."""
        import torch
        lay = am_workspace_layout(n_paths, n_dates, basis, dtype)
        ws = self.ws
        el = torch.float64 if am_storage_dtype(n_paths, dtype) == AM_FP64 else torch.float32
        sz = 8 if el == torch.float64 else 4
        S = ws[lay.off_S: lay.off_S + n_dates * lay.ld * sz].view(el).view(n_dates, lay.ld)
        PV = ws[lay.off_PV: lay.off_PV + lay.ld * sz].view(el)
        rec = ws[lay.off_rec: lay.off_rec + (n_dates + 1) * REC * 8].view(torch.float64).view(n_dates + 1, REC)
        res = ws[lay.off_result: lay.off_result + 64].view(torch.float64)
        return dict(S=S[:, :n_paths], PV=PV[:n_paths], rec=rec, result=res, layout=lay)


def price_american(S0, K, r, sigma, T, n_paths, n_dates, *, is_call=False, allow_exercise=True,
                   basis=("monomial", 2), dtype="fp64") -> Tuple[float, float]:
    """price_american(params, n_paths, n_dates, basis, dtype) -> (price, stderr)."""
    p = make_params(S0, K, r, sigma, T, is_call, allow_exercise)
    b = make_basis(*basis) if isinstance(basis, tuple) else basis
    return am_price_american(p, n_paths, n_dates, b, dtype)
