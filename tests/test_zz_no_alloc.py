"""GPU: the allocation-free entry point against am_price_american_ex.

am_price_american_noalloc runs the same kernels and tiles as
am_price_american_ex, in the library's fixed device array instead of a
caller workspace, so price and standard error must agree bit for bit.  Two
calls in a row, the second on a smaller input, check that nothing left in
the shared array from the first call leaks into the second; the device's
free memory must not shrink by anything near a workspace while they run.
"""
import sys

import numpy as np
import pytest

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
    torch.cuda.set_device(0)
    amq.lib()
    amq.am_init()
    return amq


# (params, n_paths, n_dates, basis, dtype): a large then a smaller shape per
# precision, ragged path counts, both basis kinds, a call and a put
CASES = [
    (dict(S0=100.0, K=100.0, r=0.05, sigma=0.3, T=1.0, is_call=False), 131072 - 77, 100, ("laguerre", 3), "fp64"),
    (dict(S0=36.0, K=40.0, r=0.06, sigma=0.2, T=1.0, is_call=False), 5001, 17, ("monomial", 2), "fp64"),
    (dict(S0=100.0, K=110.0, r=0.03, sigma=0.25, T=2.0, is_call=False), 262144 - 1000, 120, ("monomial", 4), "fp32"),
    (dict(S0=100.0, K=90.0, r=0.04, sigma=0.35, T=0.5, is_call=True), 20000, 33, ("monomial", 3), "fp32"),
]


def _ex(amq, torch, kw, N, M, basis, dtype, stream=None):
    p = amq.make_params(**kw)
    b = amq.make_basis(*basis)
    ws = torch.empty(amq.am_workspace_bytes(N, M, b, dtype), dtype=torch.uint8, device="cuda")
    return amq.am_price_american_ex(p, N, M, b, dtype, ws, stream), ws


def test_noalloc_equals_ex_two_calls_second_smaller(amq):
    import torch
    stream = torch.cuda.Stream()
    # reference results first, on the same stream: the runtime sets up what
    # a stream's hardware queue needs (its private-memory pool, copy staging)
    # at the first kernels and copies that use them, before the measurement
    refs, keep = [], []
    for kw, N, M, basis, dtype in CASES:
        log(f"noalloc ref: ex N={N} M={M} {basis} {dtype}")
        r, ws = _ex(amq, torch, kw, N, M, basis, dtype, stream)
        refs.append(r)
        keep.append(ws)
        assert amq.am_workspace_bytes(N, M, amq.make_basis(*basis), dtype) + 64 * M <= amq.AM_SCRATCH_BYTES
    with torch.cuda.stream(stream):
        t = torch.ones(1 << 20, device="cuda")
        h = t.cpu()
        t.copy_(h)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    biggest = max(amq.am_workspace_bytes(N, M, amq.make_basis(*b), d) for _, N, M, b, d in CASES)
    for rnd in range(2):
        for (kw, N, M, basis, dtype), want in zip(CASES, refs):
            log(f"noalloc round {rnd}: N={N} M={M} {basis} {dtype}")
            got = amq.am_price_american_noalloc(amq.make_params(**kw), N, M, amq.make_basis(*basis),
                                                dtype, stream)
            log(f"  got {got!r} want {want!r} free {torch.cuda.mem_get_info()[0]}")
            assert got == want, (got, want)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    log(f"free memory {free0} -> {free1} (largest workspace {biggest})")
    assert free0 - free1 <= 4 << 20, (free0, free1)


def test_noalloc_on_current_stream_and_after_oversize(amq):
    import torch
    kw = dict(S0=36.0, K=40.0, r=0.06, sigma=0.2, T=1.0)
    b = amq.make_basis("monomial", 2)
    want, _ = _ex(amq, torch, kw, 16384, 50, ("monomial", 2), "fp64")
    # too large for the fixed array: a clear error, nothing launched
    with pytest.raises(amq.AmError) as ei:
        amq.am_price_american_noalloc(amq.make_params(**kw), 1 << 20, 200, b, "fp64")
    assert ei.value.code == amq.AM_EWORKSPACE
    assert "allocation-free" in str(ei.value)
    got = amq.am_price_american_noalloc(amq.make_params(**kw), 16384, 50, b, "fp64")
    assert got == want


def test_noalloc_matches_oracle_small(amq, orc):
    kw = dict(S0=36.0, K=40.0, r=0.06, sigma=0.2, T=1.0)
    N, M = 16384, 50
    got = amq.am_price_american_noalloc(amq.make_params(**kw), N, M, amq.make_basis("monomial", 2), "fp64")
    want = orc.price_american(**kw, N=N, M=M, kind=orc.MONOMIAL, degree=2)
    log(f"noalloc vs oracle: {got[0]!r} {want.price!r}")
    assert abs(got[0] - want.price) <= 1e-4
    assert np.isfinite(got[1])
