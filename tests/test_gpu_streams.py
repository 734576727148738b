"""Single-option pricings enqueued on two streams at once.  Each persistent
sweep holds the whole device and waits only on its own groups, so the library
orders sweeps of different streams on one device; the interleaved results
must be bitwise those of the same calls run one at a time."""
import sys

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
    amq.lib()
    return amq


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_two_streams_interleaved(amq, dtype):
    import torch
    N, M = (1 << 18) + 77, 40
    b = amq.make_basis("laguerre", 3)
    opts = [amq.make_params(100.0, 100.0, 0.05, 0.3, 1.0), amq.make_params(95.0, 110.0, 0.03, 0.25, 2.0)]
    pricers = [amq.Pricer(0), amq.Pricer(0)]
    alone = [pr.price(p, N, M, b, dtype) for pr, p in zip(pricers, opts)]
    log(f"two streams {dtype}: alone {alone}")
    for rnd in range(4):
        for pr, p in zip(pricers, opts):
            pr.price(p, N, M, b, dtype, wait=False)
        torch.cuda.synchronize()
        for q, (pr, want) in enumerate(zip(pricers, alone)):
            res = pr.views(N, M, b, dtype)["result"].cpu().numpy()
            log(f"  round {rnd} stream {q}: price {res[0]!r} error flag {res[5]}")
            assert res[5] == 0.0
            assert (float(res[0]), float(res[1])) == want
