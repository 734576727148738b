"""Seeded synthetic workloads (the configurations the engine is measured on).

Holds parameters and seeded generators only — none of the pricing method's
arithmetic — so both the GPU tests/benchmark and the CPU oracle can take
their inputs from here.  The paper publishes no option parameters or data
sets (its experiments state only path counts and ten exercise points), so
every workload is synthetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    S0: float
    K: float
    r: float
    sigma: float
    T: float
    n_dates: int
    n_paths: int
    basis: tuple            # (kind, degree)
    dtypes: tuple           # precisions the configuration is run in
    is_call: bool = False
    allow_exercise: bool = True

    def params(self):
        return dict(S0=self.S0, K=self.K, r=self.r, sigma=self.sigma, T=self.T)


CONFIG1 = Workload("config1_put_S36_K40_M50_N2^14_mono2_fp64", 36.0, 40.0, 0.06, 0.2, 1.0,
                   50, 1 << 14, ("monomial", 2), ("fp64",))
CONFIG2 = Workload("config2_put_S100_K100_M100_N2^20_laguerre3", 100.0, 100.0, 0.05, 0.3, 1.0,
                   100, 1 << 20, ("laguerre", 3), ("fp64", "fp32"))
CONFIG4 = Workload("config4_put_S100_K110_M252_N2^24_mono4_fp32", 100.0, 110.0, 0.03, 0.25, 2.0,
                   252, 1 << 24, ("monomial", 4), ("fp32",))
CONFIGS = {1: CONFIG1, 2: CONFIG2, 4: CONFIG4}

# The paper's Table 2 shape: American option, ten exercise points, path
# counts 10 .. 10^6 (its option parameters are unstated; config 1's are used).
PAPER_TABLE2_PATHS = (10, 100, 1000, 10000, 100000, 200000, 300000, 500000, 1000000)


def batch_options(n: int = 1024, seed: int = 0x12050106, log2_paths=(14.0, 18.0),
                  dates=(16, 256)):
    """Seeded batch of options: put/call 50/50, K ~ U(80,120), S0 = 100,
    sigma ~ U(0.1,0.5), r ~ U(0,0.08), T ~ U(0.25,2), dates ~ U{lo..hi},
    paths = round(2^U(a,b)) (log-uniform, mostly not powers of two)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        out.append(dict(
            is_call=bool(rng.integers(0, 2)),
            K=float(rng.uniform(80.0, 120.0)),
            S0=100.0,
            sigma=float(rng.uniform(0.1, 0.5)),
            r=float(rng.uniform(0.0, 0.08)),
            T=float(rng.uniform(0.25, 2.0)),
            n_dates=int(rng.integers(dates[0], dates[1] + 1)),
            n_paths=int(round(2.0 ** rng.uniform(*log2_paths))),
        ))
    return out


def poisson_arrivals(rate: float = 200.0, duration: float = 60.0, seed: int = 0x12050107):
    """Arrival times (s) of a Poisson stream, exponential gaps."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            return out
        out.append(t)
