"""Write oracle results for the full-size configurations (calls only oracle/).

    python tests/golden/make_oracle_goldens.py [2] [4]

Config 4 (2^24 paths x 252 dates) needs about 34 GB of host memory and runs
single-threaded for several minutes.  Output: tests/golden/oracle_config<N>.json
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1205_0106_amd.workloads import CONFIGS  # noqa: E402


def run(cid):
    w = CONFIGS[cid]
    kind = oracle.LAGUERRE if w.basis[0] == "laguerre" else oracle.MONOMIAL
    t = time.time()
    res, d = oracle.price_american(**w.params(), N=w.n_paths, M=w.n_dates, is_call=w.is_call,
                                   allow_exercise=w.allow_exercise, kind=kind, degree=w.basis[1],
                                   detail=True)
    out = dict(config=cid, workload=w.name, n_paths=w.n_paths, n_dates=w.n_dates,
               basis=list(w.basis), price=res.price, std_err=res.std_err, mean_pv=res.mean_pv,
               t0_exercise=res.t0_exercise, n_skipped=res.n_skipped,
               n_itm=[int(v) for v in d["nitm"]], seconds=time.time() - t,
               generator="tests/golden/make_oracle_goldens.py (oracle only)")
    with open(os.path.join(HERE, f"oracle_config{cid}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(cid, res.price, out["seconds"], flush=True)


if __name__ == "__main__":
    for a in sys.argv[1:] or ["2"]:
        run(int(a))
