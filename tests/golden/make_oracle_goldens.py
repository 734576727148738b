"""Write oracle results for the full-size configurations (calls only oracle/).

    python tests/golden/make_oracle_goldens.py [--force | --redo-store32] [2] [4]

Each file holds the all-binary64 result (top level) and, for configurations
priced in FP32 bulk, the result on binary32-stored paths under "store32" (the
oracle's binary32-storage mode: path values and cashflows rounded to
binary32, binary64 arithmetic).  Results already in the file for the same
workload are kept unless --force (all) or --redo-store32 (that one) is given.
Config 4 (2^24 paths x 252 dates) needs about 34 GB of host memory and runs
single-threaded for about twelve minutes per result.
Output: tests/golden/oracle_config<N>.json
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1205_0106_amd.workloads import CONFIGS  # noqa: E402


def one(w, store32):
    kind = oracle.LAGUERRE if w.basis[0] == "laguerre" else oracle.MONOMIAL
    t = time.time()
    res, d = oracle.price_american(**w.params(), N=w.n_paths, M=w.n_dates, is_call=w.is_call,
                                   allow_exercise=w.allow_exercise, kind=kind, degree=w.basis[1],
                                   detail=True, store32=store32)
    return dict(price=res.price, std_err=res.std_err, mean_pv=res.mean_pv,
                t0_exercise=res.t0_exercise, n_skipped=res.n_skipped,
                n_itm=[int(v) for v in d["nitm"]], seconds=time.time() - t)


def run(cid, force=False, redo32=False):
    w = CONFIGS[cid]
    path = os.path.join(HERE, f"oracle_config{cid}.json")
    out = {}
    if os.path.exists(path) and not force:
        old = json.load(open(path))
        if old.get("workload") == w.name:
            out = old
            if redo32:
                out.pop("store32", None)
    if "price" not in out:
        out = dict(config=cid, workload=w.name, n_paths=w.n_paths, n_dates=w.n_dates,
                   basis=list(w.basis), **one(w, False))
        print(cid, "binary64", out["price"], out["seconds"], flush=True)
    if "fp32" in w.dtypes and "store32" not in out:
        out["store32"] = one(w, True)
        print(cid, "binary32 storage", out["store32"]["price"], out["store32"]["seconds"], flush=True)
    out["generator"] = "tests/golden/make_oracle_goldens.py (oracle only)"
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    args = sys.argv[1:]
    force, redo32 = "--force" in args, "--redo-store32" in args
    for a in [a for a in args if not a.startswith("--")] or ["2"]:
        run(int(a), force, redo32)
