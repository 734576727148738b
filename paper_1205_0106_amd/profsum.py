"""Summaries of rocprofv3 output for the pricing kernels.

    python -m paper_1205_0106_amd.profsum trace DIR [--skip N]
    python -m paper_1205_0106_amd.profsum counters DIR
    python -m paper_1205_0106_amd.profsum traffic --fetch DIR --write DIR
        --copy-fetch DIR --copy-write DIR --copy-bytes B --config C --path-steps P --out FILE
    python -m paper_1205_0106_amd.profsum valu --dir DIR --config C --path-steps P
        --trace DIR --out FILE

DIR is a rocprofv3 output directory (`-d DIR -o run --output-format csv`, or
the default CSV output of --kernel-trace / --pmc).  `trace` prints the
per-kernel launch table (calls, average duration, average after the first N
calls of each kernel); `counters` the per-kernel average of every counter.
`traffic` and `valu` write the JSON files bench.py reads (profiles/traffic.json,
profiles/valu.json): HBM bytes per launch from FETCH_SIZE / WRITE_SIZE (KiB
per dispatch), each scaled so that a plain device copy of known size reads
as its size, and SQ_INSTS_VALU / SQ_INSTS_SALU per launch; both keyed by the
kernel sources' hash, so figures taken on other sources are not reported.
Only the standard library is used; nothing here touches the GPU.
"""
import argparse
import csv
import glob
import json
import os
import sys
from collections import defaultdict

KERNELS = {"sweep_kernel": "amq::sweep_kernel", "gen_kernel": "amq::gen_kernel"}


def _rows(d, suffix):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    out = []
    for f in files:
        with open(f, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


def trace(d, skip=0, by_grid=False, first=0):
    """{kernel name: (calls, avg_us_all, avg_us_after_skip)} from a kernel
    trace; by_grid: one entry per (name, grid size), named "name [grid G]";
    first: only each kernel's first `first` launches (in time order)."""
    per = defaultdict(list)
    for r in _rows(d, "kernel_trace.csv"):
        k = r["Kernel_Name"]
        if by_grid:
            k = f"{k} [grid {r.get('Grid_Size_X', r.get('Grid_Size', '?'))}]"
        per[k].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    out = {}
    for k, v in per.items():
        v.sort()
        if first:
            v = v[:first]
        dur = [(e - s) / 1e3 for s, e in v]
        tail = dur[skip:] if len(dur) > skip else dur
        out[k] = (len(dur), sum(dur) / len(dur), sum(tail) / len(tail))
    return out


def counters(d):
    """{kernel name: {counter: average per dispatch}} from a --pmc run."""
    acc = defaultdict(lambda: defaultdict(list))
    for r in _rows(d, "counter_collection.csv"):
        acc[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in m.items()} for k, m in acc.items()}


def _pick(table, key):
    """The entry of `table` whose kernel name contains KERNELS[key]."""
    hits = [(k, v) for k, v in table.items() if KERNELS[key] in k]
    if not hits:
        return None, None
    # several instantiations: the one with the most work
    return max(hits, key=lambda kv: sum(kv[1].values()) if isinstance(kv[1], dict) else kv[1][0])


def source_hash():
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    return bench.kernel_source_hash()


def _load(path):
    if os.path.exists(path):
        return json.load(open(path))
    return {}


def write_traffic(a):
    fetch, write = counters(a.fetch), counters(a.write)
    cf, cw = counters(a.copy_fetch), counters(a.copy_write)
    copy_name = [k for k in cf if "copyBuffer" in k or "copy" in k.lower()]
    if not copy_name:
        raise SystemExit("no copy kernel in the calibration runs")
    kb_f = cf[copy_name[0]]["FETCH_SIZE"] * 1024.0
    kb_w = cw[[k for k in cw if k in copy_name or "copy" in k.lower()][0]]["WRITE_SIZE"] * 1024.0
    fetch_scale, write_scale = a.copy_bytes / kb_f, a.copy_bytes / kb_w
    h = source_hash()
    out = _load(a.out)
    if out.get("source_hash") != h:
        out = {"kernels": {}}
    out.update(source_hash=h, fetch_scale=fetch_scale, write_scale=write_scale)
    for key in KERNELS:
        name, fc = _pick(fetch, key)
        _, wc = _pick(write, key)
        if name is None:
            continue
        rd = fc["FETCH_SIZE"] * 1024.0 * fetch_scale
        wr = wc["WRITE_SIZE"] * 1024.0 * write_scale
        out["kernels"][f"cfg{a.config}:{key}"] = {
            "kernel": name, "read_bytes": rd, "write_bytes": wr, "traffic_bytes": rd + wr,
            "algorithmic_bytes": a.path_steps * a.elem_bytes}
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def write_valu(a):
    cnt = counters(a.dir)
    tr = trace(a.trace, skip=a.skip) if a.trace else {}
    h = source_hash()
    out = _load(a.out)
    if out.get("source_hash") != h:
        out = {"kernels": {}}
    out.update(source_hash=h, peak_lane_instr_per_s=256 * 4 * 16 * 2.4e9)
    for key in KERNELS:
        name, c = _pick(cnt, key)
        if name is None:
            continue
        ent = {"kernel": name, "valu_wave_instr": c.get("SQ_INSTS_VALU"),
               "salu_wave_instr": c.get("SQ_INSTS_SALU"), "path_steps": a.path_steps,
               "valu_lane_instr_per_path_step": c.get("SQ_INSTS_VALU", 0.0) * 64 / a.path_steps}
        if name in tr:
            us = tr[name][2]
            ent["trace_avg_us"] = us
            ent["issue_fraction"] = c.get("SQ_INSTS_VALU", 0.0) * 64 / (us * 1e-6) / out["peak_lane_instr_per_s"]
        out["kernels"][f"cfg{a.config}:{key}"] = ent
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--skip", type=int, default=0)
    t.add_argument("--by-grid", action="store_true")
    t.add_argument("--first", type=int, default=0)
    c = sub.add_parser("counters")
    c.add_argument("dir")
    f = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "out"):
        f.add_argument("--" + k.replace("_", "-"), required=True)
    f.add_argument("--copy-bytes", type=float, required=True)
    f.add_argument("--config", type=int, required=True)
    f.add_argument("--path-steps", type=int, required=True)
    f.add_argument("--elem-bytes", type=int, default=4)
    v = sub.add_parser("valu")
    v.add_argument("--dir", required=True)
    v.add_argument("--trace", default=None)
    v.add_argument("--skip", type=int, default=1)
    v.add_argument("--config", type=int, required=True)
    v.add_argument("--path-steps", type=int, required=True)
    v.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        rows = trace(a.dir, a.skip, a.by_grid, a.first)
        tot = sum(n * avg for n, avg, _ in rows.values())
        print("| kernel | calls | average, all calls (us) | share | average after the first "
              f"{a.skip} calls (us) |\n|---|---|---|---|---|")
        for k, (n, avg, tail) in sorted(rows.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
            print(f"| `{k}` | {n} | {avg:.1f} | {100 * n * avg / tot:.1f} % | {tail:.1f} |")
    elif a.cmd == "counters":
        for k, m in counters(a.dir).items():
            print(k[:100])
            for cn, val in sorted(m.items()):
                print(f"    {cn} = {val:.6g}")
    elif a.cmd == "traffic":
        write_traffic(a)
    else:
        write_valu(a)


if __name__ == "__main__":
    main()
