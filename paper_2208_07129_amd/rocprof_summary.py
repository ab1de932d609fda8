"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_2208_07129_amd.rocprof_summary stats <run_kernel_stats.csv> [--cmd "..."]
        -> markdown table of per-kernel call counts and durations
    python -m paper_2208_07129_amd.rocprof_summary traffic --fetch DIR --write DIR
            --cal-fetch DIR --cal-write DIR --cal-bytes N --key KEY --kernel-hash H
            [--out profiles/apply_f64_traffic.json]
        -> HBM bytes per launch of the fused apply kernel from FETCH_SIZE / WRITE_SIZE
           runs, each scaled by what the same counter reads for a plain elementwise
           kernel of known size (bytes per KiB of counter)

Each DIR holds the run_counter_collection.csv of one `rocprofv3 --pmc` run.
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import sys
from collections import defaultdict


def per_kernel(csv_path: str, counter: str) -> dict:
    vals = defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] == counter:
            vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in vals.items()}


def pick(d: dict, needle: str) -> float:
    hits = [v for k, v in d.items() if needle in k]
    if not hits:
        raise SystemExit(f"no kernel matching {needle!r} in {list(d)}")
    return hits[0]


def cmd_stats(a):
    rows = list(csv.DictReader(open(a.csv)))
    out = ["| kernel | calls | avg us | min us | max us | % |", "|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"]
        short = name.replace("mf::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        out.append(f"| `{short}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    text = "\n".join(out)
    if a.cmd:
        text = f"Command: `{a.cmd}`\n\n" + text
    print(text)


def cmd_traffic(a):
    f = per_kernel(os.path.join(a.fetch, "run_counter_collection.csv"), "FETCH_SIZE")
    w = per_kernel(os.path.join(a.write, "run_counter_collection.csv"), "WRITE_SIZE")
    cf = per_kernel(os.path.join(a.cal_fetch, "run_counter_collection.csv"), "FETCH_SIZE")
    cw = per_kernel(os.path.join(a.cal_write, "run_counter_collection.csv"), "WRITE_SIZE")
    kf, kw = pick(f, a.kernel), pick(w, a.kernel)
    cal_f, cal_w = max(cf.values()), max(cw.values())
    fetch_bytes = kf * a.cal_bytes / cal_f
    write_bytes = kw * a.cal_bytes / cal_w
    rec = {"bytes_per_launch": fetch_bytes + write_bytes, "fetch_bytes": fetch_bytes,
           "write_bytes": write_bytes, "fetch_counter_kib": kf, "write_counter_kib": kw,
           "calibration": {"bytes": a.cal_bytes, "fetch_counter_kib": cal_f, "write_counter_kib": cal_w},
           "kernel_hash": a.kernel_hash}
    db = {}
    if os.path.exists(a.out):
        db = json.load(open(a.out))
    db[a.key] = rec
    json.dump(db, open(a.out, "w"), indent=1, sort_keys=True)
    print(json.dumps(rec))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", default="")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "cal_fetch", "cal_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--cal-bytes", type=float, required=True)
    t.add_argument("--key", required=True)
    t.add_argument("--kernel", default="apply_box_kernel")
    t.add_argument("--kernel-hash", required=True)
    t.add_argument("--out", default=os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                                 "profiles", "apply_f64_traffic.json"))
    a = ap.parse_args(argv)
    (cmd_stats if a.cmd_name == "stats" else cmd_traffic)(a)


if __name__ == "__main__":
    sys.exit(main())
