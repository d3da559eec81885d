"""Profiling helpers: a device copy of known size for counter calibration,
and a reader that turns rocprofv3 CSV output into short text summaries.

`python -m paper_2509_18544_amd.profiling copy --mib 1024` runs a plain
device-to-device copy of the given size a few times; the HBM byte counters
(FETCH_SIZE, WRITE_SIZE) read for that copy give the scale factor between
counter units and real bytes on the machine at hand.

`python -m paper_2509_18544_amd.profiling stats <kernel_stats.csv>` prints
the per-kernel summary (calls, average and total device time).
`python -m paper_2509_18544_amd.profiling pmc <counter_collection.csv> <regex>`
prints the per-dispatch average of each collected counter for the kernels
whose name matches the regex.
"""
from __future__ import annotations

import argparse
import csv
import re
import sys


def copy_probe(mib: int, reps: int = 5) -> None:
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x {reps}")


def stats(path: str, top: int = 30) -> None:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print(f"{'kernel':80s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}")
    for r in rows[:top]:
        print(f"{r['Name'][:80]:80s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.1f} "
              f"{float(r['TotalDurationNs']) / 1e6:10.2f} {float(r['Percentage']):6.2f}")


def pmc(path: str, regex: str) -> None:
    rows = list(csv.DictReader(open(path)))
    pat = re.compile(regex)
    acc = {}
    for r in rows:
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or r.get("KernelName") or ""
        if not pat.search(name):
            continue
        key = (name[:80], r.get("Counter_Name") or r.get("Counter-Name") or r.get("CounterName"))
        val = float(r.get("Counter_Value") or r.get("Counter-Value") or r.get("CounterValue") or 0.0)
        disp = r.get("Dispatch_Id") or r.get("Dispatch-Id") or r.get("DispatchId")
        d = acc.setdefault(key, {})
        d[disp] = d.get(disp, 0.0) + val
    for (name, counter), per in sorted(acc.items()):
        vals = list(per.values())
        print(f"{name:80s} {counter:14s} dispatches={len(vals):4d} avg_per_dispatch={sum(vals) / len(vals):.4g}")


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    c.add_argument("--reps", type=int, default=5)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=30)
    p = sub.add_parser("pmc")
    p.add_argument("csv")
    p.add_argument("regex")
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        copy_probe(a.mib, a.reps)
    elif a.cmd == "stats":
        stats(a.csv, a.top)
    else:
        pmc(a.csv, a.regex)


if __name__ == "__main__":
    main(sys.argv[1:])
