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
`... trace <kernel_trace.csv> <regex> --last K` averages the last K dispatches
(the timed region); `... traffic <fetch.csv> <write.csv> <copy_fetch.csv>
<copy_write.csv> <regex>` turns the byte counters into calibrated HBM bytes.
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


def trace_avg(path: str, regex: str, last: int, min_us: float = 0.0) -> None:
    """Average device time of the dispatches of the kernels matching regex: the
    last `last` of them (the timed region of a run whose earlier dispatches were
    warm-up or tuning), and those lasting at least `min_us` (the batch launches
    of a run that also makes single-pair launches)."""
    rows = [r for r in csv.DictReader(open(path)) if re.search(regex, r["Kernel_Name"])]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows]
    tail = d[-last:] if last > 0 else d
    print(f"{regex}: {len(d)} dispatches, all avg {sum(d) / max(1, len(d)):.1f} us; "
          f"last {len(tail)} avg {sum(tail) / max(1, len(tail)):.1f} us")
    if min_us > 0:
        big = [x for x in d if x >= min_us]
        print(f"{regex}: {len(big)} dispatches of at least {min_us:.0f} us, avg {sum(big) / max(1, len(big)):.1f} us")


def traffic(fetch_csv: str, write_csv: str, copy_fetch_csv: str, copy_write_csv: str, regex: str,
            copy_mib: int = 1024) -> None:
    """HBM bytes per dispatch of the kernels matching regex: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) each scaled by what the counter reads for a device copy of copy_mib MiB."""
    def per_dispatch(path, pat):
        acc = {}
        for r in csv.DictReader(open(path)):
            if re.search(pat, r["Kernel_Name"]):
                acc.setdefault(r["Kernel_Name"], {}).setdefault(r["Dispatch_Id"], 0.0)
                acc[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
        return {k: sum(v.values()) / len(v) for k, v in acc.items()}
    true_kib = copy_mib * 1024.0
    cf = true_kib / max(per_dispatch(copy_fetch_csv, "copyBuffer").values())
    cw = true_kib / max(per_dispatch(copy_write_csv, "copyBuffer").values())
    print(f"calibration (copy of {copy_mib} MiB): FETCH_SIZE x {cf:.3f}, WRITE_SIZE x {cw:.3f}")
    f = per_dispatch(fetch_csv, regex)
    w = per_dispatch(write_csv, regex)
    for k in sorted(f):
        fb = f[k] * cf * 1024.0
        wb = w.get(k, 0.0) * cw * 1024.0
        print(f"{k[:70]:70s} fetch {fb / 1e6:10.1f} MB  write {wb / 1e6:8.1f} MB  total {(fb + wb) / 1e6:10.1f} MB"
              f"  ({int(round(fb + wb))} B)")


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
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("regex")
    t.add_argument("--last", type=int, default=0)
    t.add_argument("--min-us", type=float, default=0.0)
    tr = sub.add_parser("traffic")
    tr.add_argument("fetch_csv")
    tr.add_argument("write_csv")
    tr.add_argument("copy_fetch_csv")
    tr.add_argument("copy_write_csv")
    tr.add_argument("regex")
    tr.add_argument("--copy-mib", type=int, default=1024)
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        copy_probe(a.mib, a.reps)
    elif a.cmd == "stats":
        stats(a.csv, a.top)
    elif a.cmd == "trace":
        trace_avg(a.csv, a.regex, a.last, a.min_us)
    elif a.cmd == "traffic":
        traffic(a.fetch_csv, a.write_csv, a.copy_fetch_csv, a.copy_write_csv, a.regex, a.copy_mib)
    else:
        pmc(a.csv, a.regex)


if __name__ == "__main__":
    main(sys.argv[1:])
