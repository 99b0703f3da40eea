"""Summaries of rocprofv3 output for the benchmark's kernels.

  python -m paper_1810_08142_amd.profiling stats <run_kernel_stats.csv> [--top N]
  python -m paper_1810_08142_amd.profiling traffic --kernel NAME --fetch <FETCH csv> --write <WRITE csv>
                                                   --workload c2 --out profiles/NAME_c2_counters.json

`traffic` converts the per-dispatch FETCH_SIZE / WRITE_SIZE counters (KiB) of a
kernel into bytes per launch, scaled by what the same counters read for the plain
device-to-device copy (__amd_rocclr_copyBuffer) of known size in the same run, and
stamps the result with the hash of the ladder sources it was taken on.
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import sys


def kernel_stats(path: str, top: int = 12) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"{'kernel':64s} {'calls':>6s} {'total ms':>10s} {'avg ms':>10s} {'%':>6s}"]
    for r in rows[:top]:
        name = r["Name"]
        name = name if len(name) <= 64 else name[:61] + "..."
        lines.append(f"{name:64s} {int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                     f"{float(r['AverageNs']) / 1e6:10.4f} {float(r['Percentage']):6.2f}")
    return "\n".join(lines)


def _counter(path: str, kernel: str):
    vals, copy = [], []
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        if name.startswith("__amd_rocclr_copyBuffer"):
            copy.append(float(r["Counter_Value"]))
        elif kernel in name:
            vals.append(float(r["Counter_Value"]))
    return vals, max(copy) if copy else None


def traffic(kernel: str, fetch_csv: str, write_csv: str, copy_mib: int, source_hash: str):
    f, fc = _counter(fetch_csv, kernel)
    w, wc = _counter(write_csv, kernel)
    kib = copy_mib * 1024.0
    ff = kib / fc if fc else None
    fw = kib / wc if wc else None
    per = [(a * ff + b * fw) * 1024.0 for a, b in zip(f, w)]
    return dict(kernel=kernel, source_hash=source_hash, fetch_kib=f, write_kib=w,
                copy_calibration=dict(mib=copy_mib, fetch_kib=fc, write_kib=wc, fetch_factor=ff, write_factor=fw),
                hbm_bytes_per_launch=sum(per) / len(per) if per else None, launches=len(per))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=12)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-mib", type=int, default=1024)
    t.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(kernel_stats(args.csv, args.top))
    else:
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import bench
        d = traffic(args.kernel, args.fetch, args.write, args.copy_mib, bench.source_hash())
        with open(args.out, "w") as fh:
            json.dump(d, fh, indent=1)
        print(json.dumps(d))
    return 0


if __name__ == "__main__":
    sys.exit(main())
