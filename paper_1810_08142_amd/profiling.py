"""Summaries of rocprofv3 output for the benchmark's kernels.

  python -m paper_1810_08142_amd.profiling stats <run_kernel_stats.csv> [--top N]
  python -m paper_1810_08142_amd.profiling traffic --kernel NAME --fetch <FETCH csv> --write <WRITE csv>
                                                   --out profiles/NAME_c2_counters.json
  python -m paper_1810_08142_amd.profiling mfma --kernel NAME --pmc <csv> --flops F --peak P
                                                --out profiles/NAME_c2_mfma.json

`traffic` converts the per-dispatch FETCH_SIZE / WRITE_SIZE counters (KiB) of a
kernel into bytes per launch, scaled by what the same counters read for the plain
device-to-device copy (__amd_rocclr_copyBuffer) of known size in the same run, and
stamps the result with the hash of the ladder sources it was taken on.

`mfma` reads one counter run with SQ_INSTS_VALU_MFMA_MOPS_F64, _MOPS_BF16,
SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE: the MFMA FLOP the hardware executed
per launch (MOPS x 512), their rate over the dispatch duration against the peak, the
algorithmic share of them (F / executed; the rest is padding), and the fraction of
SIMD cycles with the matrix core busy.
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


SIMDS = 256 * 4  # compute units x SIMDs per unit
XCDS = 8  # GRBM_GUI_ACTIVE comes summed over the XCDs; the busy fraction wants one XCD's count


def mfma(kernel: str, pmc_csv: str, algo_flops: float, peak_tflops: float, source_hash: str):
    per = {}
    for r in csv.DictReader(open(pmc_csv)):
        if kernel not in r["Kernel_Name"]:
            continue
        d = per.setdefault(r["Dispatch_Id"], {"ns": float(r["End_Timestamp"]) - float(r["Start_Timestamp"])})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    rows = list(per.values())
    if not rows:
        return None
    n = len(rows)
    mops = sum(r.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) + r.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0)
               for r in rows) / n
    ns = sum(r["ns"] for r in rows) / n
    busy = sum(r.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for r in rows) / n
    active = sum(r.get("GRBM_GUI_ACTIVE", 0.0) for r in rows) / n
    executed = mops * 512.0
    return dict(kernel=kernel, source_hash=source_hash, launches=n, counters_per_launch={k: v for k, v in rows[0].items()},
                executed_mfma_flop_per_launch=executed, algorithmic_flop_per_launch=algo_flops,
                algorithmic_share=algo_flops / executed if executed else None,
                executed_tflops=executed / (ns * 1e-9) / 1e12 if ns else None,
                mfma_util=executed / (ns * 1e-9) / 1e12 / peak_tflops if ns else None,
                mfma_busy_frac=busy / (active / XCDS * SIMDS) if active else None, peak_tflops=peak_tflops)


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
    m = sub.add_parser("mfma")
    m.add_argument("--kernel", required=True)
    m.add_argument("--pmc", required=True)
    m.add_argument("--flops", type=float, required=True, help="algorithmic FLOP per launch")
    m.add_argument("--peak", type=float, required=True, help="peak TFLOP/s of the kernel's MFMA type")
    m.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(kernel_stats(args.csv, args.top))
    elif args.cmd == "mfma":
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import bench
        d = mfma(args.kernel, args.pmc, args.flops, args.peak, bench.source_hash())
        with open(args.out, "w") as fh:
            json.dump(d, fh, indent=1)
        print(json.dumps(d))
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
