"""Summaries of rocprofv3 output for the benchmark's kernels.

  python -m paper_1810_08142_amd.profiling stats <run_kernel_stats.csv> [--top N]
  python -m paper_1810_08142_amd.profiling traffic --kernel NAME --fetch <FETCH csv> --write <WRITE csv>
                                                   --out profiles/NAME_c2_counters.json
  python -m paper_1810_08142_amd.profiling mfma --kernel NAME --pmc <csv> --flops F --peak P
                                                --out profiles/NAME_c2_mfma.json
  python -m paper_1810_08142_amd.profiling calltraffic --label P --fetch <FETCH csv> --write <WRITE csv>
                                                       --call-ms T

`traffic` converts the per-dispatch FETCH_SIZE / WRITE_SIZE counters (KiB) of a
kernel into bytes per launch, scaled by what the same counters read for the plain
device-to-device copy (__amd_rocclr_copyBuffer) of known size in the same run, and
stamps the result with the hash of the ladder sources it was taken on.

`calltraffic` sums the same counters per kernel over all dispatches of a call.

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


def is_kernel(name: str, kernel: str) -> bool:
    """True when the profiler's kernel name (e.g. 'void ri::ppl::f<8>(double const*)')
    names the function `kernel`: its unqualified name without template arguments."""
    base = name.split("(", 1)[0].split("<", 1)[0].strip()
    return base.rsplit("::", 1)[-1].split()[-1] == kernel if base else False


def _counter(path: str, kernel: str):
    vals, copy = [], []
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        if name.startswith("__amd_rocclr_copyBuffer"):
            copy.append(float(r["Counter_Value"]))
        elif is_kernel(name, kernel):
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


def _per_kernel(path: str, prefix: str = "ri::ppl::"):
    """{kernel: [counter sum, summed dispatch ns, dispatches]} over the kernels whose
    qualified name starts with `prefix` (the ladder's), and the largest copy-kernel
    reading (the calibration copy)."""
    per, copy = {}, None
    for r in csv.DictReader(open(path)):
        n = r["Kernel_Name"]
        if n.startswith("__amd_rocclr_copyBuffer"):
            copy = max(copy or 0.0, float(r["Counter_Value"]))
            continue
        if not n.replace("void ", "", 1).startswith(prefix):
            continue
        k = n.split("(", 1)[0].split("<", 1)[0].strip().rsplit("::", 1)[-1]
        e = per.setdefault(k, [0.0, 0.0, 0])
        e[0] += float(r["Counter_Value"])
        e[1] += float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
        e[2] += 1
    return per, copy


def call_traffic(label: str, fetch_csv: str, write_csv: str, copy_mib: int, call_ms: float) -> str:
    """Per-kernel HBM bytes of a whole call (FETCH_SIZE and WRITE_SIZE summed over its
    dispatches, each scaled by the calibration copy), as text lines."""
    f, fc = _per_kernel(fetch_csv)
    w, wc = _per_kernel(write_csv)
    ff, fw = copy_mib * 1024.0 / fc, copy_mib * 1024.0 / wc
    total, lines = 0.0, []
    for k in f:
        rd, wr = f[k][0] * ff * 1024.0, w.get(k, [0.0])[0] * fw * 1024.0
        total += rd + wr
        lines.append(f"#   {k:24s} launches {f[k][2]:4d}  HBM {(rd + wr) / 1e9:10.1f} GB  ({rd / 1e9:9.1f} read, "
                     f"{wr / 1e9:8.1f} written)  {(rd + wr) / (f[k][1] * 1e-9) / 1e9:7.0f} GB/s over its own time")
    head = (f"# {label} total {total / 1e9:.1f} GB in {call_ms:.0f} ms -> {total / (call_ms * 1e-3) / 1e9:.0f} GB/s "
            f"factors {ff:.4f} {fw:.4f}")
    return "\n".join([head] + lines)


SIMDS = 256 * 4  # compute units x SIMDs per unit
XCDS = 8  # GRBM_GUI_ACTIVE comes summed over the XCDs; the busy fraction wants one XCD's count


def mfma(kernel: str, pmc_csv: str, algo_flops: float, peak_tflops: float, source_hash: str):
    per = {}
    for r in csv.DictReader(open(pmc_csv)):
        if not is_kernel(r["Kernel_Name"], kernel):
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
    keys = sorted({k for r in rows for k in r})
    mean = {k: sum(r.get(k, 0.0) for r in rows) / n for k in keys}  # "ns" included: the mean dispatch time
    return dict(kernel=kernel, source_hash=source_hash, launches=n, counters_mean_per_launch=mean,
                counters_first_dispatch={k: v for k, v in rows[0].items()},
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
    c = sub.add_parser("calltraffic")
    c.add_argument("--label", required=True)
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--copy-mib", type=int, default=1024)
    c.add_argument("--call-ms", type=float, required=True, help="the call's time from the same run's bench log")
    args = ap.parse_args(argv)
    if args.cmd == "calltraffic":
        print(call_traffic(args.label, args.fetch, args.write, args.copy_mib, args.call_ms))
    elif args.cmd == "stats":
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
