#!/usr/bin/env python3
"""Throughput of the RI-CCSD particle-particle ladder on one MI355X.

One step = one ``ri_ppl`` call (eq. pp-Ladder-0): the tau+- packing, the tile-by-tile
(ac|bd) build on MFMA, the packed contraction and the mirrored accumulation into R,
with every input already resident in HBM.  Default workload: o=16, v=256, naux=768
(seed 2), tau = MP2 t2 + t1 (x) t1, FP64.  Prints one JSON line on stdout.

  python bench.py [--steps K] [--warmup W] [--workload c2|c4] [--precision fp64|...]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PPL TFLOP/s + MFMA util; time-to-converged E_corr (≤1 µEh), mixed vs FP64"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3.0}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3 (f32 accumulate)"}
DOMINANT = {"fp64": "build_w_f64", "fp32": "build_w_f32", "bf16x3": "build_w_bf16x3"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    for name in ("ppl.hip", "ppl_bf16.hip", "ppl_shared.h", "ri_common.h"):
        with open(os.path.join(ROOT, "paper_1810_08142_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str, workload: str):
    """HBM bytes per launch from a committed counter summary, if it was taken on
    the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def mfma_from_profiles(kernel: str, workload: str):
    """Counter-measured MFMA utilisation of the kernel from a committed summary, if it
    was taken on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_mfma.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if not d or d.get("source_hash") != source_hash():
        return None
    keep = ("mfma_util", "mfma_busy_frac", "executed_tflops", "algorithmic_share", "peak_tflops")
    return {k: (round(d[k], 4) if isinstance(d.get(k), float) else d.get(k)) for k in keep}


def make_inputs(workload: str):
    """B_vv, tau (host FP64) for a ladder workload; tau = MP2 t2 + t1 (x) t1."""
    import torch
    from paper_1810_08142_amd import ccsd, ppl
    from paper_1810_08142_amd.synthetic import CONFIGS, draw_system
    c = CONFIGS[workload]
    s = draw_system(c["o"], c["v"], c["naux"], seed=c["seed"])
    B = torch.from_numpy(s.B).to("cuda")
    eps = torch.from_numpy(s.eps).to("cuda")
    t1 = torch.from_numpy(s.t1).to("cuda")
    t2, _ = ccsd.mp2_guess(B, eps, s.o)
    tau = ppl.build_tau(t1, t2)
    B_vv = B[:, s.o:, s.o:].contiguous()
    del B, t2
    torch.cuda.synchronize()
    return s, B_vv, tau


def cpu_baseline(s, workload: str, flops_call: float, seconds: float):
    """The FP64 CPU oracle on a bounded sample of the same call: R^{ab}_{ij} for
    random (a, b) pairs (all i, j), in batches until `seconds` have elapsed."""
    from oracle import ccsd as oc
    from oracle import native
    o, v = s.o, s.v
    t1, t2, _ = oc.mp2(s.B, s.eps, o)
    tau = oc.make_tau(s.t1, t2)
    B_vv = np.ascontiguousarray(s.B[:, o:, o:])
    threads = native.num_threads()
    rng = np.random.default_rng(11)
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        pairs = rng.integers(0, v, size=(2 * threads, 2))
        native.ppl_pairs(B_vv, tau, pairs)
        done += len(pairs)
    dt = time.perf_counter() - t0
    frac = done / float(v * v)
    return {"value": flops_call * frac / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} random (a,b) pairs of the {workload} call (all i,j) in {dt:.1f} s; "
                      f"credited with that fraction ({frac:.2e}) of the call's algorithmic FLOP"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c2", "c4"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one plain device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding of the ladder is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1810_08142_amd import _lib, ppl
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    log(f"[bench] drawing workload {args.workload}")
    s, B_vv, tau = make_inputs(args.workload)
    o, v, naux = s.o, s.v, s.naux
    R = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    flops = ppl.flops(o, v, naux)
    stream = torch.cuda.current_stream()

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_calibration} MiB device to device for counter calibration")
        del src, dst
    for w in range(args.warmup):
        ppl.ppl(B_vv, tau, R, precision=args.precision)
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    _lib.prof_enable(True)
    _lib.prof_report()  # clear
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for k in range(args.steps):
        ppl.ppl(B_vv, tau, R, precision=args.precision)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    _lib.prof_enable(False)
    kernels = _lib.prof_report()
    log(f"[bench] timed {args.steps} steps: {total_ms:.1f} ms")
    ms = total_ms / args.steps
    if not torch.isfinite(R).all():
        print("bench.py: non-finite result", file=sys.stderr)
        sys.exit(1)

    phases = {k["name"]: round(k["ms"] / args.steps, 4) for k in kernels}
    dom = DOMINANT[args.precision]
    kd = next(k for k in kernels if k["name"] == dom)
    achieved = kd["flops"] / (kd["ms"] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    traffic = traffic_from_profiles(dom, args.workload)
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic, "kernel": dom,
                "kernel_ms_per_launch": round(kd["ms"] / kd["count"], 4),
                "mfma_counters": mfma_from_profiles(dom, args.workload)}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(s, args.workload, flops, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(flops / (ms * 1e-3) / 1e12, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic (seeded RI factors and orbital energies; tau = MP2 t2 + t1 t1)",
        "config": {"workload": f"{args.workload}: one ladder call o={o} v={v} naux={naux}",
                   "o": o, "v": v, "naux": naux, "seed": s.seed, "precision": args.precision,
                   "algorithmic_flop_per_step": flops},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases_ms": phases,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
