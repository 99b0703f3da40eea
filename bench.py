#!/usr/bin/env python3
"""Throughput of the RI-CCSD particle-particle ladder on one MI355X.

One step = one ladder call (eq. pp-Ladder-0): the tau+- packing, the tile-by-tile
(ac|bd) build on MFMA, the packed contraction and the mirrored accumulation into R,
with every input already resident in HBM.  Default workload: o=48, v=768, naux=2304
(seed 4; B_vv, tau and R 10.9 GB each), tau = MP2 t2 + t1 (x) t1, timed in the split-bf16
arithmetic the ladder runs in inside CCSD; then the same call in FP64 (one untimed and
--fp64-steps timed calls) for the mixed-vs-FP64 comparison.  The metric's second half,
time to converged E_corr, is the `ttc` object: closed-shell RI-CCSD at o=32, v=512,
naux=1536 (seed 3, Naux-scaled generator) from the MP2 guess to max |Omega| <= 1e-8
and |dE| <= 1e-9, once with the FP64 ladder and once with the split-bf16 ladder (other
terms FP64), wall time of each solve and the energy difference (--no-ttc skips it).
Prints one JSON line on stdout.

  python bench.py [--steps K] [--warmup W] [--workload c4|c2] [--precision bf16x3|fp64|fp32]
                  [--fp64-steps N] [--no-ttc]
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


def ttc_leg():
    """Time to converged E_corr at o=32 v=512 naux=1536 with the FP64 and with the
    split-bf16 ladder (the other terms FP64 in both), each solve timed whole (its own
    setup included, inputs already on the device)."""
    import torch

    from paper_1810_08142_amd import ccsd
    from paper_1810_08142_amd.synthetic import CONFIGS, draw_system
    cfg = CONFIGS["c3"]
    s = draw_system(cfg["o"], cfg["v"], cfg["naux"], seed=cfg["seed"], scale="naux")
    B = torch.from_numpy(s.B).to("cuda")
    eps = torch.from_numpy(s.eps).to("cuda")
    torch.cuda.synchronize()
    runs = {}
    for prec in ("fp64", "bf16x3"):
        log(f"[bench] time to converged E_corr, {prec} ladder")
        _, _, rep = ccsd.solve(B, eps, s.o, max_iter=100, tol=1e-8, tol_energy=1e-9, ppl_precision=prec,
                               check_fp64=True)
        runs[prec] = rep
    f, m = runs["fp64"], runs["bf16x3"]
    de = m.e_corr - f.e_corr
    return {"workload": f"c3: RI-CCSD o={s.o} v={s.v} naux={s.naux}, seed {s.seed}, scale {s.scale:.4g}",
            "tol": 1e-8, "tol_energy": 1e-9,
            "fp64": {"seconds": round(f.seconds_total, 3), "ladder_seconds": round(f.seconds_ppl, 3),
                     "iterations": f.iterations, "converged": bool(f.converged), "e_corr": f.e_corr},
            "mixed": {"ladder": "bf16x3", "seconds": round(m.seconds_total, 3),
                      "ladder_seconds": round(m.seconds_ppl, 3), "iterations": m.iterations,
                      "converged": bool(m.converged), "e_corr": m.e_corr,
                      "fp64_residual_inf": m.residual_inf_fp64},
            "speedup_mixed_vs_fp64": round(f.seconds_total / m.seconds_total, 3),
            "delta_e_corr": de, "within_1_uEh": bool(abs(de) <= 1e-6)}


def cpu_baseline(s, workload: str, flops_call: float, seconds: float):
    """The FP64 CPU oracle on a bounded sample of the same call: R^{ab}_{ij} for
    random (a, b) pairs (all i, j), in batches until `seconds` have elapsed.  The
    oracle's work per pair does not depend on the amplitude values, so tau is any
    pair-symmetric array (all ones) rather than the MP2 amplitudes, which would take
    the host longer to form than the sample itself at the large sizes."""
    from oracle import native
    o, v, naux = s.o, s.v, s.naux
    tau = np.ones((o, o, v, v))
    B_vv = s.B_vv
    threads = native.num_threads()
    rng = np.random.default_rng(11)
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        pairs = rng.integers(0, v, size=(2 * threads, 2))
        native.ppl_pairs(B_vv, tau, pairs)
        done += len(pairs)
    dt = time.perf_counter() - t0
    frac = done / float(v * v)
    dense = 2.0 * done * v * v * (naux + o * o)  # what the oracle executes: (ac|bd) for all c, d, then tau
    return {"value": flops_call * frac / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "executed_tflops": dense / dt / 1e12,
            "sample": f"{done} random (a,b) pairs of the {workload} call (all i,j; tau = ones) in {dt:.1f} s; "
                      f"value credits the call's algorithmic FLOP for that fraction ({frac:.2e}) of its pairs; "
                      f"executed_tflops is the dense definition the oracle runs, 2 v^2 (naux + o^2) per pair"}


def cpu_plan(repeat: int = 3):
    """The CPU-baseline plan: the FP64 oracle on all host cores and on one core, the
    median of `repeat` runs each.  Workloads: c1 (o=4 v=24 naux=96) full CCSD to 1e-10;
    c2 (o=16 v=256 naux=768) one whole ladder call on all cores, and on one core a
    256-pair sample scaled to the whole call (labelled as such); c4 (o=48 v=768
    naux=2304) a 64-pair sample on all cores and a 16-pair sample on one core.  The
    oracle's work does not depend on the amplitude values, so c4 takes tau = ones; c2
    takes the oracle's own MP2 amplitudes.  FLOP are those the oracle executes (dense
    definition) and, for the ladder, also the tau+- form's count for the same share
    of the call."""
    from threadpoolctl import threadpool_limits

    from oracle import ccsd as oc
    from oracle import native
    from paper_1810_08142_amd.synthetic import CONFIGS, draw_system

    def med(f):
        ts = []
        for k in range(repeat):
            t0 = time.perf_counter()
            f()
            ts.append(time.perf_counter() - t0)
            log(f"[cpu-plan]   run {k + 1}/{repeat}: {ts[-1]:.2f} s")
        return float(np.median(ts)), [round(t, 3) for t in ts]

    def ladder_flops(o, v, naux):
        pv, pvm, po, pom = v * (v + 1) / 2, v * (v - 1) / 2, o * (o + 1) / 2, o * (o - 1) / 2
        return naux * v**3 * (v + 1) + 2 * (pv * pv * po + pvm * pvm * pom)

    systems = {}
    for name in ("c1", "c2", "c4"):
        c = CONFIGS[name]
        log(f"[cpu-plan] drawing {name}")
        systems[name] = draw_system(c["o"], c["v"], c["naux"], seed=c["seed"])
    s2 = systems["c2"]
    _, t2, _ = oc.mp2(s2.B, s2.eps, s2.o)
    tau2, B2 = oc.make_tau(s2.t1, t2), s2.B_vv
    s4 = systems["c4"]
    B4, tau4 = s4.B_vv, np.ones((s4.o, s4.o, s4.v, s4.v))
    all_cores = native.num_threads()
    rows = []
    rng = np.random.default_rng(12)
    for threads in (all_cores, 1):
        native.set_num_threads(threads)
        with threadpool_limits(limits=threads):
            c1 = systems["c1"]
            t, ts = med(lambda: oc.solve(c1.B, c1.eps, c1.o))
            rows.append(dict(workload="c1 full CCSD to 1e-10", threads=threads, median_s=t, runs_s=ts))
            log(f"[cpu-plan] {threads} threads c1 CCSD {t:.3f} s")
            o, v, naux = s2.o, s2.v, s2.naux
            if threads > 1:
                t, ts = med(lambda: native.ppl(B2, tau2))
                frac = 1.0
                what = "c2 one ladder call"
            else:
                pairs = rng.integers(0, v, size=(256, 2))
                t, ts = med(lambda: native.ppl_pairs(B2, tau2, pairs))
                frac = 256 / float(v * v)
                what = "c2 ladder, 256 (a,b) pairs; whole call extrapolated"
            dense = 2.0 * v * v * (naux + o * o) * frac * v * v
            rows.append(dict(workload=what, threads=threads, median_s=t, runs_s=ts, fraction_of_call=frac,
                             whole_call_s=t / frac, executed_gflops=dense / t / 1e9,
                             tau_pm_credited_gflops=ladder_flops(o, v, naux) * frac / t / 1e9))
            log(f"[cpu-plan] {threads} threads {what}: {t:.2f} s")
            o, v, naux = s4.o, s4.v, s4.naux
            npair = 64 if threads > 1 else 16
            pairs = rng.integers(0, v, size=(npair, 2))
            t, ts = med(lambda: native.ppl_pairs(B4, tau4, pairs))
            frac = npair / float(v * v)
            rows.append(dict(workload=f"c4 ladder, {npair} (a,b) pairs (tau = ones)", threads=threads, median_s=t,
                             runs_s=ts, fraction_of_call=frac, whole_call_s_extrapolated=t / frac,
                             executed_gflops=2.0 * v * v * (naux + o * o) * npair / t / 1e9,
                             tau_pm_credited_gflops=ladder_flops(o, v, naux) * frac / t / 1e9))
            log(f"[cpu-plan] {threads} threads c4 {npair} pairs: {t:.2f} s")
    native.set_num_threads(all_cores)
    return {"cpu_plan": rows, "all_cores": all_cores, "repeat": repeat}


def timed_calls(ppl, B_vv, tau, R, precision, steps, warmup, stream, label):
    """Warm-up calls, then `steps` calls between events on the launch stream, with the
    library's per-kernel event profiler on.  Returns (ms per call, kernel records)."""
    import torch
    from paper_1810_08142_amd import _lib
    for w in range(warmup):
        ppl.ppl(B_vv, tau, R, precision=precision)
        torch.cuda.synchronize()
        log(f"[bench] {label} warmup {w + 1}/{warmup} done")
    _lib.prof_enable(True)
    _lib.prof_report()  # clear
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for k in range(steps):
        ppl.ppl(B_vv, tau, R, precision=precision)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    _lib.prof_enable(False)
    kernels = _lib.prof_report()
    log(f"[bench] {label}: timed {steps} calls in {total_ms:.1f} ms")
    return total_ms / steps, kernels


def roofline_of(kernels, precision, workload):
    dom = DOMINANT[precision]
    kd = next(k for k in kernels if k["name"] == dom)
    achieved = kd["flops"] / (kd["ms"] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[precision]
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic_from_profiles(dom, workload), "kernel": dom,
            "kernel_ms_per_launch": round(kd["ms"] / kd["count"], 4),
            "mfma_counters": mfma_from_profiles(dom, workload)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4", choices=["c2", "c4"])
    ap.add_argument("--precision", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--fp64-steps", type=int, default=1,
                    help="timed FP64 calls after the timed steps (after one untimed call); 0 skips the leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttc", action="store_true", help="skip the time-to-converged-E_corr leg")
    ap.add_argument("--cpu-plan", action="store_true",
                    help="only time the CPU oracle on its plan of workloads (all cores and one core) and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one plain device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding of the ladder is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    if args.cpu_plan:
        print(json.dumps(cpu_plan()), flush=True)
        return

    import torch
    from paper_1810_08142_amd import ppl
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    log(f"[bench] drawing workload {args.workload}")
    s, B_vv, tau = make_inputs(args.workload)
    o, v, naux = s.o, s.v, s.naux
    R = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    flops = ppl.flops(o, v, naux)
    stream = torch.cuda.current_stream()
    log(f"[bench] inputs resident after {time.perf_counter() - t_setup:.1f} s")

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_calibration} MiB device to device for counter calibration")
        del src, dst
    ms, kernels = timed_calls(ppl, B_vv, tau, R, args.precision, args.steps, args.warmup, stream, args.precision)
    if not torch.isfinite(R).all():
        print("bench.py: non-finite result", file=sys.stderr)
        sys.exit(1)
    phases = {k["name"]: round(k["ms"] / args.steps, 4) for k in kernels}
    roofline = roofline_of(kernels, args.precision, args.workload)

    fp64 = None
    if args.fp64_steps > 0 and args.precision != "fp64":
        ms64, k64 = timed_calls(ppl, B_vv, tau, R, "fp64", args.fp64_steps, 1, stream, "fp64")
        fp64 = {"ms_per_step": round(ms64, 3), "value": round(flops / (ms64 * 1e-3) / 1e12, 3), "unit": "TFLOP/s",
                "steps": args.fp64_steps, "warmup": 1, "speedup_of_timed_precision": round(ms64 / ms, 3),
                "roofline": roofline_of(k64, "fp64", args.workload),
                "phases_ms": {k["name"]: round(k["ms"] / args.fp64_steps, 4) for k in k64}}
    del R, tau, B_vv
    torch.cuda.synchronize()

    ttc = None
    if not args.no_ttc:
        ttc = ttc_leg()
        torch.cuda.synchronize()

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
        "fp64_same_call": fp64,
        "ttc": ttc,
        "phases_ms": phases,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
