"""Command-line runs of the GPU RI-CCSD solver on the synthetic workloads.

  python -m paper_1810_08142_amd.cli ccsd --config c5 [--scale verbatim|naux] [--precision fp64|bf16x3]
                                        [--polish 1e-6] [--check-fp64] [--model net.bin]
  python -m paper_1810_08142_amd.cli ttc --config c3 --scale naux [--polish 1e-6]
  python -m paper_1810_08142_amd.cli shard --config c4 --nshards 8 [--precision fp64|fp32|bf16x3]
  python -m paper_1810_08142_amd.cli ablation --config c2 [--forms tau_pm,paper,sym]
  python -m paper_1810_08142_amd.cli triples --config c5 [--scale naux] [--precision fp64|bf16x3]

`ccsd` prints one JSON line with the report (energy, iterations, timings, scale
used).  `ttc` (time to converged E_corr) solves one system four times -- FP64
ladder, mixed ladder, mixed ladder with FP64 polish, mixed ladder with FP32 polish --
and prints one JSON line per run with its E_corr error against the FP64 run and the
FP64 residual of its final amplitudes.  `shard` times every shard k of n of one ladder call (ri_ppl_shard, the
per-device work of an n-device split over the (ab) slabs) one after another and prints
the slowest and mean shard, with the R bytes one device would contribute to the
all-gather that completes the call.  `ablation` times one ladder call in the paper's
arrangement (ri_ppl_paper: full (a, b) build, i <= j pairs) against the tau+- form
(ri_ppl, FP64) on the same inputs, and the exchange-symmetric form (ri_ppl_sym: about
half the build) beside them, with each one's own FLOP count and the largest
difference of each result from ri_ppl's.  `triples` converges CCSD and evaluates the
perturbative triples energy E_(T) (ri_ccsd_triples) at the result, with its time and
FLOP rate.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("ccsd")
    c.add_argument("--config", default="c1")
    c.add_argument("--scale", default="verbatim")
    c.add_argument("--precision", default="fp64")
    c.add_argument("--max-iter", type=int, default=100)
    c.add_argument("--tol", type=float, default=1e-8)
    c.add_argument("--tol-energy", type=float, default=1e-9)
    c.add_argument("--diis", type=int, default=6)
    c.add_argument("--verbose", action="store_true")
    c.add_argument("--polish", type=float, default=0.0)
    c.add_argument("--polish-precision", default="fp64")
    c.add_argument("--other-precision", default="fp64")
    c.add_argument("--check-fp64", action="store_true")
    c.add_argument("--model", default="")
    t = sub.add_parser("ttc")
    t.add_argument("--config", default="c3")
    t.add_argument("--scale", default="naux")
    t.add_argument("--mixed", default="bf16x3")
    t.add_argument("--polish", type=float, default=1e-6)
    t.add_argument("--other", default="fp64", help="precision of the other large contractions in the mixed runs")
    t.add_argument("--max-iter", type=int, default=100)
    t.add_argument("--tol", type=float, default=1e-8)
    t.add_argument("--tol-energy", type=float, default=1e-9)
    t.add_argument("--verbose", action="store_true")
    tr = sub.add_parser("triples")
    tr.add_argument("--config", default="c1")
    tr.add_argument("--scale", default="naux")
    tr.add_argument("--precision", default="fp64", help="ladder precision of the CCSD solve")
    tr.add_argument("--tol", type=float, default=1e-8)
    tr.add_argument("--triples-precision", default="fp64", help="arithmetic of the (T) term GEMMs: fp64 or fp32")
    tr.add_argument("--kernels", action="store_true",
                    help="one more call under the library's event profiler; per-kernel times on stderr")
    ab = sub.add_parser("ablation")
    ab.add_argument("--config", default="c2")
    ab.add_argument("--repeat", type=int, default=2)
    ab.add_argument("--forms", default="tau_pm,paper,sym",
                    help="comma list of tau_pm, paper, sym, tau_pm_fp32, tau_pm_bf16x3, sym_bf16x3, sym_fp32")
    sh = sub.add_parser("shard")
    sh.add_argument("--config", default="c4")
    sh.add_argument("--nshards", type=int, default=8)
    sh.add_argument("--precision", default="fp64")
    args = ap.parse_args(argv)
    if args.cmd == "ttc":
        return _ttc(args)
    if args.cmd == "shard":
        return _shard(args)
    if args.cmd == "ablation":
        return _ablation(args)
    if args.cmd == "triples":
        return _triples(args)

    import torch

    from . import ccsd
    from .synthetic import CONFIGS, draw_system
    cfg = CONFIGS[args.config]
    t0 = time.perf_counter()
    s = draw_system(cfg["o"], cfg["v"], cfg["naux"], seed=cfg["seed"], scale=args.scale)
    B = torch.from_numpy(s.B).to("cuda")
    eps = torch.from_numpy(s.eps).to("cuda")
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    from ._lib import RIError
    net = None
    if args.model:
        from .mlp import Net
        net = Net.load(args.model)
    try:
        t1, t2, rep = ccsd.solve(B, eps, s.o, max_iter=args.max_iter, tol=args.tol, tol_energy=args.tol_energy,
                                 diis_size=args.diis, ppl_precision=args.precision, verbose=args.verbose,
                                 polish_residual=args.polish, check_fp64=args.check_fp64, mlp=net,
                                 polish_precision=args.polish_precision, other_precision=args.other_precision)
    except RIError as e:
        print(json.dumps(dict(config=args.config, scale=s.scale, precision=args.precision, error=str(e))), flush=True)
        return 4
    out = dict(config=args.config, o=s.o, v=s.v, naux=s.naux, seed=s.seed, scale=s.scale, precision=args.precision,
               e_corr=rep.e_corr, e_mp2=rep.e_mp2, iterations=rep.iterations, converged=rep.converged,
               residual_inf=rep.residual_inf, residual_rms=rep.residual_rms,
               residual_inf_fp64=rep.residual_inf_fp64, polish_iteration=rep.polish_iteration,
               seconds_total=rep.seconds_total, seconds_ppl=rep.seconds_ppl, seconds_guess=rep.seconds_guess,
               seconds_generate=t_gen, guess="mlp" if net is not None else "mp2", max_abs_t2=float(t2.abs().max()))
    print(json.dumps(out), flush=True)
    return 0 if rep.converged else 3


def _ttc(args):
    import torch

    from . import ccsd
    from .synthetic import CONFIGS, draw_system
    cfg = CONFIGS[args.config]
    s = draw_system(cfg["o"], cfg["v"], cfg["naux"], seed=cfg["seed"], scale=args.scale)
    B = torch.from_numpy(s.B).to("cuda")
    eps = torch.from_numpy(s.eps).to("cuda")
    torch.cuda.synchronize()
    runs = [("fp64", "fp64", 0.0, "fp64", "fp64"), ("mixed", args.mixed, 0.0, "fp64", args.other),
            ("mixed+polish", args.mixed, args.polish, "fp64", args.other),
            ("mixed+fp32 polish", args.mixed, args.polish, "fp32", args.other)]
    ref = None
    rc = 0
    for name, prec, pol, pprec, oprec in runs:
        _, _, rep = ccsd.solve(B, eps, s.o, max_iter=args.max_iter, tol=args.tol, tol_energy=args.tol_energy,
                               ppl_precision=prec, polish_residual=pol, check_fp64=True, verbose=args.verbose,
                               polish_precision=pprec, other_precision=oprec)
        if ref is None:
            ref = rep
        out = dict(config=args.config, o=s.o, v=s.v, naux=s.naux, seed=s.seed, scale=s.scale, run=name,
                   precision=prec, other_precision=oprec, polish_residual=pol, polish_precision=pprec, tol=args.tol,
                   tol_energy=args.tol_energy,
                   converged=rep.converged, iterations=rep.iterations, polish_iteration=rep.polish_iteration,
                   e_corr=rep.e_corr, delta_e_vs_fp64=rep.e_corr - ref.e_corr,
                   residual_inf=rep.residual_inf, residual_inf_fp64=rep.residual_inf_fp64,
                   seconds_total=rep.seconds_total, seconds_ppl=rep.seconds_ppl,
                   speedup_vs_fp64=ref.seconds_total / rep.seconds_total)
        print(json.dumps(out), flush=True)
        rc = rc or (0 if rep.converged else 3)
    return rc


def _inputs(config):
    """B_vv and tau = MP2 t2 + t1 t1 of a ladder workload, on the device."""
    import torch

    from . import ccsd, ppl
    from .synthetic import CONFIGS, draw_system
    cfg = CONFIGS[config]
    s = draw_system(cfg["o"], cfg["v"], cfg["naux"], seed=cfg["seed"])
    o = s.o
    B = torch.from_numpy(s.B).to("cuda")
    eps = torch.from_numpy(s.eps).to("cuda")
    t1 = torch.from_numpy(s.t1).to("cuda")
    t2, _ = ccsd.mp2_guess(B, eps, o)
    tau = ppl.build_tau(t1, t2)
    B_vv = B[:, o:, o:].contiguous()
    return s.o, s.v, s.naux, B_vv, tau


def _triples(args):
    import torch

    from . import ccsd
    from .synthetic import CONFIGS, draw_system
    cfg = CONFIGS[args.config]
    s = draw_system(cfg["o"], cfg["v"], cfg["naux"], seed=cfg["seed"], scale=args.scale)
    o, v = s.o, s.v
    B = torch.from_numpy(s.B).to("cuda")
    eps = torch.from_numpy(s.eps).to("cuda")
    t1, t2, rep = ccsd.solve(B, eps, o, tol=args.tol, tol_energy=0.1 * args.tol, ppl_precision=args.precision,
                             polish_residual=1e-6 if args.precision != "fp64" else 0.0)
    print(json.dumps(dict(ccsd_iterations=rep.iterations, ccsd_seconds=rep.seconds_total, e_corr=rep.e_corr)),
          file=sys.stderr, flush=True)
    tp = args.triples_precision
    ccsd.triples(B, eps, o, t1, t2, precision=tp)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_t = ccsd.triples(B, eps, o, t1, t2, precision=tp)
    dt = time.perf_counter() - t0
    fl = ccsd.triples_flops(o, v)
    if args.kernels:
        from . import _lib
        _lib.prof_enable(True)
        _lib.prof_report()
        ccsd.triples(B, eps, o, t1, t2, precision=tp)
        _lib.prof_enable(False)
        for r in sorted(_lib.prof_report(), key=lambda r: -r["ms"]):
            print(json.dumps(r), file=sys.stderr, flush=True)
    print(json.dumps(dict(config=args.config, o=o, v=v, naux=s.naux, scale=s.scale, ccsd_precision=args.precision,
                          ccsd_converged=rep.converged, e_corr=rep.e_corr, triples_precision=tp, e_triples=e_t,
                          triples_seconds=dt,
                          triples_flop=fl, triples_tflops=fl / dt / 1e12)), flush=True)
    return 0 if rep.converged else 3


def _ablation(args):
    import torch

    from . import ppl
    o, v, naux, B_vv, tau = _inputs(args.config)
    out = dict(config=args.config, o=o, v=v, naux=naux)
    res = {}
    forms = {"tau_pm": (lambda R: ppl.ppl(B_vv, tau, R), ppl.flops(o, v, naux)),
             "paper": (lambda R: ppl.ppl_paper(B_vv, tau, R), ppl.paper_flops(o, v, naux)),
             "sym": (lambda R: ppl.ppl_sym(B_vv, tau, R), ppl.sym_flops(o, v, naux)),
             "tau_pm_fp32": (lambda R: ppl.ppl(B_vv, tau, R, precision="fp32"), ppl.flops(o, v, naux)),
             "tau_pm_bf16x3": (lambda R: ppl.ppl(B_vv, tau, R, precision="bf16x3"), ppl.flops(o, v, naux)),
             "sym_bf16x3": (lambda R: ppl.ppl_sym(B_vv, tau, R, precision="bf16x3"), ppl.sym_flops(o, v, naux)),
             "sym_fp32": (lambda R: ppl.ppl_sym(B_vv, tau, R, precision="fp32"), ppl.sym_flops(o, v, naux))}
    names = ["tau_pm"] + [f for f in args.forms.split(",") if f != "tau_pm"]
    for name in names:
        call, fl = forms[name]
        R = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
        call(R)  # warm-up (and the result compared below)
        torch.cuda.synchronize()
        best = None
        for _ in range(args.repeat):
            Rt = torch.zeros_like(R)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            call(Rt)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
            del Rt
        res[name] = R
        out[name] = dict(ms=best, flop=fl, tflops=fl / (best * 1e-3) / 1e12)
        print(json.dumps({name: out[name]}), file=sys.stderr, flush=True)
    rmax = res["tau_pm"].abs().max().item()
    for name in names[1:]:
        out[f"{name}_max_abs_diff_rel"] = (res[name] - res["tau_pm"]).abs().max().item() / rmax
        out[f"{name}_over_tau_pm_time"] = out[name]["ms"] / out["tau_pm"]["ms"]
    print(json.dumps(out), flush=True)
    return 0


def _shard(args):
    import torch

    from . import ccsd, ppl
    from .synthetic import CONFIGS, draw_system
    cfg = CONFIGS[args.config]
    s = draw_system(cfg["o"], cfg["v"], cfg["naux"], seed=cfg["seed"])
    o, v, naux = s.o, s.v, s.naux
    B = torch.from_numpy(s.B).to("cuda")
    eps = torch.from_numpy(s.eps).to("cuda")
    t1 = torch.from_numpy(s.t1).to("cuda")
    del s
    t2, _ = ccsd.mp2_guess(B, eps, o)
    tau = ppl.build_tau(t1, t2)
    B_vv = B[:, o:, o:].contiguous()
    del B, t2
    R = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    ppl.ppl(B_vv, tau, R, precision=args.precision, shard=(0, args.nshards))  # warm-up
    torch.cuda.synchronize()
    ms = []
    for k in range(args.nshards):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ppl.ppl(B_vv, tau, R, precision=args.precision, shard=(k, args.nshards))
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
        print(json.dumps(dict(shard=k, ms=ms[-1])), file=sys.stderr, flush=True)
    flops = ppl.flops(o, v, naux)
    out = dict(config=args.config, o=o, v=v, naux=naux, precision=args.precision, nshards=args.nshards,
               shard_ms=ms, max_shard_ms=max(ms), mean_shard_ms=sum(ms) / len(ms), sum_ms=sum(ms),
               imbalance=max(ms) / (sum(ms) / len(ms)),
               tflops_per_device_at_max=flops / args.nshards / (max(ms) * 1e-3) / 1e12,
               r_bytes_per_device=8.0 * o * o * v * v / args.nshards)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
