"""Command-line runs of the GPU RI-CCSD solver on the synthetic workloads.

  python -m paper_1810_08142_amd.cli ccsd --config c5 [--scale verbatim|naux] [--precision fp64|bf16x3]

Prints one JSON line with the report (energy, iterations, timings, scale used).
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
    args = ap.parse_args(argv)

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
    try:
        t1, t2, rep = ccsd.solve(B, eps, s.o, max_iter=args.max_iter, tol=args.tol, tol_energy=args.tol_energy,
                                 diis_size=args.diis, ppl_precision=args.precision, verbose=args.verbose)
    except RIError as e:
        print(json.dumps(dict(config=args.config, scale=s.scale, precision=args.precision, error=str(e))), flush=True)
        return 4
    out = dict(config=args.config, o=s.o, v=s.v, naux=s.naux, seed=s.seed, scale=s.scale, precision=args.precision,
               e_corr=rep.e_corr, e_mp2=rep.e_mp2, iterations=rep.iterations, converged=rep.converged,
               residual_inf=rep.residual_inf, seconds_total=rep.seconds_total, seconds_ppl=rep.seconds_ppl,
               seconds_generate=t_gen, max_abs_t2=float(t2.abs().max()))
    print(json.dumps(out), flush=True)
    return 0 if rep.converged else 3


if __name__ == "__main__":
    sys.exit(main())
