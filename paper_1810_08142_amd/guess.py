"""Train and evaluate the learned starting guess for the doubles amplitudes.

Training data: seeded synthetic systems (256 with o ~ U{4..12}, v ~ U{40..120}, naux = 3v,
Naux-normalised factor scale; --large adds systems with o ~ U{10..16}, v = 16 o)
converged by the GPU CCSD solver from the MP2 guess.
The network predicts the relative correction r = t2_CCSD / t2_MP2 - 1 (clipped to
[-3, 3]); each system contributes amplitudes drawn with probability proportional to
t2_MP2^2, so the mean squared error in r weighs every sample as its squared error in
t2 would.  Features come from the MP2 quantities.  The network is trained with the
library's own forward/backward/Adam kernels and saved with ri_mlp_save.

  python -m paper_1810_08142_amd.guess train --out model.bin [--systems 256]
  python -m paper_1810_08142_amd.guess evaluate --model model.bin [--config c5]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def build_dataset(shapes, per_system: int, seed: int, scale="naux", tol: float = 1e-8, log=None):
    """(X [N][8] float32, Y [N] float32, info) from converged systems: raw features of
    amplitudes drawn with probability ~ t2_MP2^2 (with replacement; ri_mlp_sample, seed
    `seed` + system number) and their relative corrections t2_CCSD / t2_MP2 - 1, clipped
    to [-3, 3] (ri_mlp_targets).  Everything but the row gather runs in the library."""
    import torch

    from . import ccsd, mlp
    from .synthetic import draw_system
    Xs, Ys = [], []
    iters = []
    t0 = time.perf_counter()
    for k, (o, v, naux, sd) in enumerate(shapes):
        s = draw_system(o, v, naux, seed=sd, scale=scale)
        B = torch.from_numpy(s.B).to("cuda")
        eps = torch.from_numpy(s.eps).to("cuda")
        t2m, _ = ccsd.mp2_guess(B, eps, o)
        X = mlp.features(B, eps, o, t2m)
        _, t2, rep = ccsd.solve(B, eps, o, tol=tol, tol_energy=tol * 0.1, max_iter=200)
        if not rep.converged:
            if log:
                log(f"  system {k} (o={o} v={v}) did not converge; skipped")
            continue
        iters.append(rep.iterations)
        idx = mlp.sample(t2m, per_system, seed + k)
        Xs.append(X.index_select(0, idx).cpu().numpy())
        Ys.append(mlp.targets(t2.contiguous(), t2m, idx).cpu().numpy())
        if log and (k % 32 == 0 or k == len(shapes) - 1):
            log(f"  system {k + 1}/{len(shapes)} o={o} v={v}: {rep.iterations} iterations, "
                f"{time.perf_counter() - t0:.1f} s elapsed")
    info = dict(systems=len(Xs), mean_iterations=float(np.mean(iters)) if iters else None,
                seconds=time.perf_counter() - t0)
    return np.concatenate(Xs), np.concatenate(Ys), info


def train(X, Y, hidden=256, layers=2, epochs=30, batch=4096, lr=5e-4, seed=0, holdout=0.05, log=None):
    """Fit the network to (X, Y) with the library's training loop; returns (net, history).

    A held-out fraction (rows chosen by a seeded permutation) measures the fit after
    each epoch (history: held-out loss per epoch).  The library fits the feature
    standardisation and the output scale to the training rows (ri_mlp_fit_scaling),
    stores them in the network and applies them (ri_mlp_standardize)."""
    import torch

    from . import mlp
    rng = np.random.default_rng(seed + 1)
    perm0 = rng.permutation(X.shape[0])
    nho = max(1, int(holdout * X.shape[0]))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    ho, tr = dev(perm0[:nho]), dev(perm0[nho:])
    Xd, Yd = dev(X), dev(Y)
    Xtr, Ytr = Xd.index_select(0, tr), Yd.index_select(0, tr)
    net = mlp.Net(X.shape[1], hidden, layers)
    net.init(seed)
    net.fit_scaling(Xtr, Ytr)
    Xn, Yn = net.standardize(Xtr, Ytr)
    Xh, Yh = net.standardize(Xd.index_select(0, ho), Yd.index_select(0, ho))
    t0 = time.perf_counter()
    tl, vl = net.train(Xn, Yn, Xh, Yh, epochs=epochs, batch=batch, lr=lr, seed=seed + 2)
    if log:
        for ep in range(epochs):
            log(f"  epoch {ep + 1}/{epochs}: mean batch loss {tl[ep]:.4e}, held-out loss {vl[ep]:.4e} "
                "(target variance 1)")
        log(f"  training: {time.perf_counter() - t0:.1f} s")
    return net, [float(x) for x in vl]


def evaluate(net, config="c5", scale="naux", precision="fp64", tol=1e-8, log=None, polish_residual=0.0,
             polish_precision="fp64"):
    """Iterations and wall time to convergence from the MP2 and from the learned guess
    (the latter through the solver's learned-guess option, so its time includes the
    features and the network), plus the error of both guesses against the converged
    amplitudes."""
    import torch

    from . import ccsd
    from .synthetic import CONFIGS, draw_system
    c = CONFIGS[config]
    s = draw_system(c["o"], c["v"], c["naux"], seed=c["seed"], scale=scale)
    B = torch.from_numpy(s.B).to("cuda")
    eps = torch.from_numpy(s.eps).to("cuda")
    torch.cuda.synchronize()
    out = dict(config=config, o=s.o, v=s.v, naux=s.naux, seed=s.seed, scale=s.scale, precision=precision, tol=tol,
               polish_residual=polish_residual, polish_precision=polish_precision)
    kw = dict(tol=tol, tol_energy=tol * 0.1, ppl_precision=precision, polish_residual=polish_residual,
              polish_precision=polish_precision)
    _, t2a, ra = ccsd.solve(B, eps, s.o, **kw)
    _, t2b, rb = ccsd.solve(B, eps, s.o, mlp=net, **kw)
    # guess errors (outside the timed solves)
    _, t2g = net.guess(B, eps, s.o)
    t2m, _ = ccsd.mp2_guess(B, eps, s.o)
    out["initial_error"] = dict(mp2_max=float((t2m - t2a).abs().max()), learned_max=float((t2g - t2a).abs().max()),
                                mp2_rms=float((t2m - t2a).pow(2).mean().sqrt()),
                                learned_rms=float((t2g - t2a).pow(2).mean().sqrt()))
    del t2m, t2g
    out["mp2_guess"] = dict(iterations=ra.iterations, seconds=ra.seconds_total, seconds_guess=ra.seconds_guess,
                            e_corr=ra.e_corr, converged=ra.converged)
    out["learned_guess"] = dict(iterations=rb.iterations, seconds=rb.seconds_total, seconds_guess=rb.seconds_guess,
                                e_corr=rb.e_corr, converged=rb.converged, guess_used=rb.guess_used)
    out["delta_e_corr"] = rb.e_corr - ra.e_corr
    out["max_abs_delta_t2"] = float((t2a - t2b).abs().max())
    out["speedup"] = ra.seconds_total / rb.seconds_total
    if log:
        log(json.dumps(out))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", required=True)
    t.add_argument("--systems", type=int, default=256)
    t.add_argument("--large", type=int, default=0)
    t.add_argument("--per-system", type=int, default=8192)
    t.add_argument("--epochs", type=int, default=30)
    t.add_argument("--batch", type=int, default=4096)
    t.add_argument("--lr", type=float, default=5e-4)
    t.add_argument("--evaluate", default="")
    e = sub.add_parser("evaluate")
    e.add_argument("--model", required=True)
    e.add_argument("--config", default="c5")
    e.add_argument("--precision", default="fp64")
    e.add_argument("--polish", type=float, default=0.0)
    e.add_argument("--polish-precision", default="fp64")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    from . import mlp
    from .synthetic import training_shapes
    if args.cmd == "train":
        shapes = training_shapes(args.systems, large=args.large)
        log(f"[guess] building dataset from {len(shapes)} systems")
        X, Y, info = build_dataset(shapes, args.per_system, seed=12345, log=log)
        log(f"[guess] {X.shape[0]} samples from {info['systems']} systems in {info['seconds']:.1f} s")
        t0 = time.perf_counter()
        net, hist = train(X, Y, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
        t_train = time.perf_counter() - t0
        net.save(args.out)
        res = dict(samples=int(X.shape[0]), dataset=info, train_seconds=t_train, heldout_loss_first=hist[0],
                   heldout_loss_final=hist[-1], out=args.out)
        if args.evaluate:
            res["evaluation"] = evaluate(net, args.evaluate, log=log)
        print(json.dumps(res), flush=True)
    else:
        net = mlp.Net.load(args.model)
        print(json.dumps(evaluate(net, args.config, precision=args.precision, log=log, polish_residual=args.polish,
                                  polish_precision=args.polish_precision)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
