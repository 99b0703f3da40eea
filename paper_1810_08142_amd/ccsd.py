"""Closed-shell RI-CCSD through the C ABI (Sec. II.A): MP2 guess, residual, energy
and the Jacobi + DIIS solver.  Argument marshalling only; the work runs in the
library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib
from .ppl import _need, _prec, _stream


def _system(B: torch.Tensor, eps: torch.Tensor, o: int) -> _lib.RISystem:
    naux, n = B.shape[0], B.shape[1]
    _need(B, "B", (naux, n, n))
    _need(eps, "eps", (n,))
    if not 0 < o < n:
        raise ValueError("need 0 < o < n")
    return _lib.RISystem(o, n - o, naux, B.data_ptr(), eps.data_ptr())


def mp2_guess(B: torch.Tensor, eps: torch.Tensor, o: int, stream=None):
    """(t2, E_MP2) with t2[i][j][a][b] = (ia|jb) / D (t1 = 0)."""
    sy = _system(B, eps, o)
    v = sy.v
    t1 = torch.empty((o, v), dtype=torch.float64, device=B.device)
    t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=B.device)
    e = ctypes.c_double()
    _lib.check(_lib.lib().ri_mp2_guess(ctypes.byref(sy), t1.data_ptr(), t2.data_ptr(), ctypes.byref(e),
                                       _stream(stream)), "ri_mp2_guess")
    return t2, e.value


def energy(B, eps, o, t1, t2, stream=None) -> float:
    sy = _system(B, eps, o)
    _need(t1, "t1", (o, sy.v))
    _need(t2, "t2", (o, o, sy.v, sy.v))
    e = ctypes.c_double()
    _lib.check(_lib.lib().ri_ccsd_energy(ctypes.byref(sy), t1.data_ptr(), t2.data_ptr(), ctypes.byref(e),
                                         _stream(stream)), "ri_ccsd_energy")
    return e.value


def triples(B, eps, o, t1, t2, precision="fp64", stream=None) -> float:
    """Perturbative triples energy E_(T) of CCSD(T) at the amplitudes (ri_ccsd_triples_ex);
    precision "fp64" or "fp32" (the term GEMMs)."""
    sy = _system(B, eps, o)
    _need(t1, "t1", (o, sy.v))
    _need(t2, "t2", (o, o, sy.v, sy.v))
    e = ctypes.c_double()
    _lib.check(_lib.lib().ri_ccsd_triples_ex(ctypes.byref(sy), t1.data_ptr(), t2.data_ptr(), _prec(precision),
                                             ctypes.byref(e), _stream(stream)), "ri_ccsd_triples")
    return e.value


def triples_flops(o: int, v: int) -> float:
    return float(_lib.lib().ri_ccsd_triples_flops(o, v))


def residual(B, eps, o, t1, t2, ppl_precision="fp64", stream=None):
    """(Omega1 [o][v], Omega2 [o][o][v][v]) at the given amplitudes."""
    sy = _system(B, eps, o)
    v = sy.v
    _need(t1, "t1", (o, v))
    _need(t2, "t2", (o, o, v, v))
    om1 = torch.empty_like(t1)
    om2 = torch.empty_like(t2)
    _lib.check(_lib.lib().ri_ccsd_residual(ctypes.byref(sy), t1.data_ptr(), t2.data_ptr(), om1.data_ptr(),
                                           om2.data_ptr(), _prec(ppl_precision), _stream(stream)),
               "ri_ccsd_residual")
    return om1, om2


@dataclasses.dataclass
class Report:
    e_corr: float
    e_mp2: float
    residual_inf: float
    iterations: int
    converged: bool
    seconds_total: float
    seconds_ppl: float
    status: int
    residual_rms: float = float("nan")
    residual_inf_fp64: float = float("nan")
    polish_iteration: int = -1
    seconds_guess: float = float("nan")
    guess_used: int = 0  # 0 MP2, 1 user amplitudes, 2 learned (falls back to 0)


def solve(B, eps, o, t1=None, t2=None, max_iter=100, tol=1e-10, tol_energy=1e-10, diis_size=6,
          diis_start=2, ppl_precision="fp64", verbose=False, stream=None, raise_on_noconv=False,
          polish_residual=0.0, check_fp64=False, mlp=None, polish_precision="fp64", other_precision="fp64"):
    """Jacobi + DIIS from the MP2 guess, from t1/t2 when given, or from the learned
    guess of `mlp` (a paper_1810_08142_amd.mlp.Net).  With a mixed-precision ladder,
    `polish_residual` > 0 switches the ladder to `polish_precision` (FP64 or FP32) once
    max |Omega| falls below it,
    and `check_fp64` evaluates the FP64 residual of the final amplitudes.
    `other_precision` "fp32" runs the large non-ladder contractions on the FP32 MFMA.
    Returns (t1, t2, Report); t1/t2 passed in are overwritten."""
    sy = _system(B, eps, o)
    v = sy.v
    L = _lib.lib()
    op = _lib.RICcsdOpts()
    L.ri_ccsd_default_opts(ctypes.byref(op))
    op.max_iter, op.tol_residual, op.tol_energy = max_iter, tol, tol_energy
    op.diis_size, op.diis_start, op.ppl_precision = diis_size, diis_start, _prec(ppl_precision)
    op.verbose = 1 if verbose else 0
    op.polish_residual = float(polish_residual)
    op.polish_precision = _prec(polish_precision)
    op.other_precision = _prec(other_precision)
    op.check_fp64 = 1 if check_fp64 else 0
    if mlp is not None and t2 is not None:
        raise ValueError("pass either a network or starting amplitudes, not both")
    if t2 is None:
        op.guess = 2 if mlp is not None else 0
        if mlp is not None:
            op.mlp = mlp.handle
        t1 = torch.empty((o, v), dtype=torch.float64, device=B.device)
        t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=B.device)
    else:
        op.guess = 1
        if t1 is None:
            t1 = torch.zeros((o, v), dtype=torch.float64, device=B.device)
        _need(t1, "t1", (o, v))
        _need(t2, "t2", (o, o, v, v))
    rep = _lib.RICcsdReport()
    rc = L.ri_ccsd_iterate(ctypes.byref(sy), t1.data_ptr(), t2.data_ptr(), ctypes.byref(op), ctypes.byref(rep),
                           _stream(stream))
    if rc not in (0, 5) or (rc == 5 and raise_on_noconv):
        _lib.check(rc, "ri_ccsd_iterate")
    r = Report(rep.e_corr, rep.e_mp2, rep.residual_inf, rep.iterations, bool(rep.converged), rep.seconds_total,
               rep.seconds_ppl, rc, rep.residual_rms, rep.residual_inf_fp64, rep.polish_iteration,
               rep.seconds_guess, rep.guess_used)
    return t1, t2, r
