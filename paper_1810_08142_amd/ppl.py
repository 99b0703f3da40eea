"""Particle-particle ladder through the C ABI (Sec. II.C, eq. pp-Ladder-0).

Thin wrappers: check tensor shapes, dtypes and devices, then pass raw device
pointers and the current HIP stream to ``libriccsd.so``.  All arithmetic runs
in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib

FP64, FP32, BF16X3 = 0, 1, 2
_PREC = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}


def _prec(p) -> int:
    return _PREC[p] if isinstance(p, str) else int(p)


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _need(t: torch.Tensor, name: str, shape, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def ppl(B_vv: torch.Tensor, tau: torch.Tensor, R: torch.Tensor, precision="fp64",
        workspace: torch.Tensor | None = None, stream=None, shard=None) -> torch.Tensor:
    """R += sum_cd (ac|bd) tau^{cd}_{ij}; B_vv [naux][v][v], tau and R [o][o][v][v].
    ``shard=(k, n)`` adds only shard k of n of the (ab) slabs (ri_ppl_shard)."""
    naux, v = B_vv.shape[0], B_vv.shape[1]
    o = tau.shape[0]
    _need(B_vv, "B_vv", (naux, v, v))
    _need(tau, "tau", (o, o, v, v))
    _need(R, "R", (o, o, v, v))
    L = _lib.lib()
    if workspace is None:
        ws, nbytes = None, 0
    else:
        if not workspace.is_cuda or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous device tensor")
        ws, nbytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    k, n = (0, 1) if shard is None else shard
    rc = L.ri_ppl_shard(B_vv.data_ptr(), tau.data_ptr(), o, v, naux, R.data_ptr(), _prec(precision),
                        int(k), int(n), ws, nbytes, _stream(stream))
    _lib.check(rc, "ri_ppl")
    return R


def ppl_noalloc(B_vv: torch.Tensor, tau: torch.Tensor, R: torch.Tensor, precision="fp64",
                stream=None) -> torch.Tensor:
    """The ladder of ``ppl`` with the library's fixed scratch array as its workspace
    (ri_ppl_noalloc): the call allocates no device memory.  Sizes whose workspace does
    not fit the array raise with status RI_E_NOMEM."""
    naux, v = B_vv.shape[0], B_vv.shape[1]
    o = tau.shape[0]
    _need(B_vv, "B_vv", (naux, v, v))
    _need(tau, "tau", (o, o, v, v))
    _need(R, "R", (o, o, v, v))
    rc = _lib.lib().ri_ppl_noalloc(B_vv.data_ptr(), tau.data_ptr(), o, v, naux, R.data_ptr(), _prec(precision),
                                   _stream(stream))
    _lib.check(rc, "ri_ppl_noalloc")
    return R


def ppl_paper(B_vv: torch.Tensor, tau: torch.Tensor, R: torch.Tensor, stream=None) -> torch.Tensor:
    """The same sum in the paper's arrangement (full (a, b) build, i <= j pairs only;
    ri_ppl_paper), FP64: the ablation of the tau+- form."""
    naux, v = B_vv.shape[0], B_vv.shape[1]
    o = tau.shape[0]
    _need(B_vv, "B_vv", (naux, v, v))
    _need(tau, "tau", (o, o, v, v))
    _need(R, "R", (o, o, v, v))
    _lib.check(_lib.lib().ri_ppl_paper(B_vv.data_ptr(), tau.data_ptr(), o, v, naux, R.data_ptr(), _stream(stream)),
               "ri_ppl_paper")
    return R


def ppl_sym(B_vv: torch.Tensor, tau: torch.Tensor, R: torch.Tensor, precision="fp64", stream=None) -> torch.Tensor:
    """The same sum for factors symmetric in their two virtual indices, using the
    exchange symmetry of the integral matrix to build about half of it (ri_ppl_sym_ex)."""
    naux, v = B_vv.shape[0], B_vv.shape[1]
    o = tau.shape[0]
    _need(B_vv, "B_vv", (naux, v, v))
    _need(tau, "tau", (o, o, v, v))
    _need(R, "R", (o, o, v, v))
    _lib.check(_lib.lib().ri_ppl_sym_ex(B_vv.data_ptr(), tau.data_ptr(), o, v, naux, R.data_ptr(), _prec(precision),
                                        _stream(stream)), "ri_ppl_sym")
    return R


def sym_flops(o: int, v: int, naux: int) -> float:
    """Algorithmic FLOP of ri_ppl_sym over its slab schedule."""
    return float(_lib.lib().ri_ppl_sym_flops(o, v, naux))


def paper_flops(o: int, v: int, naux: int) -> float:
    """FLOP of ri_ppl_paper: 2 Naux v^4 (full build) + v^4 o(o+1) (i <= j contraction)."""
    return float(_lib.lib().ri_ppl_paper_flops(o, v, naux))


def workspace_bytes(o: int, v: int, naux: int, precision="fp64") -> int:
    return int(_lib.lib().ri_ppl_workspace_bytes(o, v, naux, _prec(precision)))


def flops(o: int, v: int, naux: int) -> float:
    """Algorithmic FLOP of one ladder call as executed (build half + packed contraction)."""
    return float(_lib.lib().ri_ppl_flops(o, v, naux))


def build_tau(t1: torch.Tensor, t2: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """tau = t2 + t1 (x) t1 (eq. pp-Ladder-01)."""
    o, v = t1.shape
    _need(t1, "t1", (o, v))
    _need(t2, "t2", (o, o, v, v))
    if out is None:
        out = torch.empty_like(t2)
    _need(out, "tau", (o, o, v, v))
    _lib.check(_lib.lib().ri_build_tau(t1.data_ptr(), t2.data_ptr(), o, v, out.data_ptr(), _stream(stream)),
               "ri_build_tau")
    return out


def pair_asymmetry(tau: torch.Tensor, stream=None):
    """(max |tau^{cd}_{ij} - tau^{dc}_{ji}|, max |tau|) of tau [o][o][v][v]."""
    o, v = tau.shape[0], tau.shape[2]
    _need(tau, "tau", (o, o, v, v))
    r = (ctypes.c_double * 2)()
    _lib.check(_lib.lib().ri_tau_pair_asymmetry(tau.data_ptr(), o, v, r, _stream(stream)), "ri_tau_pair_asymmetry")
    return r[0], r[1]
