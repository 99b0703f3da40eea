"""Reduced-precision ladders on the GPU: split-bf16 (three products) and plain FP32
operands, both on MFMA with FP32 accumulation.

Error model: a split operand x = hi + lo is exact to 2^-18 |x|, and dropping lo*lo
adds another 2^-18 |a||b|, so one split product is within 3 * 2^-18 |a||b|; an FP32
operand is exact to 2^-24 |x|.  The build and the contraction each round their
operands once and accumulate in FP32, hence, element by element,

    |R_mixed - R_fp64| <= eps * sum_cd sum_Q |B_ac| |B_bd| |tau^{cd}_{ij}|  = eps * L(|B|, |tau|)

with eps = 2e-4 (two rounding stages, FP32 accumulation over up to ~1e4 terms).  The
right-hand side is the oracle's ladder of the element-wise absolute values."""
import os

import numpy as np
import pytest

from gpu_util import dev, host
from oracle import ccsd as oc
from oracle import native
from paper_1810_08142_amd.synthetic import CONFIGS, draw_matrix, draw_pair_symmetric, draw_system

pytestmark = pytest.mark.gpu
EPS = 2e-4


def _ladder(B_vv, tau, precision="bf16x3"):
    import torch
    from paper_1810_08142_amd import ppl
    o, v = tau.shape[0], tau.shape[2]
    R = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    ppl.ppl(dev(B_vv), dev(tau), R, precision=precision)
    return host(R)


PRECS = ["bf16x3", "fp32"]


# (16, 37, 29): the tau- contraction (120 pairs) takes the 256 x 128 tiles, tau+ (136) the
# row strips; (48, 40, 24): tau+ (1176 pairs) the 256 x 256 and tau- (1128) the 256 x 192
# tiles, as at o=48 v=768 naux=2304
@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("o,v,naux", [(1, 3, 2), (2, 17, 7), (3, 33, 20), (4, 24, 96), (5, 40, 37), (2, 50, 130),
                                      (16, 37, 29), (48, 40, 24)])
def test_mixed_within_split_error_bound(o, v, naux, precision):
    print(f"{precision} o={o} v={v} naux={naux}", flush=True)
    s = draw_system(o, v, naux, seed=900 + v)
    tau = draw_pair_symmetric(o, v, 901 + v)
    got = _ladder(s.B_vv, tau, precision)
    ref = native.ppl(s.B_vv, tau)
    bound = EPS * native.ppl(np.abs(s.B_vv), np.abs(tau))
    err = np.abs(got - ref)
    print("max rel err", float(err.max() / np.abs(ref).max()), "max err/bound", float((err / bound).max()))
    assert bool(np.all(err <= bound))
    # and it is not accidentally the FP64 result: the split error is visible
    assert float(err.max()) > 0.0


@pytest.mark.parametrize("precision", PRECS)
def test_mixed_nonsymmetric_factors_and_symmetry(precision):
    o, v, naux = 3, 29, 17
    s = draw_system(o, v, naux, seed=911, scale=0.2)
    t1 = draw_matrix((o, v), 912, 0.1)
    Bd = np.ascontiguousarray(oc.dress(s.B, t1)[:, o:, o:])
    tau = draw_pair_symmetric(o, v, 913)
    got = _ladder(Bd, tau, precision)
    ref = native.ppl(Bd, tau)
    assert bool(np.all(np.abs(got - ref) <= EPS * native.ppl(np.abs(Bd), np.abs(tau))))
    # exact pair symmetry needs (ac|bd) - (ad|bc) to vanish exactly at a == b
    assert np.array_equal(got, got.transpose(1, 0, 3, 2))
    assert np.array_equal(got, _ladder(Bd, tau, precision))


def test_fp32_operands_are_more_accurate_than_split_bf16():
    o, v, naux = 4, 40, 60
    s = draw_system(o, v, naux, seed=915)
    tau = draw_pair_symmetric(o, v, 916)
    ref = native.ppl(s.B_vv, tau)
    e32 = np.abs(_ladder(s.B_vv, tau, "fp32") - ref).max()
    e16 = np.abs(_ladder(s.B_vv, tau, "bf16x3") - ref).max()
    print("max error fp32", e32, "bf16x3", e16, flush=True)
    assert 0.0 < e32 < e16


@pytest.mark.parametrize("precision", PRECS)
def test_mixed_slabs_do_not_change_result(precision):
    o, v, naux = 3, 70, 18
    s = draw_system(o, v, naux, seed=921)
    tau = draw_pair_symmetric(o, v, 922)
    R1 = _ladder(s.B_vv, tau, precision)
    os.environ["RI_PPL_SLAB_PAIRS"] = "3"
    try:
        R2 = _ladder(s.B_vv, tau, precision)
    finally:
        del os.environ["RI_PPL_SLAB_PAIRS"]
    assert np.array_equal(R1, R2)


@pytest.mark.parametrize("precision", PRECS)
def test_ccsd_with_mixed_ladder_energy_within_microhartree(precision):
    from paper_1810_08142_amd import ccsd
    c = CONFIGS["c1"]
    o, v, naux = c["o"], c["v"], c["naux"]
    s = draw_system(o, v, naux, seed=c["seed"])
    B, eps = dev(s.B), dev(s.eps)
    _, _, r64 = ccsd.solve(B, eps, o)
    _, _, rmx = ccsd.solve(B, eps, o, ppl_precision=precision, tol=1e-8, tol_energy=1e-9)
    print("E fp64", r64.e_corr, f"E {precision}", rmx.e_corr, "diff", rmx.e_corr - r64.e_corr, flush=True)
    assert r64.converged and rmx.converged
    assert abs(rmx.e_corr - r64.e_corr) <= 1e-6


def _bf16_rne(x32):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    u = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _split(x):
    """x = hi + lo: hi = bf16(fp32(x)), lo = bf16(fp32(x - hi))."""
    hi = _bf16_rne(np.asarray(x, dtype=np.float64).astype(np.float32))
    lo = _bf16_rne((np.asarray(x, dtype=np.float64) - hi).astype(np.float32))
    return hi, lo


def _split_ladder_emulated(B_vv, tau):
    """The split-bf16 ladder's arithmetic on the host: operands split once, products
    hi*lo + lo*hi + hi*hi (exact in FP64), integrals rounded to FP32 and split again for
    the contraction, S and A rounded to FP32.  Only the FP32 accumulation order of the
    device differs."""
    o, v = tau.shape[0], tau.shape[2]
    Bh, Bl = _split(B_vv)
    prod = lambda x, y: (np.einsum("Qac,Qbd->abcd", x[0], y[1]) + np.einsum("Qac,Qbd->abcd", x[1], y[0])
                         + np.einsum("Qac,Qbd->abcd", x[0], y[0]))
    v1 = prod((Bh, Bl), (Bh, Bl)).astype(np.float32)          # (ac|bd)[a, b, c, d]
    v2 = v1.transpose(0, 1, 3, 2)                             # (ad|bc)
    Wp = _split((v1 + v2).astype(np.float32))
    Wm = _split((v1 - v2).astype(np.float32))
    tp = 0.5 * (tau + tau.transpose(0, 1, 3, 2))  # (tau^{cd} + tau^{dc}) / 2 (tau is pair-symmetric)
    tm = 0.5 * (tau - tau.transpose(0, 1, 3, 2))
    iu = np.triu_indices(v)
    sig = np.where(iu[0] == iu[1], 0.5, 1.0)
    Tp = _split(tp[:, :, iu[0], iu[1]] * sig)
    iu1 = np.triu_indices(v, 1)
    Tm = _split(tm[:, :, iu1[0], iu1[1]])
    c3 = lambda W, T, idx: (np.einsum("abk,ijk->ijab", W[0][:, :, idx[0], idx[1]], T[1])
                            + np.einsum("abk,ijk->ijab", W[1][:, :, idx[0], idx[1]], T[0])
                            + np.einsum("abk,ijk->ijab", W[0][:, :, idx[0], idx[1]], T[0]))
    S = c3(Wp, Tp, iu).astype(np.float32).astype(np.float64)
    A = c3(Wm, Tm, iu1).astype(np.float32).astype(np.float64)
    return S + A


def test_split_emulation_reproduces_the_device_result():
    o, v, naux = 2, 20, 40
    s = draw_system(o, v, naux, seed=971)
    tau = draw_pair_symmetric(o, v, 972)
    got = _ladder(s.B_vv, tau, "bf16x3")
    emu = _split_ladder_emulated(s.B_vv, tau)
    ref = native.ppl(s.B_vv, tau)
    scale = native.ppl(np.abs(s.B_vv), np.abs(tau))
    d_emu = np.abs(got - emu)
    d_ref = np.abs(got - ref)
    print("device vs emulation", float(d_emu.max()), "device vs FP64", float(d_ref.max()), flush=True)
    # the device differs from the emulation only by FP32 accumulation order ...
    assert bool(np.all(d_emu <= 1e-6 * scale))
    # ... which is far below the split error it shares with the emulation
    assert float(d_emu.max()) < 0.1 * float(d_ref.max())
