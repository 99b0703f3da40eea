"""GPU RI-CCSD driver (through the C ABI) against the CPU oracle.

Residual/energy/MP2 tolerance: max|d| / max|ref| <= 1e-11 (FP64 both sides,
different summation order).  Converged-solution tolerance: |dE| <= 1e-10 Eh and
max|dt2| <= 1e-9 (both solvers stop at ||Omega||_inf <= 1e-10)."""
import numpy as np
import pytest

from gpu_util import dev, host, rel_max
from oracle import ccsd as oc
from paper_1810_08142_amd.synthetic import CONFIGS, draw_matrix, draw_pair_symmetric, draw_system

pytestmark = pytest.mark.gpu


def _cc():
    from paper_1810_08142_amd import ccsd
    return ccsd


SHAPES = [(1, 4, 5, 800), (2, 5, 7, 801), (3, 17, 20, 802), (4, 24, 96, 803), (5, 37, 41, 804)]


@pytest.mark.parametrize("o,v,naux,seed", SHAPES)
def test_mp2_and_energy(o, v, naux, seed):
    print(f"mp2 o={o} v={v} naux={naux}", flush=True)
    s = draw_system(o, v, naux, seed=seed)
    B, eps = dev(s.B), dev(s.eps)
    t2, e = _cc().mp2_guess(B, eps, o)
    _, t2r, er = oc.mp2(s.B, s.eps, o)
    assert rel_max(host(t2), t2r) <= 1e-12
    assert abs(e - er) <= 1e-12 * abs(er)
    t1 = draw_matrix((o, v), seed + 1, 0.01)
    e2 = _cc().energy(B, eps, o, dev(t1), t2)
    assert abs(e2 - oc.energy(s.B, o, t1, t2r)) <= 1e-12 * abs(er)


@pytest.mark.parametrize("o,v,naux,seed", SHAPES)
def test_residual_parity(o, v, naux, seed):
    print(f"residual o={o} v={v} naux={naux}", flush=True)
    s = draw_system(o, v, naux, seed=seed, scale=0.2)
    t1 = draw_matrix((o, v), seed + 2, 0.05)
    t2 = draw_pair_symmetric(o, v, seed + 3, 0.05)
    om1, om2 = _cc().residual(dev(s.B), dev(s.eps), o, dev(t1), dev(t2))
    r1, r2 = oc.residual(s.B, s.eps, o, t1, t2)
    assert rel_max(host(om1), r1) <= 1e-11
    assert rel_max(host(om2), r2) <= 1e-11


def test_residual_at_zero_is_mp2_numerator():
    o, v, naux = 3, 11, 13
    s = draw_system(o, v, naux, seed=810)
    z1, z2 = np.zeros((o, v)), np.zeros((o, o, v, v))
    om1, om2 = _cc().residual(dev(s.B), dev(s.eps), o, dev(z1), dev(z2))
    K = oc.ovov(s.B, o)
    assert np.abs(host(om1)).max() <= 1e-15
    assert rel_max(host(om2), K.transpose(0, 2, 1, 3)) <= 1e-13


def test_c1_converged_solution():
    c = CONFIGS["c1"]
    o, v, naux = c["o"], c["v"], c["naux"]
    s = draw_system(o, v, naux, seed=c["seed"])
    t1, t2, rep = _cc().solve(dev(s.B), dev(s.eps), o, max_iter=100, tol=1e-10, tol_energy=1e-10)
    ref = oc.solve(s.B, s.eps, o, max_iter=100, tol=1e-10, tol_energy=1e-10)
    print("gpu", rep, "cpu", ref.e_corr, ref.iterations, flush=True)
    assert rep.converged and ref.converged
    assert abs(rep.e_corr - ref.e_corr) <= 1e-10
    assert np.abs(host(t2) - ref.t2).max() <= 1e-9
    assert np.abs(host(t1) - ref.t1).max() <= 1e-9
    assert abs(rep.e_mp2 - ref.e_mp2) <= 1e-12
    assert rep.iterations == ref.iterations


def test_solver_variants_same_fixed_point():
    o, v, naux = 3, 20, 40
    s = draw_system(o, v, naux, seed=820)
    B, eps = dev(s.B), dev(s.eps)
    _, _, r6 = _cc().solve(B, eps, o, diis_size=6, tol=1e-11, tol_energy=1e-12)
    _, _, r3 = _cc().solve(B, eps, o, diis_size=3, tol=1e-11, tol_energy=1e-12)
    _, _, rj = _cc().solve(B, eps, o, diis_size=0, max_iter=400, tol=1e-11, tol_energy=1e-12)
    assert r6.converged and r3.converged and rj.converged
    assert abs(r6.e_corr - r3.e_corr) <= 1e-10 and abs(r6.e_corr - rj.e_corr) <= 1e-10


def test_resume_and_iteration_limit():
    o, v, naux = 3, 20, 40
    s = draw_system(o, v, naux, seed=830)
    B, eps = dev(s.B), dev(s.eps)
    _, _, full = _cc().solve(B, eps, o, tol=1e-10, tol_energy=1e-11)
    t1, t2, part = _cc().solve(B, eps, o, max_iter=4)
    assert part.status == 5 and not part.converged and np.isfinite(host(t2)).all()
    t1, t2, rest = _cc().solve(B, eps, o, t1=t1, t2=t2, tol=1e-10, tol_energy=1e-11)
    assert rest.converged
    assert abs(rest.e_corr - full.e_corr) <= 1e-10
    # starting from the solution converges at once
    _, _, again = _cc().solve(B, eps, o, t1=t1, t2=t2, tol=1e-10, tol_energy=1e-11)
    assert again.converged and again.iterations <= 2


def test_numeric_failure_is_reported():
    from paper_1810_08142_amd import _lib
    o, v, naux = 2, 8, 9
    s = draw_system(o, v, naux, seed=840)
    t2 = np.zeros((o, o, v, v))
    t2[0, 1, 2, 3] = t2[1, 0, 3, 2] = np.nan
    with pytest.raises(_lib.RIError) as e:
        _cc().solve(dev(s.B), dev(s.eps), o, t1=dev(np.zeros((o, v))), t2=dev(t2))
    assert e.value.status == 6


def test_report_rms_matches_final_residual():
    import torch
    o, v, naux = 3, 20, 40
    s = draw_system(o, v, naux, seed=850)
    B, eps = dev(s.B), dev(s.eps)
    t1, t2, rep = _cc().solve(B, eps, o, tol=1e-9, tol_energy=1e-10)
    assert rep.converged and np.isfinite(rep.seconds_guess) and 0 < rep.seconds_guess <= rep.seconds_total
    om1, om2 = _cc().residual(B, eps, o, t1, t2)
    om = torch.cat([om1.reshape(-1), om2.reshape(-1)])
    # the last residual of a converged run is the residual of the returned amplitudes
    assert float(om.abs().max()) == rep.residual_inf
    assert abs(float(om.pow(2).mean().sqrt()) - rep.residual_rms) <= 1e-12 * rep.residual_rms
    assert rep.residual_inf_fp64 == rep.residual_inf and rep.polish_iteration == -1


def test_mixed_ladder_with_fp64_polish_reaches_fp64_fixed_point():
    c = CONFIGS["c1"]
    o = c["o"]
    s = draw_system(o, c["v"], c["naux"], seed=c["seed"])
    B, eps = dev(s.B), dev(s.eps)
    _, t2a, r64 = _cc().solve(B, eps, o, tol=1e-10, tol_energy=1e-10)
    _, t2b, rp = _cc().solve(B, eps, o, ppl_precision="bf16x3", polish_residual=1e-6, tol=1e-10, tol_energy=1e-10)
    print("fp64", r64, "polished", rp, flush=True)
    assert rp.converged and rp.polish_iteration > 0
    assert rp.residual_inf_fp64 == rp.residual_inf <= 1e-10
    assert abs(rp.e_corr - r64.e_corr) <= 1e-10
    assert float((t2a - t2b).abs().max()) <= 1e-9
    # without polish the FP64 residual of the mixed fixed point is evaluated on request
    _, _, rm = _cc().solve(B, eps, o, ppl_precision="bf16x3", tol=1e-8, tol_energy=1e-9, check_fp64=True)
    assert rm.converged and rm.polish_iteration == -1
    assert np.isfinite(rm.residual_inf_fp64) and rm.residual_inf_fp64 <= 1e-6
    assert abs(rm.e_corr - r64.e_corr) <= 1e-6


def test_learned_guess_option_matches_guess_then_user_start():
    from paper_1810_08142_amd import mlp
    o, v, naux = 3, 20, 40
    s = draw_system(o, v, naux, seed=860)
    B, eps = dev(s.B), dev(s.eps)
    net = mlp.Net()
    net.set_params(mlp.init_params(8, 256, 2, seed=5))
    net.set_scaling(np.zeros(8), np.ones(8), 1e-4)
    g1, g2 = net.guess(B, eps, o)
    _, ta, ra = _cc().solve(B, eps, o, t1=g1, t2=g2, tol=1e-10, tol_energy=1e-11)
    _, tb, rb = _cc().solve(B, eps, o, mlp=net, tol=1e-10, tol_energy=1e-11)
    assert ra.converged and rb.converged and ra.iterations == rb.iterations
    assert ra.e_corr == rb.e_corr and bool((ta == tb).all())
    assert np.isnan(rb.e_mp2)


@pytest.mark.parametrize("o,v,naux,seed", [(3, 32, 40, 870), (5, 48, 37, 871), (2, 64, 64, 872)])
def test_residual_parity_large_tile_contractions(o, v, naux, seed, monkeypatch):
    """v a multiple of 16 with the large-tile threshold lowered to one tile, so every
    contraction whose innermost summed extent allows it runs on the 128 x 128 kernel."""
    monkeypatch.setenv("RI_GEMM_LARGE_MIN_TILES", "1")
    s = draw_system(o, v, naux, seed=seed, scale=0.2)
    t1 = draw_matrix((o, v), seed + 2, 0.05)
    t2 = draw_pair_symmetric(o, v, seed + 3, 0.05)
    om1, om2 = _cc().residual(dev(s.B), dev(s.eps), o, dev(t1), dev(t2))
    r1, r2 = oc.residual(s.B, s.eps, o, t1, t2)
    assert rel_max(host(om1), r1) <= 1e-11
    assert rel_max(host(om2), r2) <= 1e-11


def test_mixed_ladder_with_fp32_polish():
    c = CONFIGS["c1"]
    o = c["o"]
    s = draw_system(o, c["v"], c["naux"], seed=c["seed"])
    B, eps = dev(s.B), dev(s.eps)
    _, _, r64 = _cc().solve(B, eps, o, tol=1e-10, tol_energy=1e-10)
    _, _, rp = _cc().solve(B, eps, o, ppl_precision="bf16x3", polish_residual=1e-6, polish_precision="fp32",
                           tol=1e-9, tol_energy=1e-10, check_fp64=True)
    print("fp64", r64, "fp32-polished", rp, flush=True)
    assert rp.converged and rp.polish_iteration > 0
    # converged on an FP32-ladder residual; the FP64 residual of the result is evaluated
    assert np.isfinite(rp.residual_inf_fp64) and rp.residual_inf_fp64 <= 1e-7
    assert abs(rp.e_corr - r64.e_corr) <= 1e-8


def test_fp32_other_contractions_and_fp64_polish(monkeypatch):
    """The large non-ladder contractions in FP32 (forced onto the large-tile kernel at
    this size) stay within 1e-7 Eh of FP64; an FP64 polish returns to the FP64
    fixed point."""
    monkeypatch.setenv("RI_GEMM_LARGE_MIN_TILES", "1")
    o, v, naux = 3, 32, 40
    s = draw_system(o, v, naux, seed=880)
    B, eps = dev(s.B), dev(s.eps)
    _, _, r64 = _cc().solve(B, eps, o, tol=1e-10, tol_energy=1e-10)
    _, _, r32 = _cc().solve(B, eps, o, other_precision="fp32", tol=1e-8, tol_energy=1e-9, check_fp64=True)
    print("fp64", r64, "fp32 others", r32, flush=True)
    assert r32.converged and abs(r32.e_corr - r64.e_corr) <= 1e-7
    assert np.isfinite(r32.residual_inf_fp64) and r32.residual_inf_fp64 <= 1e-6
    _, _, rp = _cc().solve(B, eps, o, other_precision="fp32", polish_residual=1e-6, tol=1e-10, tol_energy=1e-10)
    assert rp.converged and rp.polish_iteration > 0
    assert rp.residual_inf_fp64 == rp.residual_inf <= 1e-10
    assert abs(rp.e_corr - r64.e_corr) <= 1e-10


def test_learned_guess_falls_back_to_mp2():
    from paper_1810_08142_amd import mlp
    o, v, naux = 3, 20, 40
    s = draw_system(o, v, naux, seed=890)
    B, eps = dev(s.B), dev(s.eps)
    _, _, r0 = _cc().solve(B, eps, o, tol=1e-10, tol_energy=1e-11)
    net = mlp.Net()
    theta = mlp.init_params(8, 256, 2, seed=6)
    theta[-1] = np.nan  # a broken network: every amplitude becomes NaN
    net.set_params(theta)
    net.set_scaling(np.zeros(8), np.ones(8), 1.0)
    _, _, r = _cc().solve(B, eps, o, mlp=net, tol=1e-10, tol_energy=1e-11)
    assert r.guess_used == 0 and r.converged
    assert r.e_corr == r0.e_corr and r.iterations == r0.iterations
    assert r0.guess_used == 0
    good = mlp.Net()
    good.set_params(mlp.init_params(8, 256, 2, seed=5))
    good.set_scaling(np.zeros(8), np.ones(8), 1e-4)
    _, _, r2 = _cc().solve(B, eps, o, mlp=good, tol=1e-10, tol_energy=1e-11)
    assert r2.guess_used == 2 and r2.converged
