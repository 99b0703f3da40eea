"""Ladder parity on the GPU: the HIP path (through the C ABI) against the CPU oracle.

Tolerance (FP64 path): max|dR| / max|R_ref| <= 1e-11 and ||dR||_F / ||R_ref||_F <= 1e-11
(the config's "within 1e-11 relative"; element-wise relative error is ill-posed
near zeros).  Both sides accumulate sums of v^2 * naux products in FP64 in a
different order; their rounding differs by O(1e-15) relative to the terms."""
import os

import numpy as np
import pytest

from gpu_util import dev, host, rel_fro, rel_max
from oracle import ccsd as oc
from oracle import native
from paper_1810_08142_amd.synthetic import CONFIGS, draw_matrix, draw_pair_symmetric, draw_system

pytestmark = pytest.mark.gpu
TOL = 1e-11


def _ppl():
    from paper_1810_08142_amd import ppl
    return ppl


def _gpu_ladder(B_vv, tau, R0=None, precision="fp64"):
    import torch
    o, v = tau.shape[0], tau.shape[2]
    R = dev(R0) if R0 is not None else torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    _ppl().ppl(dev(B_vv), dev(tau), R, precision=precision)
    return host(R)


SHAPES = [  # (o, v, naux): tiny, one tile, ragged tails across several tiles, the CCSD config
    (1, 3, 2), (1, 16, 16), (2, 17, 7), (3, 33, 20), (4, 24, 96), (5, 40, 37), (2, 50, 130),
]


@pytest.mark.parametrize("o,v,naux", SHAPES)
def test_parity_small(o, v, naux):
    print(f"ppl parity o={o} v={v} naux={naux}", flush=True)
    s = draw_system(o, v, naux, seed=300 + v)
    tau = draw_pair_symmetric(o, v, 400 + v)
    R0 = draw_matrix((o, o, v, v), 500 + v)
    got = _gpu_ladder(s.B_vv, tau, R0)
    ref = native.ppl(s.B_vv, tau, R0.copy())
    assert rel_max(got - R0, ref - R0) <= TOL
    assert rel_fro(got - R0, ref - R0) <= TOL


def test_nonsymmetric_factors():
    # t1-dressed factors are not symmetric in (a, c)
    o, v, naux = 3, 21, 11
    s = draw_system(o, v, naux, seed=601, scale=0.2)
    t1 = draw_matrix((o, v), 602, 0.1)
    Bd = np.ascontiguousarray(oc.dress(s.B, t1)[:, o:, o:])
    assert np.abs(Bd - Bd.transpose(0, 2, 1)).max() > 1e-3
    tau = draw_pair_symmetric(o, v, 603)
    got = _gpu_ladder(Bd, tau)
    ref = native.ppl(Bd, tau)
    assert rel_max(got, ref) <= TOL


def test_uses_pair_symmetric_part_of_tau():
    o, v, naux = 3, 19, 9
    s = draw_system(o, v, naux, seed=611)
    x = draw_matrix((o, o, v, v), 612)
    got = _gpu_ladder(s.B_vv, x)
    ref = native.ppl(s.B_vv, 0.5 * (x + x.transpose(1, 0, 3, 2)))
    assert rel_max(got, ref) <= TOL


def test_pair_symmetry_bitwise_and_deterministic():
    o, v, naux = 4, 37, 25
    s = draw_system(o, v, naux, seed=621)
    tau = draw_pair_symmetric(o, v, 622)
    R1 = _gpu_ladder(s.B_vv, tau)
    R2 = _gpu_ladder(s.B_vv, tau)
    assert np.array_equal(R1, R2)
    assert np.array_equal(R1, R1.transpose(1, 0, 3, 2))


def test_slabs_do_not_change_result():
    o, v, naux = 3, 70, 18
    s = draw_system(o, v, naux, seed=631)
    tau = draw_pair_symmetric(o, v, 632)
    R1 = _gpu_ladder(s.B_vv, tau)
    os.environ["RI_PPL_SLAB_PAIRS"] = "2"
    try:
        R2 = _gpu_ladder(s.B_vv, tau)
    finally:
        del os.environ["RI_PPL_SLAB_PAIRS"]
    assert np.array_equal(R1, R2)


def test_caller_workspace_and_errors():
    import torch
    from paper_1810_08142_amd import _lib
    ppl = _ppl()
    o, v, naux = 2, 20, 8
    s = draw_system(o, v, naux, seed=641)
    tau = draw_pair_symmetric(o, v, 642)
    nbytes = ppl.workspace_bytes(o, v, naux)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    R = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    ppl.ppl(dev(s.B_vv), dev(tau), R, workspace=ws)
    assert rel_max(host(R), native.ppl(s.B_vv, tau)) <= TOL
    small = torch.empty(nbytes // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.RIError) as e:
        ppl.ppl(dev(s.B_vv), dev(tau), R, workspace=small)
    assert e.value.status == 3
    T = dev(tau)
    with pytest.raises(_lib.RIError) as e:
        ppl.ppl(dev(s.B_vv), T, T)  # R aliases tau
    assert e.value.status == 2


def test_build_tau():
    o, v = 3, 11
    t1 = draw_matrix((o, v), 651, 0.1)
    t2 = draw_pair_symmetric(o, v, 652)
    got = host(_ppl().build_tau(dev(t1), dev(t2)))
    ref = oc.make_tau(t1, t2)
    # one rounding of a fused multiply-add vs two roundings on the host
    bound = 2.0 * np.finfo(np.float64).eps * (np.abs(t2) + np.abs(np.einsum("ia,jb->ijab", t1, t1)))
    assert bool(np.all(np.abs(got - ref) <= bound))


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_c4_full_size_sampled_fp64_and_mixed():
    """c4 (o=48, v=768, naux=2304: B_vv, tau and R 10.9 GB each) through both ladder
    precisions in one pass of the inputs; tau is the oracle's MP2 t2 + t1 (x) t1.
    The oracle recomputes 64 sampled (a, b) pairs for all (i, j): FP64 to 1e-11,
    split-bf16 within eps * L(|B|, |tau|) (eps = 2e-4, the split error model)."""
    import torch
    c = CONFIGS["c4"]
    o, v, naux = c["o"], c["v"], c["naux"]
    print("c4: drawing system", flush=True)
    s = draw_system(o, v, naux, seed=c["seed"])
    print("c4: oracle MP2 amplitudes", flush=True)
    _, t2, _ = oc.mp2(s.B, s.eps, o)
    tau = oc.make_tau(s.t1, t2)
    del t2
    B_vv = s.B_vv
    del s
    rng = np.random.default_rng(44)
    pairs = [(int(a), int(b)) for a, b in rng.integers(0, v, size=(60, 2))] + [(0, 0), (v - 1, v - 1), (0, v - 1), (v - 1, 0)]
    a_idx = torch.tensor([p[0] for p in pairs], device="cuda")
    b_idx = torch.tensor([p[1] for p in pairs], device="cuda")
    Bd, Td = dev(B_vv), dev(tau)
    got = {}
    for prec in ("fp64", "bf16x3"):
        print(f"c4: GPU ladder {prec}", flush=True)
        R = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
        _ppl().ppl(Bd, Td, R, precision=prec)
        got[prec] = R[:, :, a_idx, b_idx].permute(2, 0, 1).cpu().numpy()
        mirror = R[:, :, b_idx, a_idx].permute(2, 1, 0).cpu().numpy()
        assert np.array_equal(got[prec], mirror)  # R^{ab}_{ij} = R^{ba}_{ji}, bitwise
        assert np.isfinite(got[prec]).all()
        del R
    del Bd, Td
    print("c4: oracle sample", flush=True)
    ref = native.ppl_pairs(B_vv, tau, pairs)
    assert np.abs(got["fp64"] - ref).max() / np.abs(ref).max() <= TOL
    assert np.linalg.norm(got["fp64"] - ref) / np.linalg.norm(ref) <= TOL
    print("c4: oracle bound sample", flush=True)
    bound = 2e-4 * native.ppl_pairs(np.abs(B_vv), np.abs(tau), pairs)
    err = np.abs(got["bf16x3"] - ref)
    print("c4 bf16x3 max rel err", float(err.max() / np.abs(ref).max()), flush=True)
    assert bool(np.all(err <= bound))


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_shards_add_up_to_the_whole_call(precision, monkeypatch):
    """Shards k of n of the (ab) slabs together add bitwise what one call adds."""
    import torch
    monkeypatch.setenv("RI_PPL_SLAB_PAIRS", "2")
    o, v, naux = 3, 70, 18  # 15 block pairs -> 8 slabs of at most 2
    s = draw_system(o, v, naux, seed=941)
    tau = draw_pair_symmetric(o, v, 942)
    B, T = dev(s.B_vv), dev(tau)
    full = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    _ppl().ppl(B, T, full, precision=precision)
    total = torch.zeros_like(full)
    for k in range(3):
        part = torch.zeros_like(full)
        _ppl().ppl(B, T, part, precision=precision, shard=(k, 3))
        assert float(part.abs().max()) > 0.0
        # shards touch disjoint entries
        assert not bool(((total != 0) & (part != 0)).any())
        total += part
    assert bool((total == full).all())
    from paper_1810_08142_amd import _lib
    with pytest.raises(_lib.RIError):
        _ppl().ppl(B, T, full, precision=precision, shard=(3, 3))


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_power_of_two_scaling_is_bitwise(precision):
    """R(2^k B, 2^m tau) = 2^(2k+m) R(B, tau) exactly: power-of-two scaling commutes
    with every rounding step, the bf16 hi/lo split included (no under/overflow here)."""
    import torch
    o, v, naux = 3, 37, 29
    s = draw_system(o, v, naux, seed=961)
    tau = draw_pair_symmetric(o, v, 962)
    R1 = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    R2 = torch.zeros_like(R1)
    _ppl().ppl(dev(s.B_vv), dev(tau), R1, precision=precision)
    _ppl().ppl(dev(s.B_vv * 4.0), dev(tau * 0.5), R2, precision=precision)  # 2^(2*2 - 1) = 8
    assert bool((R2 == 8.0 * R1).all())


def test_pair_asymmetry_measure_and_debug_check(monkeypatch):
    """ri_tau_pair_asymmetry returns max |tau_ij^cd - tau_ji^dc| and max |tau|
    exactly; with RI_PPL_CHECK_TAU set the ladder rejects a tau that is not
    pair-symmetric and leaves R untouched."""
    import torch
    from paper_1810_08142_amd import _lib, ppl
    o, v, naux = 3, 21, 10
    s = draw_system(o, v, naux, seed=8)
    T = draw_pair_symmetric(o, v, 31, 0.01)
    assert ppl.pair_asymmetry(dev(T)) == (0.0, float(np.abs(T).max()))
    bad = T.copy()
    bad[2, 0, 5, 17] += 3e-4
    ref = np.abs(bad - bad.transpose(1, 0, 3, 2)).max()
    asym, amax = ppl.pair_asymmetry(dev(bad))
    assert asym == ref and amax == np.abs(bad).max()
    nan = T.copy()
    nan[1, 1, 3, 3] = np.nan
    assert np.isnan(ppl.pair_asymmetry(dev(nan))[0])
    B = dev(np.ascontiguousarray(s.B_vv))
    monkeypatch.setenv("RI_PPL_CHECK_TAU", "1")
    R = torch.full((o, o, v, v), 0.5, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.RIError) as ei:
        ppl.ppl(B, dev(bad), R)
    assert ei.value.status == 1 and "pair-symmetric" in str(ei.value)
    assert bool((R == 0.5).all())
    ppl.ppl(B, dev(T), R)  # a symmetric tau passes the check
    monkeypatch.setenv("RI_PPL_CHECK_TAU", "0")
    ppl.ppl(B, dev(bad), R)  # check off: the symmetric part is used
    torch.cuda.synchronize()


@pytest.mark.parametrize("o,v,naux", [(1, 3, 2), (2, 17, 7), (3, 33, 20), (4, 40, 37), (2, 50, 130)])
def test_paper_arrangement_matches_oracle_and_tau_pm(o, v, naux):
    """ri_ppl_paper (full (a, b) build, i <= j pairs) gives the oracle's ladder to 1e-11
    and ri_ppl's to rounding; entries with i < j and their mirrors are bitwise equal."""
    import torch
    ppl = _ppl()
    s = draw_system(o, v, naux, seed=o * 100 + v)
    T = draw_pair_symmetric(o, v, 7 + v, 0.01)
    R0 = draw_matrix((o, o, v, v), 3)
    ref = native.ppl(np.ascontiguousarray(s.B_vv), T, R0.copy())
    R = dev(R0)
    ppl.ppl_paper(dev(np.ascontiguousarray(s.B_vv)), dev(T), R)
    got = host(R)
    assert rel_max(got - R0, ref - R0) <= TOL and rel_fro(got - R0, ref - R0) <= TOL
    Rt = _gpu_ladder(s.B_vv, T, R0)
    assert rel_max(got - R0, Rt - R0) <= TOL
    Z = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    ppl.ppl_paper(dev(np.ascontiguousarray(s.B_vv)), dev(T), Z)
    add = host(Z)
    for i in range(o):
        for j in range(i + 1, o):
            assert np.array_equal(add[i, j], add[j, i].T)


def test_paper_arrangement_pair_symmetrises_tau_and_checks_arguments():
    import torch
    from paper_1810_08142_amd import _lib
    ppl = _ppl()
    o, v, naux = 3, 21, 11
    s = draw_system(o, v, naux, seed=4)
    T = draw_matrix((o, o, v, v), 9)  # not pair-symmetric
    Ts = 0.5 * (T + T.transpose(1, 0, 3, 2))
    B = dev(np.ascontiguousarray(s.B_vv))
    R1 = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    R2 = torch.zeros_like(R1)
    ppl.ppl_paper(B, dev(T), R1)
    ppl.ppl_paper(B, dev(Ts), R2)
    assert rel_max(host(R1), host(R2)) <= 1e-13
    assert ppl.paper_flops(o, v, naux) == 2.0 * naux * v**4 + v**4 * o * (o + 1)
    L = _lib.lib()
    assert L.ri_ppl_paper(None, B.data_ptr(), o, v, naux, R1.data_ptr(), None) == 1
    assert L.ri_ppl_paper(B.data_ptr(), B.data_ptr(), o, v, naux, B.data_ptr(), None) == 2
    torch.cuda.synchronize()


def test_paper_arrangement_chunks_do_not_change_result(monkeypatch):
    """The chunk of a values per build step (RI_PPL_PAPER_V_BYTES: 1, 7 with a ragged
    last chunk, all 40) changes the result only by rounding."""
    import torch
    ppl = _ppl()
    o, v, naux = 2, 40, 24
    s = draw_system(o, v, naux, seed=6)
    T = dev(draw_pair_symmetric(o, v, 5, 0.01))
    B = dev(np.ascontiguousarray(s.B_vv))
    outs = []
    for vb in (v**3 * 8, 7 * v**3 * 8, 1 << 30):
        monkeypatch.setenv("RI_PPL_PAPER_V_BYTES", str(vb))
        R = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
        ppl.ppl_paper(B, T, R)
        outs.append(host(R))
    assert rel_max(outs[1], outs[0]) <= 1e-13 and rel_max(outs[2], outs[0]) <= 1e-13


SYM_SHAPES = [  # (o, v, naux, slabs)
    (1, 3, 2, 8),        # one block pair: a single slab, no second product
    (2, 17, 7, 8),       # three block pairs, one per slab
    (1, 50, 20, 3),      # o = 1 (no antisymmetric part) over several slabs
    (3, 33, 20, 3),      # ragged slabs
    (4, 40, 37, 8),
    (2, 50, 130, 4),
    (3, 70, 24, 1000),   # one block pair per slab (15 slabs)
    (5, 64, 40, 2),      # v a multiple of 16, two slabs
]


@pytest.mark.parametrize("o,v,naux,slabs", SYM_SHAPES)
def test_exchange_symmetric_form_matches_oracle(o, v, naux, slabs, monkeypatch):
    """ri_ppl_sym (half the build through the (ab) <-> (cd) exchange symmetry) gives the
    oracle's ladder to 1e-11 and ri_ppl's to rounding, for any slab schedule."""
    import torch
    ppl = _ppl()
    print(f"ppl_sym o={o} v={v} naux={naux} slabs={slabs}", flush=True)
    monkeypatch.setenv("RI_PPL_SYM_SLABS", str(slabs))
    s = draw_system(o, v, naux, seed=o * 100 + v + 7)
    B = np.ascontiguousarray(s.B_vv)
    T = draw_pair_symmetric(o, v, 11 + v, 0.01)
    R0 = draw_matrix((o, o, v, v), 13)
    ref = native.ppl(B, T, R0.copy())
    R = dev(R0)
    ppl.ppl_sym(dev(B), dev(T), R)
    got = host(R)
    assert rel_max(got - R0, ref - R0) <= TOL and rel_fro(got - R0, ref - R0) <= TOL
    Rt = _gpu_ladder(B, T, R0)
    assert rel_max(got - R0, Rt - R0) <= TOL
    torch.cuda.synchronize()


# (16, 37, 29) and (48, 40, 24) reach the split path's 256 x 64k contraction tiles, in the
# slab contractions and in the second products
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("o,v,naux,slabs", [SYM_SHAPES[i] for i in (1, 3, 5, 6, 7)]
                         + [(16, 37, 29, 3), (48, 40, 24, 8), (4, 160, 48, 2)])
def test_exchange_symmetric_form_reduced_precision(o, v, naux, slabs, precision, monkeypatch):
    """ri_ppl_sym_ex in FP32 and split bf16: within the split error bound 2e-4 L(|B|, |tau|)
    of the oracle element by element (L: the oracle's ladder of the absolute values), and
    exactly pair-symmetric.  At o=4 v=160 (two slabs of 28 block pairs) the split form's
    second product is too small to fill the chip and runs as 13 k splits summed by
    sum_splits_f32; the smaller shapes take one or two."""
    import torch
    ppl = _ppl()
    print(f"ppl_sym {precision} o={o} v={v} naux={naux} slabs={slabs}", flush=True)
    monkeypatch.setenv("RI_PPL_SYM_SLABS", str(slabs))
    s = draw_system(o, v, naux, seed=o * 100 + v + 9)
    B = np.ascontiguousarray(s.B_vv)
    T = draw_pair_symmetric(o, v, 17 + v, 0.01)
    R = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    ppl.ppl_sym(dev(B), dev(T), R, precision=precision)
    got = host(R)
    ref = native.ppl(B, T)
    bound = 2e-4 * native.ppl(np.abs(B), np.abs(T))
    err = np.abs(got - ref)
    print("max rel err", float(err.max() / np.abs(ref).max()), "max err/bound", float((err / bound).max()))
    assert bool(np.all(err <= bound))
    assert float(err.max()) > 0.0
    assert np.array_equal(got, got.transpose(1, 0, 3, 2))


def test_exchange_symmetric_form_checks_its_factors_and_arguments():
    """Dressed (non-symmetric) factors are rejected with R untouched; a symmetric
    B passes; null and overlapping arguments give their status codes."""
    import torch
    from paper_1810_08142_amd import _lib
    ppl = _ppl()
    o, v, naux = 3, 21, 11
    s = draw_system(o, v, naux, seed=601, scale=0.2)
    t1 = draw_matrix((o, v), 602, 0.1)
    Bd = dev(np.ascontiguousarray(oc.dress(s.B, t1)[:, o:, o:]))
    T = dev(draw_pair_symmetric(o, v, 603))
    R = torch.full((o, o, v, v), 0.5, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.RIError) as ei:
        ppl.ppl_sym(Bd, T, R)
    assert ei.value.status == 1 and "not symmetric" in str(ei.value)
    assert bool((R == 0.5).all())
    B = dev(np.ascontiguousarray(s.B_vv))
    ppl.ppl_sym(B, T, R)
    assert not bool((R == 0.5).all())
    L = _lib.lib()
    assert L.ri_ppl_sym(None, T.data_ptr(), o, v, naux, R.data_ptr(), None) == 1
    assert L.ri_ppl_sym(B.data_ptr(), T.data_ptr(), o, v, naux, T.data_ptr(), None) == 2
    assert L.ri_ppl_sym_ex(B.data_ptr(), T.data_ptr(), o, v, naux, R.data_ptr(), 7, None) == 1
    torch.cuda.synchronize()
