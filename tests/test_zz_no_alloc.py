"""The allocation-free ladder (ri_ppl_noalloc, through the C ABI) against the ladder
with an allocated workspace (ri_ppl_ex) on the same inputs, two calls in a row, the
second smaller, in every precision.  Both share the library's fixed scratch array
across calls, so the second call also shows that nothing of the first one's
contents leaks into its result.

Bar (as for ri_ppl_ex against the oracle): FP64 max|dR| / max|dR_ex| and the Frobenius
ratio <= 1e-11; the reduced precisions each within 2e-4 L(|B|, |tau|) of the oracle
(the split error model), and of each other within twice that."""
import numpy as np
import pytest

from gpu_util import dev, host, rel_fro, rel_max
from oracle import native
from paper_1810_08142_amd.synthetic import draw_matrix, draw_pair_symmetric, draw_system

pytestmark = pytest.mark.gpu
TOL = 1e-11
EPS = 2e-4


def _both(B_vv, tau, R0, precision):
    from paper_1810_08142_amd import ppl
    Bd, Td = dev(B_vv), dev(tau)
    Ra, Rb = dev(R0), dev(R0)
    ppl.ppl(Bd, Td, Ra, precision=precision)
    ppl.ppl_noalloc(Bd, Td, Rb, precision=precision)
    return host(Ra), host(Rb)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_noalloc_matches_allocating_ladder_twice_shrinking(precision):
    # the first size spans several slabs of the fixed workspace in FP64; the second
    # is smaller and ragged
    for k, (o, v, naux) in enumerate([(6, 90, 250), (3, 37, 29)]):
        print(f"noalloc {precision} call {k + 1}: o={o} v={v} naux={naux}", flush=True)
        s = draw_system(o, v, naux, seed=1300 + v)
        tau = draw_pair_symmetric(o, v, 1301 + v)
        # from R = 0 the added part is exactly pair-symmetric
        _, r0 = _both(s.B_vv, tau, np.zeros((o, o, v, v)), precision)
        assert np.isfinite(r0).all()
        assert np.array_equal(r0, r0.transpose(1, 0, 3, 2))
        # accumulation into a non-zero R
        R0 = draw_matrix((o, o, v, v), 1302 + v)
        ra, rb = _both(s.B_vv, tau, R0, precision)
        da, db = ra - R0, rb - R0
        if precision == "fp64":
            assert rel_max(db, da) <= TOL and rel_fro(db, da) <= TOL
        else:
            ref = native.ppl(s.B_vv, tau)
            bound = EPS * native.ppl(np.abs(s.B_vv), np.abs(tau))
            assert bool(np.all(np.abs(db - ref) <= bound))
            assert bool(np.all(np.abs(da - ref) <= bound))
            assert bool(np.all(np.abs(db - da) <= 2 * bound))


def test_noalloc_rejects_a_size_beyond_its_scratch_and_leaves_R():
    import torch
    from paper_1810_08142_amd import _lib, ppl
    o, v, naux = 8, 128, 384
    B = torch.zeros((naux, v, v), dtype=torch.float64, device="cuda")
    T = torch.zeros((o, o, v, v), dtype=torch.float64, device="cuda")
    R = torch.full((o, o, v, v), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.RIError) as e:
        ppl.ppl_noalloc(B, T, R, precision="fp64")
    assert e.value.status == 3
    assert bool((R == 3.0).all())


def test_noalloc_pair_symmetry_check_uses_the_scratch(monkeypatch):
    """With RI_PPL_CHECK_TAU set the check's partial maxima also live in the scratch
    array: a pair-symmetric tau passes and gives the unchecked result bitwise, a
    perturbed one is rejected with R untouched."""
    from paper_1810_08142_amd import _lib, ppl
    o, v, naux = 3, 37, 29
    s = draw_system(o, v, naux, seed=1310)
    tau = draw_pair_symmetric(o, v, 1311)
    Bd, Td = dev(s.B_vv), dev(tau)
    R0 = draw_matrix((o, o, v, v), 1312)
    plain = dev(R0)
    ppl.ppl_noalloc(Bd, Td, plain)
    monkeypatch.setenv("RI_PPL_CHECK_TAU", "1")
    checked = dev(R0)
    ppl.ppl_noalloc(Bd, Td, checked)
    assert np.array_equal(host(plain), host(checked))
    bad = tau.copy()
    bad[0, 1, 2, 3] += 1e-6
    R = dev(R0)
    with pytest.raises(_lib.RIError) as e:
        ppl.ppl_noalloc(Bd, dev(bad), R)
    assert e.value.status == 1
    assert np.array_equal(host(R), R0)
