"""Perturbative triples energy on the GPU (through the C ABI) against the oracle.

Both sides sum o^3 v^3 FP64 terms in different orders; the tolerance is 1e-10
relative to the energy (the terms themselves are of the energy's size)."""
import numpy as np
import pytest

from gpu_util import dev
from oracle import ccsd as oc
from paper_1810_08142_amd.synthetic import draw_matrix, draw_pair_symmetric, draw_system

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("o,v,naux,seed", [(1, 6, 8, 1), (2, 3, 6, 2), (3, 9, 12, 3), (4, 17, 20, 4),
                                           (5, 24, 40, 5), (3, 33, 50, 6)])
def test_triples_energy_matches_oracle(o, v, naux, seed):
    """Arbitrary amplitudes, ragged v (not a multiple of the 8-wide tiles), every
    triplet kind (all equal, two equal, distinct)."""
    from paper_1810_08142_amd import ccsd
    s = draw_system(o, v, naux, seed=seed, scale=0.3)
    t1 = draw_matrix((o, v), seed + 1, 0.05)
    t2 = draw_pair_symmetric(o, v, seed + 2, 0.05)
    ref = oc.triples(s.B, s.eps, o, t1, t2)
    got = ccsd.triples(dev(s.B), dev(s.eps), o, dev(t1), dev(t2))
    if o == 1:
        assert abs(got) <= 1e-14
    else:
        assert abs(got - ref) <= 1e-10 * abs(ref)


def test_triples_at_converged_ccsd_and_t1_part():
    """At the converged CCSD amplitudes of a small system the GPU (T) equals the
    oracle's, and so does its t2-only part (t1 = 0)."""
    import torch
    from paper_1810_08142_amd import ccsd
    o, v, naux = 4, 24, 96
    s = draw_system(o, v, naux, seed=1)
    B, eps = dev(s.B), dev(s.eps)
    t1, t2, rep = ccsd.solve(B, eps, o, tol=1e-10, tol_energy=1e-12)
    assert rep.converged
    t1h, t2h = t1.cpu().numpy(), t2.cpu().numpy()
    ref = oc.triples(s.B, s.eps, o, t1h, t2h)
    got = ccsd.triples(B, eps, o, t1, t2)
    assert ref < 0 and abs(got - ref) <= 1e-10 * abs(ref)
    ref2 = oc.triples(s.B, s.eps, o, np.zeros_like(t1h), t2h)
    got2 = ccsd.triples(B, eps, o, torch.zeros_like(t1), t2)
    assert abs(got2 - ref2) <= 1e-10 * abs(ref2)
    assert ccsd.triples_flops(o, v) == o * (o + 1) * (o + 2) * (2.0 * v**4 + 2.0 * v**3 * o)


@pytest.mark.parametrize("o,v,naux,seed", [(3, 24, 30, 7), (4, 33, 40, 8)])
def test_triples_fp32_gemms_within_their_rounding(o, v, naux, seed, monkeypatch):
    """With the term GEMMs in FP32 (forced onto the 128 x 128 tile kernel at these
    small sizes), E_(T) stays within 1e-6 of its size of the oracle, and does differ
    from the FP64 result (the FP32 path really runs)."""
    from paper_1810_08142_amd import ccsd
    monkeypatch.setenv("RI_GEMM_LARGE_MIN_TILES", "1")
    s = draw_system(o, v, naux, seed=seed, scale=0.3)
    t1 = draw_matrix((o, v), seed + 1, 0.05)
    t2 = draw_pair_symmetric(o, v, seed + 2, 0.05)
    ref = oc.triples(s.B, s.eps, o, t1, t2)
    args = (dev(s.B), dev(s.eps), o, dev(t1), dev(t2))
    e64 = ccsd.triples(*args)
    e32 = ccsd.triples(*args, precision="fp32")
    assert abs(e64 - ref) <= 1e-10 * abs(ref)
    assert abs(e32 - ref) <= 1e-6 * abs(ref)
    assert e32 != e64
