"""Pins of the CPU RI-CCSD oracle.

The paper does not print its working equations (Sec. II names the spin-adapted
closed-shell formulation only), so the residual is pinned against a
determinant-space evaluation built literally from eqs. ccsd-1..3 and the
cluster operators of eqs. t1/t2 (tests/pins/detspace.py), and the solver against
two-electron exactness (CCSD = full CI for one occupied orbital)."""
import numpy as np
import pytest

from oracle import ccsd as oc
from paper_1810_08142_amd.synthetic import CONFIGS, draw_matrix, draw_pair_symmetric, draw_system
from pins.detspace import DetSpace


def _setup(o, v, naux, seed, scale=0.3):
    s = draw_system(o, v, naux, seed=seed, scale=scale)
    h, e_ref = oc.core_hamiltonian(s.B, s.eps, o)
    g = oc.eri(s.B, s.B)
    return s, h, e_ref, g


@pytest.mark.parametrize("o,v,naux,seed", [(2, 3, 6, 100), (2, 4, 8, 101), (1, 5, 6, 102), (3, 5, 10, 103)])
def test_residual_equals_determinant_space(o, v, naux, seed):
    s, h, e_ref, g = _setup(o, v, naux, seed)
    t1 = draw_matrix((o, v), seed + 1, 0.1)
    t2 = draw_pair_symmetric(o, v, seed + 2, 0.1)
    ds = DetSpace(o + v, o)
    e0, om1, om2 = ds.projections(h, g, t1, t2)
    O1, O2, terms = oc.residual(s.B, s.eps, o, t1, t2, terms=True)
    # every doubles term is far above the tolerance, so dropping any one fails
    for name, t in terms.items():
        assert np.abs(t).max() > 1e-3, name
    assert np.abs(O1 - om1).max() <= 1e-12
    assert np.abs(O2 - om2).max() <= 1e-12
    # energy expression of Sec. II.A at the same amplitudes
    assert abs((e0 - e_ref) - oc.energy(s.B, o, t1, t2)) <= 1e-12


def test_reference_energy_is_expectation_value():
    s, h, e_ref, g = _setup(2, 4, 8, 110)
    ds = DetSpace(6, 2)
    x = ds.reference()
    assert abs(x @ ds.apply_H(h, g, x) - e_ref) <= 1e-12


def test_iteration_zero_is_mp2():
    s, h, e_ref, g = _setup(3, 7, 9, 120, scale=0.05)
    o = 3
    z1 = np.zeros((o, 7))
    z2 = np.zeros((o, o, 7, 7))
    O1, O2 = oc.residual(s.B, s.eps, o, z1, z2)
    K = oc.ovov(s.B, o)
    D1, D2 = oc.denominators(s.eps, o)
    assert np.abs(O1).max() <= 1e-15
    np.testing.assert_allclose(O2, K.transpose(0, 2, 1, 3), rtol=0, atol=1e-15)
    t2 = O2 / D2
    e_closed = float(np.sum(K * (2 * K - K.transpose(0, 3, 2, 1)) / D2.transpose(0, 2, 1, 3)))
    _, t2m, em = oc.mp2(s.B, s.eps, o)
    np.testing.assert_allclose(t2, t2m, rtol=1e-14, atol=0)
    assert abs(em - e_closed) <= 1e-14 * abs(e_closed)
    r = oc.solve(s.B, s.eps, o, max_iter=1, t1=z1, t2=z2)
    np.testing.assert_allclose(r.t2, t2m, rtol=1e-14, atol=0)


@pytest.mark.parametrize("v,seed", [(4, 130), (9, 131)])
def test_two_electron_ccsd_is_exact(v, seed):
    s = draw_system(1, v, 2 * v, seed=seed, scale=0.3)
    r = oc.solve(s.B, s.eps, 1, max_iter=200, tol=1e-11, tol_energy=1e-12)
    assert r.converged
    e_fci = oc.fci_two_electron(s.B, s.eps)
    assert abs(r.e_corr - e_fci) <= 1e-10


def test_two_electron_fci_routines_agree():
    s, h, e_ref, g = _setup(1, 4, 6, 140)
    ds = DetSpace(5, 1)
    assert abs((ds.ground_energy(h, g) - e_ref) - oc.fci_two_electron(s.B, s.eps)) <= 1e-12


def test_converged_amplitudes_solve_determinant_space_equations():
    o, v = 2, 4
    s, h, e_ref, g = _setup(o, v, 8, 150)
    r = oc.solve(s.B, s.eps, o, max_iter=200, tol=1e-12, tol_energy=1e-13)
    assert r.converged
    ds = DetSpace(o + v, o)
    e0, om1, om2 = ds.projections(h, g, r.t1, r.t2)
    assert max(np.abs(om1).max(), np.abs(om2).max()) <= 1e-10
    assert abs((e0 - e_ref) - r.e_corr) <= 1e-10


def test_fixed_point_is_solver_independent():
    c = CONFIGS["c1"]
    s = draw_system(c["o"], c["v"], c["naux"], seed=c["seed"])
    kw = dict(max_iter=400, tol=1e-11, tol_energy=1e-12)
    r6 = oc.solve(s.B, s.eps, c["o"], diis_size=6, **kw)
    r3 = oc.solve(s.B, s.eps, c["o"], diis_size=3, **kw)
    rj = oc.solve(s.B, s.eps, c["o"], diis_size=0, **kw)
    assert r6.converged and r3.converged and rj.converged
    assert abs(r6.e_corr - r3.e_corr) <= 1e-10 and abs(r6.e_corr - rj.e_corr) <= 1e-10
    assert np.abs(r6.t2 - rj.t2).max() <= 1e-9
    assert r6.iterations < rj.iterations


def test_c1_workload_converges():
    c = CONFIGS["c1"]
    s = draw_system(c["o"], c["v"], c["naux"], seed=c["seed"])
    r = oc.solve(s.B, s.eps, c["o"], max_iter=100, tol=1e-10, tol_energy=1e-10)
    assert r.converged
    assert r.e_corr < r.e_mp2 * 0.5  # same sign, same order as MP2
    # pair symmetry is preserved by the iteration
    assert np.abs(r.t2 - r.t2.transpose(1, 0, 3, 2)).max() <= 1e-13


def test_diis_drops_oldest_when_singular():
    d = oc.DIIS(4)
    e = np.array([1.0, 2.0, 3.0])
    d.push(np.ones(3), e)
    d.push(2 * np.ones(3), e)          # identical error vectors: singular Gram system
    x = d.extrapolate()
    assert x is None and len(d.vecs) == 1
    d.push(3 * np.ones(3), np.array([1.0, 0.0, 0.0]))
    x = d.extrapolate()
    assert x is not None
    # coefficients sum to one
    c_sum = (x[0] - 3.0) / (2.0 - 3.0)
    assert np.isfinite(c_sum)


def test_dressing_is_similarity_transform():
    # B~ = (1 - t) B (1 + t) with t nilpotent: (1 - t)(1 + t) = 1, so the dressed
    # factors of B = identity are the identity, and undressing restores B.
    o, v = 2, 5
    n = o + v
    t1 = draw_matrix((o, v), 160, 0.2)
    I = np.eye(n)[None]
    np.testing.assert_allclose(oc.dress(I, t1)[0], np.eye(n), atol=1e-15)
    s = draw_system(o, v, 3, seed=161)
    back = oc.dress(oc.dress(s.B, t1), -t1)
    np.testing.assert_allclose(back, s.B, atol=1e-15)


def _triples_det_space(ds, h, g, eps, t1, t2):
    """E_(T) as the perturbative functional on the triply excited determinants T:
    sum_T x_T (x_T + y_T) / D_T with x = <T|H T2|0>, y = <T|H T1|0> and D_T the sum of
    the orbital energies of the vacated minus the filled spin orbitals (with a Fock
    matrix diag(eps) the one-electron part cannot reach T from singles or doubles)."""
    o, v = t1.shape
    ref = ds.reference()
    x = ds.apply_H(h, g, ds.apply_T(np.zeros_like(t1), t2, ref))
    y = ds.apply_H(h, g, ds.apply_T(t1, np.zeros_like(t2), ref))
    occ = (1 << o) - 1
    m = len(ds.strs)
    e = 0.0
    for ka, sa in enumerate(ds.strs):
        for kb, sb in enumerate(ds.strs):
            holes = [p for p in range(o) if not (sa >> p) & 1] + [p for p in range(o) if not (sb >> p) & 1]
            parts = [p for p in range(o, o + v) if (sa >> p) & 1] + [p for p in range(o, o + v) if (sb >> p) & 1]
            if len(holes) != 3:
                continue
            k = ka * m + kb
            d = sum(eps[p] for p in holes) - sum(eps[p] for p in parts)
            e += x[k] * (x[k] + y[k]) / d
    return e


@pytest.mark.parametrize("o,v,naux,seed", [(2, 3, 6, 200), (2, 4, 8, 201), (3, 4, 9, 202), (3, 5, 10, 203)])
def test_triples_energy_equals_determinant_space_functional(o, v, naux, seed):
    """The closed-shell (T) formula of Sec. II.A equals the (T) functional evaluated
    on explicit triply excited determinants, at arbitrary pair-symmetric amplitudes;
    both of its parts (through t2 alone and through t1) are far above the tolerance."""
    s, h, e_ref, g = _setup(o, v, naux, seed)
    t1 = draw_matrix((o, v), seed + 1, 0.1)
    t2 = draw_pair_symmetric(o, v, seed + 2, 0.1)
    ds = DetSpace(o + v, o)
    ref = _triples_det_space(ds, h, g, s.eps, t1, t2)
    got = oc.triples(s.B, s.eps, o, t1, t2)
    only_t2 = oc.triples(s.B, s.eps, o, np.zeros_like(t1), t2)
    assert abs(only_t2) > 1e-3 and abs(got - only_t2) > 1e-4
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))
    assert abs(only_t2 - _triples_det_space(ds, h, g, s.eps, np.zeros_like(t1), t2)) <= 1e-12


@pytest.mark.parametrize("v,seed", [(4, 300), (9, 301)])
def test_triples_vanish_for_two_electrons(v, seed):
    """With one occupied orbital there are no triple excitations: E_(T) = 0."""
    s = draw_system(1, v, 2 * v, seed=seed, scale=0.3)
    t1 = draw_matrix((1, v), seed + 1, 0.2)
    t2 = draw_pair_symmetric(1, v, seed + 2, 0.2)
    assert abs(oc.triples(s.B, s.eps, 1, t1, t2)) <= 1e-14
