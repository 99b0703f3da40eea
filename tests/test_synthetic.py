"""Properties of the seeded input generator (no method arithmetic involved)."""
import numpy as np

from paper_1810_08142_amd.synthetic import (CONFIGS, draw_pair_symmetric, draw_system, naux_scale,
                                            training_shapes)


def test_factors_symmetric_and_banded():
    s = draw_system(3, 20, 200, seed=7)
    assert s.B.shape == (200, 23, 23)
    assert np.array_equal(s.B, s.B.transpose(0, 2, 1))
    # standard deviation follows scale * exp(-|p-q|/8) along each band
    for dist in (0, 4, 12):
        band = np.concatenate([np.diagonal(s.B, offset=dist, axis1=1, axis2=2).ravel()])
        expect = 0.05 * np.exp(-dist / 8.0)
        assert abs(band.std() / expect - 1.0) < 0.05


def test_orbital_energies_and_singles():
    s = draw_system(5, 30, 10, seed=8)
    eo, ev = s.eps[:5], s.eps[5:]
    assert np.all(np.diff(eo) >= 0) and np.all(np.diff(ev) >= 0)
    assert eo.min() >= -1.5 and eo.max() <= -0.3 and ev.min() >= 0.2 and ev.max() <= 3.0
    assert s.t1.shape == (5, 30) and 0.5e-3 < s.t1.std() < 2e-3


def test_seeded_and_deterministic():
    a = draw_system(2, 6, 5, seed=3)
    b = draw_system(2, 6, 5, seed=3)
    c = draw_system(2, 6, 5, seed=4)
    assert np.array_equal(a.B, b.B) and np.array_equal(a.eps, b.eps) and np.array_equal(a.t1, b.t1)
    assert not np.array_equal(a.B, c.B)


def test_scale_options():
    assert naux_scale(96) == 0.05
    s = draw_system(2, 4, 384, seed=5, scale="naux")
    assert abs(s.scale - 0.025) < 1e-15


def test_pair_symmetric_draw():
    x = draw_pair_symmetric(3, 5, 9)
    assert np.array_equal(x, x.transpose(1, 0, 3, 2))


def test_training_shapes():
    sh = training_shapes()
    assert len(sh) == 256
    assert all(4 <= o <= 12 and 40 <= v <= 120 and n == 3 * v for o, v, n, _ in sh)
    assert sh[0][3] == 1000 and sh[-1][3] == 1255
    assert set(CONFIGS) == {"c1", "c2", "c3", "c4", "c5"}
