"""Pins of the CPU oracle of the learned guess: a hand-worked forward pass,
central finite differences of the loss, the exact-fit stationary point, closed
forms of Adam's steps (the first step, a constant gradient over several steps, a
single kick decaying over later steps), and the symmetry of the features."""
import math
import os

import numpy as np

from oracle import ccsd as oc
from oracle import mlp
from paper_1810_08142_amd.synthetic import draw_matrix, draw_system

HERE = os.path.dirname(os.path.abspath(__file__))


def test_hand_worked_forward():
    theta = np.array([1.0, -1.0, 0.0, 0.5, 2.0, -3.0, 0.25])
    x, y = np.loadtxt(os.path.join(HERE, "golden", "mlp_hand_1x2.txt"))
    got, _ = mlp.forward(theta, np.array([[x]]), 1, 2, 1)
    assert abs(got[0] - y) <= 1e-15
    assert abs(math.tanh(0.5) - (math.e - 1) / (math.e + 1)) <= 1e-16


def test_gradient_matches_central_differences():
    d_in, h, layers, n = 3, 5, 2, 7
    rng = np.random.default_rng(3)
    theta = 0.5 * rng.standard_normal(mlp.num_params(d_in, h, layers))
    X = rng.standard_normal((n, d_in))
    Y = rng.standard_normal(n)
    L, g = mlp.gradient(theta, X, Y, d_in, h, layers)
    assert abs(L - mlp.loss(theta, X, Y, d_in, h, layers)) <= 1e-15
    step = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = step
        fd[k] = (mlp.loss(theta + e, X, Y, d_in, h, layers) - mlp.loss(theta - e, X, Y, d_in, h, layers)) / (2 * step)
    assert np.abs(g - fd).max() <= 1e-6 * max(1.0, np.abs(g).max())


def test_exact_fit_is_stationary():
    d_in, h, layers = 2, 4, 2
    rng = np.random.default_rng(4)
    theta = rng.standard_normal(mlp.num_params(d_in, h, layers))
    X = rng.standard_normal((5, d_in))
    Y, _ = mlp.forward(theta, X, d_in, h, layers)
    L, g = mlp.gradient(theta, X, Y, d_in, h, layers)
    assert L == 0.0 and np.abs(g).max() == 0.0


def test_adam_first_step_closed_form():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    new, m, v = mlp.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # bias-corrected moments of step one are g and g^2
    np.testing.assert_allclose(new, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_adam_constant_gradient_moves_by_the_same_step_every_time():
    # With the same gradient g at every step the moments are m_t = (1 - b1^t) g and
    # v_t = (1 - b2^t) g^2 (geometric sums), so the bias-corrected update is
    # lr g / (|g| + eps) at every t.  A bias correction with a wrong step-count
    # dependence (for example 1 - b1 t) moves differently from t = 2 on.
    theta0 = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.3, -4.0, 1e-3, 2.5e-6])
    lr = 0.01
    step = lr * g / (np.abs(g) + 1e-8)
    theta, m, v = theta0.copy(), np.zeros(4), np.zeros(4)
    for t in range(1, 8):
        new, m, v = mlp.adam_step(theta, g, m, v, t, lr=lr)
        np.testing.assert_allclose(theta - new, step, rtol=1e-12, atol=1e-17)
        theta = new
    np.testing.assert_allclose(theta, theta0 - 7 * step, rtol=1e-12, atol=1e-15)


def test_adam_single_kick_decays_geometrically():
    # Gradient g at step 1 and zero afterwards: m_t = b1^(t-1) (1 - b1) g and
    # v_t = b2^(t-1) (1 - b2) g^2, so step t moves theta by
    #   lr * [b1^(t-1) (1 - b1) / (1 - b1^t)] g
    #      / (sqrt(b2^(t-1) (1 - b2) / (1 - b2^t)) |g| + eps).
    # This fixes which of beta and 1 - beta weights the old moment and that the
    # square root is taken of the second moment only.
    b1, b2, eps, lr = 0.9, 0.999, 1e-8, 0.05
    g1 = np.array([0.7, -1.5, 2.0])
    theta, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 7):
        g = g1 if t == 1 else np.zeros(3)
        new, m, v = mlp.adam_step(theta, g, m, v, t, lr=lr, beta1=b1, beta2=b2, eps=eps)
        mhat = b1 ** (t - 1) * (1 - b1) / (1 - b1 ** t) * g1
        shat = math.sqrt(b2 ** (t - 1) * (1 - b2) / (1 - b2 ** t)) * np.abs(g1)
        np.testing.assert_allclose(theta - new, lr * mhat / (shat + eps), rtol=1e-12, atol=0)
        theta = new


def test_features_pair_symmetric_and_defined():
    o, v = 3, 7
    s = draw_system(o, v, 9, seed=170)
    _, t2, _ = oc.mp2(s.B, s.eps, o)
    F = mlp.features(s.B, s.eps, o, t2)
    assert F.shape == (o, o, v, v, mlp.N_FEATURES)
    np.testing.assert_allclose(F, F.transpose(1, 0, 3, 2, 4), rtol=1e-15, atol=1e-18)
    i, j, a, b = 0, 2, 5, 1
    iajb = sum(s.B[q, i, o + a] * s.B[q, j, o + b] for q in range(9))
    ibja = sum(s.B[q, i, o + b] * s.B[q, j, o + a] for q in range(9))
    iaia = sum(s.B[q, i, o + a] ** 2 for q in range(9))
    jbjb = sum(s.B[q, j, o + b] ** 2 for q in range(9))
    e = s.eps
    want = [t2[i, j, a, b], t2[i, j, b, a], iajb, ibja, e[i] + e[j] - e[o + a] - e[o + b],
            (e[o + a] - e[o + b]) ** 2, (e[i] - e[j]) ** 2, math.sqrt(iaia * jbjb)]
    np.testing.assert_allclose(F[i, j, a, b], want, rtol=1e-13, atol=1e-16)


def test_splitmix64_reproduces_the_published_sequence():
    # the generator's reference output for state 0 (Vigna's splitmix64.c test values)
    assert [mlp.splitmix64(0, c) for c in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                        0x06C45D188009454F]
    u = mlp.sample_uniforms(1000, 9)
    assert u.min() > 0.0 and u.max() < 1.0


def test_sampler_inverse_cdf_hand_example():
    # weights 1, 0, 3 (t2 = 1, 0, sqrt 3): cumulative 1, 1, 4; a threshold below 1
    # picks index 0, one in [1, 4) picks index 2, and index 1 (zero weight) never
    idx, cum, u = mlp.sample_indices(np.array([1.0, 0.0, math.sqrt(3.0)]), 400, 5)
    np.testing.assert_allclose(cum, [1.0, 1.0, 4.0], rtol=1e-15)
    assert np.array_equal(idx, np.where(u < 1.0, 0, 2))


def test_sampler_frequencies_follow_the_squared_amplitudes():
    rng = np.random.default_rng(31)
    t = rng.standard_normal(7)
    t[3] = 0.0
    n = 60000
    idx, _, _ = mlp.sample_indices(t, n, 123)
    p = t**2 / np.sum(t**2)
    freq = np.bincount(idx, minlength=7) / n
    # binomial standard error sqrt(p (1 - p) / n) <= 0.0021; 5 sigma
    assert np.all(np.abs(freq - p) <= 5 * np.sqrt(p * (1 - p) / n) + 1e-12)
    assert freq[3] == 0.0


def test_targets_and_scaling_definitions():
    t2m = np.array([0.5, -0.25, 0.1, 2.0])
    t2c = np.array([0.75, -0.25, 1.0, -10.0])
    # 0.75/0.5 - 1 = 0.5; -0.25/-0.25 - 1 = 0; 1.0/0.1 - 1 = 9 -> clipped 3; -10/2 - 1 = -6 -> -3
    np.testing.assert_array_equal(mlp.targets(t2c, t2m, [0, 1, 2, 3]), [0.5, 0.0, 3.0, -3.0])
    X = np.array([[1.0, 5.0], [3.0, 5.0]])
    Y = np.array([2.0, 6.0])
    mean, std, ys = mlp.scaling(X, Y)
    # column 0: mean 2, deviations +-1 -> std 1; column 1 constant -> std 1 by convention
    np.testing.assert_array_equal(mean, [2.0, 5.0])
    np.testing.assert_array_equal(std, [1.0, 1.0])
    assert ys == 2.0
