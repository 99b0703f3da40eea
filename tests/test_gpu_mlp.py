"""Learned-guess network kernels on the GPU against the FP64 CPU oracle.

GPU arithmetic is FP32 (sums of at most 256 products per unit and of the batch
for gradients); tolerance 1e-4 relative to the largest value."""
import os
import tempfile

import numpy as np
import pytest

from gpu_util import dev, host
from oracle import ccsd as oc
from oracle import mlp as om
from paper_1810_08142_amd.synthetic import draw_matrix, draw_system

pytestmark = pytest.mark.gpu


def _net(d_in=8, hidden=256, layers=2, seed=1):
    from paper_1810_08142_amd import mlp
    net = mlp.Net(d_in, hidden, layers)
    theta = mlp.init_params(d_in, hidden, layers, seed)
    theta[-1] = 0.3  # a non-zero output bias
    net.set_params(theta)
    return net, theta.astype(np.float64)


@pytest.mark.parametrize("hidden,layers,n", [(16, 1, 37), (256, 2, 1000), (64, 3, 513)])
def test_forward_and_gradient_match_oracle(hidden, layers, n):
    import torch
    net, theta = _net(8, hidden, layers, seed=hidden + layers)
    X = draw_matrix((n, 8), 5).astype(np.float32)
    Y = (0.5 * draw_matrix(n, 6)).astype(np.float32)
    y = host(net.forward(dev(X)))
    yr, _ = om.forward(theta, X.astype(np.float64), 8, hidden, layers)
    assert np.abs(y - yr).max() <= 1e-4 * max(1.0, np.abs(yr).max())
    loss, g = net.gradient(dev(X), dev(Y))
    Lr, gr = om.gradient(theta, X.astype(np.float64), Y.astype(np.float64), 8, hidden, layers)
    assert abs(loss - Lr) <= 1e-4 * Lr
    g = host(g)
    assert np.abs(g - gr).max() <= 1e-4 * np.abs(gr).max()


def test_adam_step_matches_oracle():
    net, theta = _net(8, 32, 2, seed=9)
    n = 300
    X = draw_matrix((n, 8), 7).astype(np.float32)
    Y = draw_matrix(n, 8).astype(np.float32)
    lr = 1e-2
    loss = net.train_step(dev(X), dev(Y), lr)
    new = net.get_params().astype(np.float64)
    L, g = om.gradient(theta, X.astype(np.float64), Y.astype(np.float64), 8, 32, 2)
    ref, _, _ = om.adam_step(theta, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    assert abs(loss - L) <= 1e-4 * L
    clear = np.abs(g) > 1e-3 * np.abs(g).max()  # the first step is lr*sign(g): skip g ~ 0
    assert np.abs(new - ref)[clear].max() <= 1e-5


def test_adam_steps_follow_the_oracle_trajectory():
    """Five consecutive ri_mlp_train_step calls on one batch against the oracle's own
    FP64 trajectory (its gradient, then its Adam step with the step count t = 1..5):
    after every step the parameters agree to 1e-5, so the library's step counter
    reaches the bias corrections as the oracle's does.  Parameters whose gradient is
    within FP32 noise of zero at some step are left out (there Adam's normalised step
    may take either sign)."""
    hidden, layers, n, lr = 32, 2, 300, 1e-3
    net, theta = _net(8, hidden, layers, seed=19)
    X = draw_matrix((n, 8), 17).astype(np.float32)
    Y = draw_matrix(n, 18).astype(np.float32)
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    Xd, Yd = dev(X), dev(Y)
    ref, m, v = theta.copy(), np.zeros_like(theta), np.zeros_like(theta)
    clear = np.ones(theta.size, dtype=bool)
    worst = 0.0
    for t in range(1, 6):
        loss = net.train_step(Xd, Yd, lr)
        L, g = om.gradient(ref, X64, Y64, 8, hidden, layers)
        ref, m, v = om.adam_step(ref, g, m, v, t, lr)
        clear &= np.abs(g) > 1e-3 * np.abs(g).max()
        got = net.get_params().astype(np.float64)
        assert abs(loss - L) <= 1e-4 * L
        err = float(np.abs(got - ref)[clear].max())
        worst = max(worst, err)
        print(f"adam step {t}: max |theta_gpu - theta_oracle| = {err:.2e} over {int(clear.sum())} parameters",
              flush=True)
        assert err <= 1e-5
    assert clear.sum() > 0.5 * theta.size


def test_sampling_matches_oracle():
    """ri_mlp_sample against the oracle's inverse-CDF sampler on the same SplitMix64
    stream.  The running sums are formed in another order (chunks of 4096), so an index
    may differ only where the threshold lies within rounding of a cumulative boundary;
    there the device's pick must still bracket the threshold."""
    from paper_1810_08142_amd import mlp
    o, v = 3, 70  # 44100 amplitudes: eleven chunks and a ragged last one
    t2m = draw_matrix((o, o, v, v), 41)
    t2m[0, 0, :5, :] = 0.0  # zero weights are never drawn
    n, seed = 20000, 77
    got = host(mlp.sample(dev(t2m), n, seed))
    ref, cum, u = om.sample_indices(t2m, n, seed)
    diff = np.nonzero(got != ref)[0]
    print(f"sampling: {diff.size} of {n} indices differ from the oracle's", flush=True)
    for s_ in diff:
        k = got[s_]
        lo = cum[k - 1] if k > 0 else 0.0
        assert lo - 1e-12 * cum[-1] <= u[s_] < cum[k] + 1e-12 * cum[-1]
    assert diff.size <= 2
    assert np.all(t2m.ravel()[got] != 0.0)


def test_targets_and_scaling_match_oracle():
    import torch
    from paper_1810_08142_amd import mlp
    shape = (2, 2, 9, 9)
    t2m = draw_matrix(shape, 51)
    t2c = t2m * (1.0 + 0.5 * draw_matrix(shape, 52))
    t2c.ravel()[:3] = 20.0 * t2m.ravel()[:3]  # beyond the clip
    idx = np.arange(0, t2m.size, 3, dtype=np.int64)
    Y = host(mlp.targets(dev(t2c), dev(t2m), dev(idx)))
    Yr = om.targets(t2c, t2m, idx).astype(np.float32)  # FP64 arithmetic, one rounding to FP32
    assert np.array_equal(Y, Yr)
    net = mlp.Net(8, 16, 1)
    n = 20001  # three row chunks, ragged
    X = (3.0 + 2.0 * draw_matrix((n, 8), 53)).astype(np.float32)
    X[:, 6] = 1.5  # a constant column: std 1 by convention
    Yv = (0.1 * draw_matrix(n, 54)).astype(np.float32)
    net.fit_scaling(dev(X), dev(Yv))
    mean, std, ys = net.get_scaling()
    mr, sr, ysr = om.scaling(X.astype(np.float64), Yv.astype(np.float64))
    np.testing.assert_allclose(mean, mr, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(std, sr, rtol=1e-6)
    assert abs(ys - ysr) <= 1e-6 * ysr
    Xn, Yn = net.standardize(dev(X), dev(Yv))
    Xr = (X.astype(np.float64) - mean.astype(np.float64)) / std.astype(np.float64)
    np.testing.assert_allclose(host(Xn), Xr, rtol=0, atol=1e-5)
    np.testing.assert_allclose(host(Yn), Yv.astype(np.float64) / float(ys), rtol=1e-6, atol=1e-7)
    Xn2, Yn2 = net.standardize(dev(X))
    assert Yn2 is None and torch.equal(Xn2, Xn)


def test_features_match_oracle():
    from paper_1810_08142_amd import mlp
    o, v, naux = 3, 13, 20
    s = draw_system(o, v, naux, seed=950)
    _, t2, _ = oc.mp2(s.B, s.eps, o)
    X = host(mlp.features(dev(s.B), dev(s.eps), o, dev(t2)))
    ref = om.features(s.B, s.eps, o, t2).reshape(-1, om.N_FEATURES)
    scale = np.abs(ref).max(axis=0)
    assert np.all(np.abs(X - ref) <= 1e-6 * scale + 1e-12)


@pytest.mark.parametrize("d_in,hidden,layers,n", [(8, 256, 2, 1000), (8, 64, 3, 4097), (4, 16, 1, 63),
                                                    (8, 48, 2, 65)])
def test_infer_equals_forward_bit_for_bit(d_in, hidden, layers, n):
    """The one-kernel inference keeps forward's operation order: equal y bit for bit
    (ragged row counts, 1-3 hidden layers, widths that are and are not multiples of 64)."""
    net, theta = _net(d_in, hidden, layers, seed=hidden + 7 * layers)
    X = draw_matrix((n, d_in), 17).astype(np.float32)
    yf = host(net.forward(dev(X)))
    yi = host(net.infer(dev(X)))
    assert np.array_equal(yf, yi)
    yr, _ = om.forward(theta, X.astype(np.float64), d_in, hidden, layers)
    assert np.abs(yi - yr).max() <= 1e-4 * max(1.0, np.abs(yr).max())


def test_infer_rejects_unsupported_widths():
    from paper_1810_08142_amd import _lib, mlp
    net = mlp.Net(8, 20, 2)
    with pytest.raises(_lib.RIError, match="ri_mlp_infer"):
        net.infer(dev(np.zeros((4, 8), dtype=np.float32)))


def test_guess_matches_oracle_on_the_pair_symmetric_half():
    """The guess runs the network on the i <= j amplitudes and mirrors them to
    (j, i, b, a); i == j averages the two orders of (a, b).  Oracle: features, the
    network in FP64 and the same composition."""
    from paper_1810_08142_amd import mlp
    o, v, naux = 3, 21, 40
    s = draw_system(o, v, naux, seed=961)
    net, theta = _net(8, 64, 2, seed=11)
    mean = np.array([0.0, 0.0, 0.01, 0.01, -2.0, 1.0, 0.1, 0.02], dtype=np.float32)
    std = np.array([0.05, 0.05, 0.02, 0.02, 1.0, 2.0, 0.2, 0.03], dtype=np.float32)
    ys = 0.05
    net.set_scaling(mean, std, ys)
    t1, t2 = net.guess(dev(s.B), dev(s.eps), o)
    t2 = host(t2)
    _, t2m, _ = oc.mp2(s.B, s.eps, o)
    F = om.features(s.B, s.eps, o, t2m).reshape(-1, om.N_FEATURES)
    Xn = (F - mean.astype(np.float64)) / std.astype(np.float64)
    y, _ = om.forward(theta, Xn, 8, 64, 2)
    val = (t2m * (1.0 + float(np.float32(ys)) * y.reshape(o, o, v, v)))
    ref = np.empty_like(val)
    for i in range(o):
        for j in range(o):
            if i < j:
                ref[i, j] = val[i, j]
            elif i > j:
                ref[i, j] = val[j, i].T
            else:
                ref[i, i] = 0.5 * (val[i, i] + val[i, i].T)
    assert np.abs(host(t1)).max() == 0.0
    assert np.array_equal(t2, t2.transpose(1, 0, 3, 2))
    assert np.abs(t2 - ref).max() <= 1e-5 * np.abs(t2m).max()


def test_zero_network_gives_mp2_and_correction_is_applied():
    from paper_1810_08142_amd import mlp
    o, v, naux = 2, 11, 15
    s = draw_system(o, v, naux, seed=960)
    B, eps = dev(s.B), dev(s.eps)
    net = mlp.Net()
    net.set_scaling(np.zeros(8), np.ones(8), 1.0)
    t1, t2 = net.guess(B, eps, o)
    _, t2r, _ = oc.mp2(s.B, s.eps, o)
    assert np.abs(host(t1)).max() == 0.0
    assert np.abs(host(t2) - t2r).max() <= 1e-15 * np.abs(t2r).max()
    theta = np.zeros(net.num_params, dtype=np.float32)
    theta[-1] = 0.5  # output bias only: every amplitude is scaled by 1 + y_scale * 0.5
    net.set_params(theta)
    net.set_scaling(np.zeros(8), np.ones(8), 0.01)
    _, t2c = net.guess(B, eps, o)
    factor = 1.0 + 0.5 * float(np.float32(0.01))  # the scale is stored in FP32
    assert float(np.abs(host(t2c) - factor * t2r).max()) <= 1e-15 * np.abs(t2r).max()


def test_save_load_roundtrip():
    from paper_1810_08142_amd import mlp
    net, theta = _net(8, 64, 2, seed=3)
    net.set_scaling(np.arange(8), np.arange(1, 9), 0.25)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.bin")
        net.save(path)
        other = mlp.Net.load(path)
    assert other.num_params == net.num_params
    assert np.array_equal(other.get_params(), net.get_params())
    m, sd, ys = other.get_scaling()
    assert np.array_equal(m, np.arange(8, dtype=np.float32)) and ys == np.float32(0.25)


def test_training_reduces_loss():
    import torch
    from paper_1810_08142_amd import mlp
    net, _ = _net(8, 64, 2, seed=4)
    n = 4096
    X = draw_matrix((n, 8), 11).astype(np.float32)
    Y = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]).astype(np.float32)
    Xd, Yd = dev(X), dev(Y)
    first = net.train_step(Xd, Yd, 3e-3)
    for _ in range(300):
        last = net.train_step(Xd, Yd, 3e-3, want_loss=False)
    last = net.train_step(Xd, Yd, 3e-3)
    assert last < 0.1 * first


def test_trained_guess_cuts_iterations_on_held_out_system():
    """Train on 128 small synthetic systems with the GPU kernels, then solve the
    held-out o=24 v=384 Naux=1152 system from the MP2 and from the learned guess:
    the learned start must reach the same solution in fewer iterations, and with the
    split-bf16 ladder and an FP64 polish in less wall time (network included)."""
    from paper_1810_08142_amd import guess
    from paper_1810_08142_amd.synthetic import training_shapes
    print("building training set", flush=True)
    X, Y, info = guess.build_dataset(training_shapes()[:128], 8192, seed=12345)
    print("training on", X.shape[0], "samples", flush=True)
    net, hist = guess.train(X, Y, epochs=20)
    print("held-out loss", hist[0], hist[-1], flush=True)
    assert hist[-1] < 0.5 * hist[0]
    res = guess.evaluate(net, "c5")
    print(res, flush=True)
    ie = res["initial_error"]
    assert ie["learned_rms"] < 0.5 * ie["mp2_rms"] and ie["learned_max"] < 0.5 * ie["mp2_max"]
    assert res["mp2_guess"]["converged"] and res["learned_guess"]["converged"]
    # the same CCSD solution (several exist), reached in fewer iterations
    assert abs(res["delta_e_corr"]) <= 1e-8 and res["max_abs_delta_t2"] <= 1e-6
    assert res["learned_guess"]["iterations"] < res["mp2_guess"]["iterations"]
    mix = guess.evaluate(net, "c5", precision="bf16x3", polish_residual=1e-6)
    print(mix, flush=True)
    assert mix["mp2_guess"]["converged"] and mix["learned_guess"]["converged"]
    assert abs(mix["delta_e_corr"]) <= 1e-8 and mix["max_abs_delta_t2"] <= 1e-6
    assert mix["learned_guess"]["seconds"] < mix["mp2_guess"]["seconds"]


# SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), output c of the stream seeded
# with `seed`, written here from its definition for the test.
_M64 = (1 << 64) - 1


def _splitmix(seed, c):
    c = np.asarray(c, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _fisher_yates(n, seed, ctr):
    xs = _splitmix(seed, np.arange(ctr, ctr + n - 1, dtype=np.uint64)).tolist()
    perm = list(range(n))
    for k, i in enumerate(range(n - 1, 0, -1)):
        j = (int(xs[k]) * (i + 1)) >> 64
        perm[i], perm[j] = perm[j], perm[i]
    return np.array(perm), ctr + n - 1


def test_seeded_init_is_box_muller_of_splitmix():
    from paper_1810_08142_amd import mlp
    d_in, hidden, layers, seed = 8, 64, 2, 77
    net = mlp.Net(d_in, hidden, layers)
    net.init(seed)
    got = net.get_params()
    ref, off = [], 0
    dims = [d_in] + [hidden] * layers + [1]
    for k in range(len(dims) - 1):
        nw = dims[k] * dims[k + 1]
        i = np.arange(off, off + nw, dtype=np.uint64)
        u1 = ((_splitmix(seed, 2 * i) >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0**-53
        u2 = (_splitmix(seed, 2 * i + np.uint64(1)) >> np.uint64(11)).astype(np.float64) * 2.0**-53
        ref.append(np.sqrt(-2.0 * np.log(u1)) * np.cos(2 * np.pi * u2) / np.sqrt(dims[k]))
        ref.append(np.zeros(dims[k + 1]))
        off += nw + dims[k + 1]
    ref = np.concatenate(ref).astype(np.float32)
    assert got.size == ref.size
    np.testing.assert_allclose(got, ref, rtol=2e-6, atol=1e-7)
    # the hidden-to-hidden weights are N(0, 1/64)
    w = got[d_in * hidden + hidden:][:hidden * hidden] * np.sqrt(hidden)
    assert abs(w.mean()) < 0.05 and abs(w.std() - 1.0) < 0.05
    other = mlp.Net(d_in, hidden, layers)
    other.init(seed + 1)
    assert not np.array_equal(other.get_params(), got)


@pytest.mark.parametrize("shuffle", [True, False])
def test_library_training_loop_equals_its_steps(shuffle):
    """ri_mlp_train (shuffle, batches, warm-up + cosine schedule, validation) gives
    bit for bit the parameters of the same steps taken one ri_mlp_train_step at a
    time, with the permutation and learning rates computed here from their
    definitions; 2000 rows in batches of 256 leave a ragged 208-row remainder."""
    import math

    import torch
    from paper_1810_08142_amd import mlp
    n, nv, batch, epochs, seed = 2000, 300, 256, 3, 5
    lr, warmup = np.float32(3e-3), np.float32(0.1)
    X = draw_matrix((n, 8), 21).astype(np.float32)
    Y = (np.sin(X[:, 0]) + 0.3 * X[:, 1] * X[:, 3]).astype(np.float32)
    Xv = draw_matrix((nv, 8), 22).astype(np.float32)
    Yv = (np.sin(Xv[:, 0]) + 0.3 * Xv[:, 1] * Xv[:, 3]).astype(np.float32)
    a = mlp.Net(8, 64, 2)
    a.init(3)
    tl, vl = a.train(dev(X), dev(Y), dev(Xv), dev(Yv), epochs=epochs, batch=batch, lr=float(lr),
                     warmup=float(warmup), seed=seed, shuffle=shuffle)
    b = mlp.Net(8, 64, 2)
    b.init(3)
    steps = n // batch
    total = epochs * steps
    warm = max(1, int(total * float(warmup)))
    ctr, it = 0, 0
    tl_ref, vl_ref = [], []
    for ep in range(epochs):
        perm = np.arange(n)
        if shuffle:
            perm, ctr = _fisher_yates(n, seed, ctr)
        Xe, Ye = dev(X[perm]), dev(Y[perm])
        acc = np.float32(0)
        for st in range(steps):
            rate = float(lr) * min(1.0, (it + 1) / warm) * 0.5 * (1.0 + math.cos(math.pi * it / total))
            loss = b.train_step(Xe[st * batch:(st + 1) * batch], Ye[st * batch:(st + 1) * batch], rate)
            acc = np.float32(acc + np.float32(1.0 / steps) * np.float32(loss))
            it += 1
        tl_ref.append(acc)
        yv = host(b.forward(dev(Xv))).astype(np.float64)
        vl_ref.append(np.mean((yv - Yv) ** 2))
    torch.cuda.synchronize()
    assert np.array_equal(a.get_params(), b.get_params())
    np.testing.assert_allclose(tl, tl_ref, rtol=1e-5)
    np.testing.assert_allclose(vl, vl_ref, rtol=1e-5)
    assert vl[-1] < vl[0]


def test_library_training_loop_argument_checks():
    import torch
    from paper_1810_08142_amd import _lib, mlp
    net = mlp.Net(8, 16, 1)
    X = dev(np.zeros((10, 8), dtype=np.float32))
    Y = dev(np.zeros(10, dtype=np.float32))
    with pytest.raises(_lib.RIError):
        net.train(X, Y, epochs=0)
    with pytest.raises(_lib.RIError):
        net.train(X, Y, lr=0.0)
    with pytest.raises(_lib.RIError):
        net.train(X, Y, warmup=1.5)
    # batch larger than the set: one step of all rows per epoch
    tl, vl = net.train(X, Y, epochs=2, batch=64)
    assert vl is None and tl.shape == (2,) and np.isfinite(tl).all()
    torch.cuda.synchronize()
