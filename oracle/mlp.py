"""Oracle -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this module; the product path never does.

Plain FP64 numpy version of the learned starting guess for the doubles
amplitudes: per-amplitude MP2 features, the training data (amplitudes sampled with
probability proportional to t2_MP2^2, their clipped relative corrections, the
standardisation statistics), a fully connected network with tanh hidden layers,
its mean-squared-error loss, the hand-derived backward pass and the Adam update.  (The paper has no learned component; this implements the
method the GPU library adds on top of the MP2 guess of Sec. II.A.)

Parameters are a flat FP64 vector in the order W1, b1, W2, b2, ..., W_out, b_out,
each W row-major [fan_in][fan_out].
"""
from __future__ import annotations

import numpy as np

N_FEATURES = 8


def shapes(d_in: int, hidden: int, layers: int):
    dims = [d_in] + [hidden] * layers + [1]
    out = []
    for k in range(len(dims) - 1):
        out.append((dims[k], dims[k + 1]))
        out.append((dims[k + 1],))
    return out


def num_params(d_in: int, hidden: int, layers: int) -> int:
    return int(sum(np.prod(s) for s in shapes(d_in, hidden, layers)))


def unflatten(theta: np.ndarray, d_in: int, hidden: int, layers: int):
    arrs, off = [], 0
    for s in shapes(d_in, hidden, layers):
        n = int(np.prod(s))
        arrs.append(theta[off:off + n].reshape(s))
        off += n
    assert off == theta.size
    return arrs


def forward(theta, X, d_in, hidden, layers):
    """y [n] and the hidden activations (for the backward pass)."""
    arrs = unflatten(theta, d_in, hidden, layers)
    H = [X]
    for k in range(layers):
        W, b = arrs[2 * k], arrs[2 * k + 1]
        H.append(np.tanh(H[-1] @ W + b))
    W, b = arrs[-2], arrs[-1]
    y = (H[-1] @ W + b)[:, 0]
    return y, H


def loss(theta, X, Y, d_in, hidden, layers) -> float:
    """mean over the batch of (y - Y)^2."""
    y, _ = forward(theta, X, d_in, hidden, layers)
    return float(np.mean((y - Y) ** 2))


def gradient(theta, X, Y, d_in, hidden, layers):
    """(loss, d loss / d theta) by the chain rule through each layer."""
    arrs = unflatten(theta, d_in, hidden, layers)
    y, H = forward(theta, X, d_in, hidden, layers)
    n = X.shape[0]
    r = y - Y
    L = float(np.mean(r ** 2))
    grads = [None] * len(arrs)
    delta = (2.0 / n) * r[:, None]                  # d loss / d (pre-activation of the output)
    grads[-2] = H[-1].T @ delta
    grads[-1] = delta.sum(axis=0)
    for k in range(layers - 1, -1, -1):
        W_next = arrs[2 * (k + 1)]
        dH = delta @ W_next.T                        # d loss / d H[k+1]
        delta = dH * (1.0 - H[k + 1] ** 2)           # tanh' = 1 - tanh^2
        grads[2 * k] = H[k].T @ delta
        grads[2 * k + 1] = delta.sum(axis=0)
    return L, np.concatenate([g.ravel() for g in grads])


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step t >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def features(B: np.ndarray, eps: np.ndarray, o: int, t2: np.ndarray) -> np.ndarray:
    """Per-amplitude inputs [o][o][v][v][8] from MP2 quantities (pair-symmetric):

    0: t2[i,j,a,b]           1: t2[i,j,b,a]
    2: (ia|jb)               3: (ib|ja)
    4: e_i + e_j - e_a - e_b 5: (e_a - e_b)^2
    6: (e_i - e_j)^2         7: sqrt((ia|ia) (jb|jb))
    """
    Bov = B[:, :o, o:]
    K = np.einsum("Qia,Qjb->iajb", Bov, Bov, optimize=True)
    v = Bov.shape[2]
    eo, ev = eps[:o], eps[o:]
    F = np.empty((o, o, v, v, N_FEATURES))
    F[..., 0] = t2
    F[..., 1] = t2.transpose(0, 1, 3, 2)
    F[..., 2] = K.transpose(0, 2, 1, 3)
    F[..., 3] = K.transpose(0, 2, 3, 1)
    F[..., 4] = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    F[..., 5] = np.broadcast_to(((ev[:, None] - ev[None, :]) ** 2)[None, None], (o, o, v, v))
    F[..., 6] = np.broadcast_to(((eo[:, None] - eo[None, :]) ** 2)[:, :, None, None], (o, o, v, v))
    diag = np.einsum("iaia->ia", K)
    F[..., 7] = np.sqrt(diag[:, None, :, None] * diag[None, :, None, :])
    return F


# ---------------------------------------------------------------- training data
_M64 = (1 << 64) - 1


def splitmix64(seed: int, c: int) -> int:
    """Output number c (0, 1, ...) of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
    seeded with `seed`: the state advanced c + 1 times by the golden-ratio increment,
    then mixed."""
    z = (seed + (c + 1) * 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def sample_uniforms(n: int, seed: int) -> np.ndarray:
    """u_s = ((x_s >> 11) + 1/2) 2^-53 in (0, 1), x_s = SplitMix64 output s of seed."""
    return np.array([((splitmix64(seed, k) >> 11) + 0.5) * 2.0**-53 for k in range(n)])


def sample_indices(t2_mp2: np.ndarray, n: int, seed: int):
    """n indices drawn with probability t2_mp2[k]^2 / sum t2_mp2^2 by the inverse of the
    cumulative weight: sample s picks the first k whose running sum of weights exceeds
    u_s times the total.  Returns (indices, running sums, thresholds)."""
    w = np.asarray(t2_mp2, dtype=np.float64).ravel() ** 2
    cum = np.cumsum(w)
    u = sample_uniforms(n, seed) * cum[-1]
    return np.searchsorted(cum, u, side="right"), cum, u


def targets(t2_ccsd: np.ndarray, t2_mp2: np.ndarray, idx, clip: float = 3.0) -> np.ndarray:
    """Relative corrections t2_CCSD / t2_MP2 - 1 at the flat indices, clipped to [-clip, clip]."""
    a, b = np.asarray(t2_ccsd).ravel()[idx], np.asarray(t2_mp2).ravel()[idx]
    return np.clip(a / b - 1.0, -clip, clip)


def scaling(X: np.ndarray, Y: np.ndarray):
    """(mean, std, y_scale): column means and standard deviations of X (divided by n; a
    zero deviation becomes 1) and the standard deviation of Y (0 becomes 1)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    mean = X.mean(axis=0)
    std = np.sqrt(((X - mean) ** 2).mean(axis=0))
    std[std <= 0] = 1.0
    ys = float(np.sqrt(((Y - Y.mean()) ** 2).mean()))
    return mean, std, (ys if ys > 0 else 1.0)
