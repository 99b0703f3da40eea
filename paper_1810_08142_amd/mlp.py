"""Learned starting guess for the doubles amplitudes through the C ABI.

``Net`` wraps an ``ri_mlp`` handle: parameters and Adam state live on the GPU and
every forward, backward and update step runs in the library's kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .ccsd import _system
from .ppl import _need, _stream

N_FEATURES = 8


def _fp(x: np.ndarray):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Net:
    def __init__(self, d_in: int = N_FEATURES, hidden: int = 256, layers: int = 2, handle=None):
        L = _lib.lib()
        self._h = handle if handle is not None else L.ri_mlp_create(d_in, hidden, layers)
        if not self._h:
            raise _lib.RIError(1, "ri_mlp_create", L.ri_last_error_msg().decode())
        self.d_in, self.hidden, self.layers = d_in, hidden, layers

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.lib().ri_mlp_destroy(h)
            self._h = None

    @property
    def num_params(self) -> int:
        return int(_lib.lib().ri_mlp_num_params(self._h))

    def set_params(self, theta: np.ndarray):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        assert theta.size == self.num_params
        _lib.check(_lib.lib().ri_mlp_set_params(self._h, _fp(theta)), "ri_mlp_set_params")

    def get_params(self) -> np.ndarray:
        out = np.empty(self.num_params, dtype=np.float32)
        _lib.check(_lib.lib().ri_mlp_get_params(self._h, _fp(out)), "ri_mlp_get_params")
        return out

    def set_scaling(self, mean, std, y_scale: float):
        mean = np.ascontiguousarray(mean, dtype=np.float32)
        std = np.ascontiguousarray(std, dtype=np.float32)
        _lib.check(_lib.lib().ri_mlp_set_scaling(self._h, _fp(mean), _fp(std), float(y_scale)), "ri_mlp_set_scaling")

    def get_scaling(self):
        mean = np.empty(self.d_in, dtype=np.float32)
        std = np.empty(self.d_in, dtype=np.float32)
        ys = ctypes.c_float()
        _lib.check(_lib.lib().ri_mlp_get_scaling(self._h, _fp(mean), _fp(std), ctypes.byref(ys)), "ri_mlp_get_scaling")
        return mean, std, ys.value

    def forward(self, X: torch.Tensor, stream=None) -> torch.Tensor:
        n = X.shape[0]
        _need(X, "X", (n, self.d_in), torch.float32)
        y = torch.empty(n, dtype=torch.float32, device=X.device)
        _lib.check(_lib.lib().ri_mlp_forward(self._h, X.data_ptr(), n, y.data_ptr(), _stream(stream)), "ri_mlp_forward")
        return y

    def infer(self, X: torch.Tensor, stream=None) -> torch.Tensor:
        """The forward values without keeping the hidden activations (ri_mlp_infer)."""
        n = X.shape[0]
        _need(X, "X", (n, self.d_in), torch.float32)
        y = torch.empty(n, dtype=torch.float32, device=X.device)
        _lib.check(_lib.lib().ri_mlp_infer(self._h, X.data_ptr(), n, y.data_ptr(), _stream(stream)), "ri_mlp_infer")
        return y

    def gradient(self, X: torch.Tensor, Y: torch.Tensor, stream=None):
        n = X.shape[0]
        _need(X, "X", (n, self.d_in), torch.float32)
        _need(Y, "Y", (n,), torch.float32)
        g = torch.empty(self.num_params, dtype=torch.float32, device=X.device)
        loss = ctypes.c_float()
        _lib.check(_lib.lib().ri_mlp_gradient(self._h, X.data_ptr(), Y.data_ptr(), n, g.data_ptr(),
                                              ctypes.byref(loss), _stream(stream)), "ri_mlp_gradient")
        return loss.value, g

    def train_step(self, X: torch.Tensor, Y: torch.Tensor, lr: float, want_loss: bool = True, stream=None):
        n = X.shape[0]
        _need(X, "X", (n, self.d_in), torch.float32)
        _need(Y, "Y", (n,), torch.float32)
        loss = ctypes.c_float()
        _lib.check(_lib.lib().ri_mlp_train_step(self._h, X.data_ptr(), Y.data_ptr(), n, float(lr),
                                                ctypes.byref(loss) if want_loss else None, _stream(stream)),
                   "ri_mlp_train_step")
        return loss.value if want_loss else None

    def init(self, seed: int, stream=None):
        """Seeded starting parameters drawn on the device (ri_mlp_init)."""
        _lib.check(_lib.lib().ri_mlp_init(self._h, int(seed), _stream(stream)), "ri_mlp_init")

    def train(self, X: torch.Tensor, Y: torch.Tensor, X_val: torch.Tensor | None = None,
              Y_val: torch.Tensor | None = None, epochs: int = 30, batch: int = 4096, lr: float = 5e-4,
              warmup: float = 0.05, seed: int = 1, shuffle: bool = True, stream=None):
        """The whole training loop in the library (ri_mlp_train).

        Returns (train_loss, val_loss): per-epoch mean batch loss and validation loss
        (None without a validation set)."""
        n = X.shape[0]
        _need(X, "X", (n, self.d_in), torch.float32)
        _need(Y, "Y", (n,), torch.float32)
        nv = 0
        if X_val is not None:
            nv = X_val.shape[0]
            _need(X_val, "X_val", (nv, self.d_in), torch.float32)
            _need(Y_val, "Y_val", (nv,), torch.float32)
        o = _lib.RIMlpTrainOpts()
        _lib.lib().ri_mlp_default_train_opts(ctypes.byref(o))
        o.epochs, o.batch, o.lr, o.warmup = int(epochs), int(batch), float(lr), float(warmup)
        o.seed, o.shuffle = int(seed), 1 if shuffle else 0
        tl = np.zeros(o.epochs, dtype=np.float32)
        vl = np.zeros(o.epochs, dtype=np.float32)
        _lib.check(_lib.lib().ri_mlp_train(self._h, X.data_ptr(), Y.data_ptr(), n,
                                           X_val.data_ptr() if nv else None, Y_val.data_ptr() if nv else None, nv,
                                           ctypes.byref(o), _fp(tl), _fp(vl) if nv else None, _stream(stream)),
                   "ri_mlp_train")
        return tl, (vl if nv else None)

    @property
    def handle(self):
        """The ri_mlp handle (an integer address) for the C ABI."""
        return self._h

    def guess(self, B: torch.Tensor, eps: torch.Tensor, o: int, stream=None):
        """(t1, t2): the MP2 amplitudes corrected by the network, FP64."""
        sy = _system(B, eps, o)
        v = sy.v
        t1 = torch.empty((o, v), dtype=torch.float64, device=B.device)
        t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=B.device)
        _lib.check(_lib.lib().ri_mlp_guess(self._h, ctypes.byref(sy), t1.data_ptr(), t2.data_ptr(), _stream(stream)),
                   "ri_mlp_guess")
        return t1, t2

    def fit_scaling(self, X: torch.Tensor, Y: torch.Tensor, stream=None):
        """Set the feature standardisation and output scale from the raw training data
        (column means and deviations of X, deviation of Y; ri_mlp_fit_scaling)."""
        n = X.shape[0]
        _need(X, "X", (n, self.d_in), torch.float32)
        _need(Y, "Y", (n,), torch.float32)
        _lib.check(_lib.lib().ri_mlp_fit_scaling(self._h, X.data_ptr(), Y.data_ptr(), n, _stream(stream)),
                   "ri_mlp_fit_scaling")

    def standardize(self, X: torch.Tensor, Y: torch.Tensor | None = None, stream=None):
        """(Xn, Yn) = ((X - mean) / std, Y / y_scale) with the network's scaling
        (ri_mlp_standardize); Yn is None when Y is."""
        n = X.shape[0]
        _need(X, "X", (n, self.d_in), torch.float32)
        Xn = torch.empty_like(X)
        Yn = None
        if Y is not None:
            _need(Y, "Y", (n,), torch.float32)
            Yn = torch.empty_like(Y)
        _lib.check(_lib.lib().ri_mlp_standardize(self._h, X.data_ptr(), None if Y is None else Y.data_ptr(), n,
                                                 Xn.data_ptr(), None if Yn is None else Yn.data_ptr(),
                                                 _stream(stream)), "ri_mlp_standardize")
        return Xn, Yn

    def save(self, path: str):
        _lib.check(_lib.lib().ri_mlp_save(self._h, path.encode()), "ri_mlp_save")

    @classmethod
    def load(cls, path: str) -> "Net":
        L = _lib.lib()
        h = L.ri_mlp_load(path.encode())
        if not h:
            raise _lib.RIError(1, "ri_mlp_load", L.ri_last_error_msg().decode())
        # sizes are stored in the file; read them back from the header
        hdr = np.fromfile(path, dtype=np.int32, count=4)
        return cls(int(hdr[1]), int(hdr[2]), int(hdr[3]), handle=h)


def features(B: torch.Tensor, eps: torch.Tensor, o: int, t2_mp2: torch.Tensor, stream=None) -> torch.Tensor:
    """Raw per-amplitude features [o*o*v*v][8] (FP32) from the MP2 amplitudes."""
    sy = _system(B, eps, o)
    v = sy.v
    _need(t2_mp2, "t2", (o, o, v, v))
    X = torch.empty((o * o * v * v, N_FEATURES), dtype=torch.float32, device=B.device)
    _lib.check(_lib.lib().ri_mlp_features(ctypes.byref(sy), t2_mp2.data_ptr(), X.data_ptr(), _stream(stream)),
               "ri_mlp_features")
    return X


def sample(t2_mp2: torch.Tensor, n: int, seed: int, stream=None) -> torch.Tensor:
    """n amplitude indices (int64, flat) drawn with probability ~ t2_MP2^2 (ri_mlp_sample)."""
    if not t2_mp2.is_cuda or t2_mp2.dtype != torch.float64 or not t2_mp2.is_contiguous():
        raise TypeError("t2_mp2 must be a contiguous FP64 device tensor")
    idx = torch.empty(n, dtype=torch.int64, device=t2_mp2.device)
    _lib.check(_lib.lib().ri_mlp_sample(t2_mp2.data_ptr(), t2_mp2.numel(), n, int(seed), idx.data_ptr(),
                                        _stream(stream)), "ri_mlp_sample")
    return idx


def targets(t2_ccsd: torch.Tensor, t2_mp2: torch.Tensor, idx: torch.Tensor, clip: float = 3.0,
            stream=None) -> torch.Tensor:
    """Y[s] = clamp(t2_CCSD / t2_MP2 - 1, -clip, clip) at the flat indices idx (ri_mlp_targets)."""
    for t, name in ((t2_ccsd, "t2_ccsd"), (t2_mp2, "t2_mp2")):
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous FP64 device tensor")
    if idx.dtype != torch.int64 or not idx.is_cuda or not idx.is_contiguous():
        raise TypeError("idx must be a contiguous int64 device tensor")
    Y = torch.empty(idx.numel(), dtype=torch.float32, device=idx.device)
    _lib.check(_lib.lib().ri_mlp_targets(t2_ccsd.data_ptr(), t2_mp2.data_ptr(), idx.data_ptr(), idx.numel(),
                                         float(clip), Y.data_ptr(), _stream(stream)), "ri_mlp_targets")
    return Y


def init_params(d_in: int = N_FEATURES, hidden: int = 256, layers: int = 2, seed: int = 0) -> np.ndarray:
    """Seeded starting parameters: weights N(0, 1/fan_in), biases zero (flat FP32)."""
    rng = np.random.default_rng(seed)
    dims = [d_in] + [hidden] * layers + [1]
    out = []
    for k in range(len(dims) - 1):
        out.append(rng.standard_normal((dims[k], dims[k + 1])) / np.sqrt(dims[k]))
        out.append(np.zeros(dims[k + 1]))
    return np.concatenate([x.ravel() for x in out]).astype(np.float32)
