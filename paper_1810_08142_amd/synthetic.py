"""Seeded synthetic RI systems (input generation only).

The paper's workloads are real molecules whose RI factors come from an atom-centred
basis (Sec. II.B, eq. RIM and eq. ri-v); none of that is available here, so every
input is drawn from a seeded generator that mimics their structure:

* RI factors ``B[Q][p][q]`` (the ``m^mu_pq`` of eq. RIM), symmetric in ``p, q``,
  with entries ``N(0, 1) * scale * exp(-|p-q|/8)`` over energy-ordered MOs
  (occupied first, then virtual; locality decays with the orbital-energy distance).
* canonical orbital energies: occupied ``U(-1.5, -0.3)`` and virtual ``U(0.2, 3.0)``
  Hartree, each block sorted ascending.
* singles amplitudes ``t1[i][a] ~ N(0, 1e-3)``.

This module holds no arithmetic of the method itself (no integrals, amplitudes or
energies): it only draws numbers.  Both the oracle and the GPU path take their
inputs from here.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

VERBATIM_SCALE = 0.05
DECAY = 8.0


def naux_scale(naux: int) -> float:
    """Generator scale that keeps amplitudes O(0.1) at any auxiliary size.

    ``0.05 * sqrt(96 / naux)``; equal to the verbatim 0.05 at ``naux = 96``.
    """
    return VERBATIM_SCALE * math.sqrt(96.0 / naux)


@dataclasses.dataclass
class System:
    o: int
    v: int
    naux: int
    seed: int
    scale: float
    B: np.ndarray  # [naux][n][n] float64, symmetric in the last two indices
    eps: np.ndarray  # [n] float64, occupied first, each block ascending
    t1: np.ndarray  # [o][v] float64

    @property
    def n(self) -> int:
        return self.o + self.v

    @property
    def B_vv(self) -> np.ndarray:
        return np.ascontiguousarray(self.B[:, self.o:, self.o:])

    @property
    def B_ov(self) -> np.ndarray:
        return np.ascontiguousarray(self.B[:, :self.o, self.o:])


def draw_system(o: int, v: int, naux: int, seed: int, scale: float | str = "verbatim",
                with_full_B: bool = True) -> System:
    """Draw one synthetic closed-shell system.

    Draw order (numpy ``default_rng(seed)``, PCG64):
      1. for each Q in order: ``G = standard_normal((n, n))``; the upper triangle
         (diagonal included) is kept and mirrored, then multiplied by
         ``scale * exp(-|p - q| / 8)``;
      2. ``eps_occ = sort(uniform(-1.5, -0.3, o))``, ``eps_vir = sort(uniform(0.2, 3.0, v))``;
      3. ``t1 = 1e-3 * standard_normal((o, v))``.
    ``scale`` is a float, ``"verbatim"`` (0.05) or ``"naux"`` (0.05*sqrt(96/naux)).
    """
    if o <= 0 or v <= 0 or naux <= 0:
        raise ValueError("o, v, naux must be positive")
    if scale == "verbatim":
        s = VERBATIM_SCALE
    elif scale == "naux":
        s = naux_scale(naux)
    else:
        s = float(scale)
    n = o + v
    rng = np.random.default_rng(seed)
    idx = np.arange(n)
    env = s * np.exp(-np.abs(idx[:, None] - idx[None, :]) / DECAY)
    upper = np.triu(np.ones((n, n), dtype=bool))
    B = np.empty((naux, n, n), dtype=np.float64)
    for q in range(naux):
        g = rng.standard_normal((n, n))
        g = np.where(upper, g, g.T)
        np.multiply(g, env, out=B[q])
    eps_occ = np.sort(rng.uniform(-1.5, -0.3, o))
    eps_vir = np.sort(rng.uniform(0.2, 3.0, v))
    t1 = 1e-3 * rng.standard_normal((o, v))
    return System(o=o, v=v, naux=naux, seed=seed, scale=s, B=B,
                  eps=np.concatenate([eps_occ, eps_vir]), t1=t1)


def draw_pair_symmetric(o: int, v: int, seed: int, std: float = 1.0) -> np.ndarray:
    """A random ``x[i][j][c][d]`` with pair symmetry ``x[i][j][c][d] == x[j][i][d][c]``.

    Used as a generic amplitude-shaped input for tests of the ladder contraction.
    """
    rng = np.random.default_rng(seed)
    g = std * rng.standard_normal((o, o, v, v))
    return 0.5 * (g + g.transpose(1, 0, 3, 2))


def draw_matrix(shape, seed: int, std: float = 1.0) -> np.ndarray:
    """Plain seeded normal array (generic test input)."""
    rng = np.random.default_rng(seed)
    return std * rng.standard_normal(shape)


# Workloads (seed, sizes) used by tests and the benchmark.
CONFIGS = {
    # full plain CCSD on CPU and GPU
    "c1": dict(o=4, v=24, naux=96, seed=1),
    # one ladder call, FP64
    "c2": dict(o=16, v=256, naux=768, seed=2),
    # full CCSD with mixed-precision ladder
    "c3": dict(o=32, v=512, naux=1536, seed=3),
    # large ladder, mixed vs FP64
    "c4": dict(o=48, v=768, naux=2304, seed=4),
    # held-out system of the learned-guess evaluation
    "c5": dict(o=24, v=384, naux=1152, seed=2000),
}


def training_shapes(count: int = 256, seed: int = 999, large: int = 0):
    """(o, v, naux, seed) of the learned-guess training systems: `count` small ones with
    o ~ U{4..12}, v ~ U{40..120}, naux = 3v, seeds 1000, 1001, ...; then `large` ones at
    the occupied/virtual ratio of the o=24 v=384 case, o ~ U{10..16}, v = 16 o,
    naux = 3v, seeds 5000, 5001, ..."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        o = int(rng.integers(4, 13))
        v = int(rng.integers(40, 121))
        out.append((o, v, 3 * v, 1000 + k))
    rng = np.random.default_rng(seed + 1)
    for k in range(large):
        o = int(rng.integers(10, 17))
        out.append((o, 16 * o, 48 * o, 5000 + k))
    return out
