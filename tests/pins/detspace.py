"""Determinant-space evaluation of the CCSD equations (eqs. ccsd-1..3), for pins.

Nothing here is derived from working equations.  The Hamiltonian is written in
second quantisation from the one-electron matrix h and the integrals (pq|rs),

    H = sum_pq h_pq E_pq + 1/2 sum_pqrs (pq|rs) (E_pq E_rs - delta_qr E_ps),

with the spin-free generators E_pq = a+_pa a_qa + a+_pb a_qb acting on all Sz = 0
determinants of 2o electrons in n spatial orbitals.  The cluster operators are
built from the same generators exactly as defined in the paper (eqs. t1, t2):

    T1 = sum_ia t^a_i E_ai,     T2 = 1/2 sum_ijab t^{ab}_{ij} E_ai E_bj,

and exp(+-T) are their finite power series.  The projections of
exp(-T) H exp(T) |0> give the energy (eq. ccsd-1) and, read off on the
alpha-single and alpha-beta-double determinants, the residual components that
multiply E_ai|0> and 1/2 E_ai E_bj |0> in its singles and doubles part.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp


def _strings(n: int, k: int):
    return [sum(1 << p for p in c) for c in itertools.combinations(range(n), k)]


def _excite(s: int, p: int, q: int):
    """a+_p a_q on an occupation bit string of one spin; (new, sign) or None."""
    if not (s >> q) & 1:
        return None
    if p == q:
        return s, 1
    t = s & ~(1 << q)
    if (t >> p) & 1:
        return None
    lo, hi = (p, q) if p < q else (q, p)
    between = bin(t & (((1 << hi) - 1) & ~((1 << (lo + 1)) - 1))).count("1")
    return t | (1 << p), (-1) ** between


class DetSpace:
    """All Sz = 0 determinants of 2o electrons in n spatial orbitals.

    Spin orbitals are ordered all-alpha then all-beta; a determinant is the
    ordered product of its alpha then beta creation operators on the vacuum."""

    def __init__(self, n: int, o: int):
        self.n, self.o = n, o
        self.strs = _strings(n, o)
        self.pos = {s: k for k, s in enumerate(self.strs)}
        m = len(self.strs)
        self.dim = m * m
        ref = (1 << o) - 1
        self.ref = self.pos[ref] * m + self.pos[ref]
        self._Ea = {}
        self._E = {}

    def _spin_op(self, p: int, q: int, spin: int):
        key = (p, q, spin)
        if key in self._Ea:
            return self._Ea[key]
        m = len(self.strs)
        rows, cols, vals = [], [], []
        for ka, sa in enumerate(self.strs):
            for kb, sb in enumerate(self.strs):
                s = sa if spin == 0 else sb
                r = _excite(s, p, q)
                if r is None:
                    continue
                t, sign = r
                if spin == 0:
                    dst = self.pos[t] * m + kb
                else:
                    # moving past the o alpha electrons twice leaves the sign unchanged
                    dst = ka * m + self.pos[t]
                rows.append(dst)
                cols.append(ka * m + kb)
                vals.append(float(sign))
        op = sp.csr_matrix((vals, (rows, cols)), shape=(self.dim, self.dim))
        self._Ea[key] = op
        return op

    def E(self, p: int, q: int):
        key = (p, q)
        if key not in self._E:
            self._E[key] = (self._spin_op(p, q, 0) + self._spin_op(p, q, 1)).tocsr()
        return self._E[key]

    def reference(self):
        x = np.zeros(self.dim)
        x[self.ref] = 1.0
        return x

    # --- operators on vectors --------------------------------------------------
    def apply_H(self, h: np.ndarray, g: np.ndarray, x: np.ndarray) -> np.ndarray:
        """H x with g[p][q][r][s] = (pq|rs)."""
        n = self.n
        k = h - 0.5 * np.einsum("pqqs->ps", g)
        phi = np.array([self.E(r, s) @ x for r in range(n) for s in range(n)])  # [rs][dim]
        w = g.reshape(n * n, n * n) @ phi
        out = np.zeros_like(x)
        for p in range(n):
            for q in range(n):
                Epq = self.E(p, q)
                out += Epq @ (k[p, q] * x + 0.5 * w[p * n + q])
        return out

    def apply_T(self, t1: np.ndarray, t2: np.ndarray, x: np.ndarray) -> np.ndarray:
        o, v = t1.shape
        Ex = np.array([[self.E(o + b, j) @ x for b in range(v)] for j in range(o)])  # [j][b][dim]
        out = np.zeros_like(x)
        for i in range(o):
            for a in range(v):
                inner = 0.5 * np.einsum("jb,jbx->x", t2[i, :, a, :], Ex)
                out += self.E(o + a, i) @ (t1[i, a] * x + inner)
        return out

    def exp_T(self, t1, t2, x, sign=1.0):
        term = x.copy()
        out = x.copy()
        for k in range(1, 4 * self.o + 2):
            term = sign * self.apply_T(t1, t2, term) / k
            if not np.any(term):
                break
            out += term
        return out

    # --- CC quantities ---------------------------------------------------------
    def transformed(self, h, g, t1, t2):
        """exp(-T) H exp(T) |0>."""
        psi = self.exp_T(t1, t2, self.reference())
        return self.exp_T(t1, t2, self.apply_H(h, g, psi), sign=-1.0)

    def _single(self, a_orb: int, i: int):
        return self._spin_op(a_orb, i, 0) @ self.reference()

    def _double_ab(self, a_orb: int, i: int, b_orb: int, j: int):
        return self._spin_op(a_orb, i, 0) @ (self._spin_op(b_orb, j, 1) @ self.reference())

    def projections(self, h, g, t1, t2):
        """(<0|Hbar|0>, Omega1 [i][a], Omega2 [i][j][a][b])."""
        o, v = t1.shape
        chi = self.transformed(h, g, t1, t2)
        e0 = chi[self.ref]
        om1 = np.zeros((o, v))
        om2 = np.zeros((o, o, v, v))
        for i in range(o):
            for a in range(v):
                om1[i, a] = self._single(o + a, i) @ chi
        for i in range(o):
            for j in range(o):
                for a in range(v):
                    for b in range(v):
                        om2[i, j, a, b] = self._double_ab(o + a, i, o + b, j) @ chi
        return e0, om1, om2

    def ground_energy(self, h, g):
        """Lowest eigenvalue of H in this space (dense diagonalisation)."""
        cols = []
        for k in range(self.dim):
            e = np.zeros(self.dim)
            e[k] = 1.0
            cols.append(self.apply_H(h, g, e))
        Hm = np.array(cols).T
        return float(np.linalg.eigvalsh(0.5 * (Hm + Hm.T))[0])


def n_dets(n: int, o: int) -> int:
    return math.comb(n, o) ** 2
