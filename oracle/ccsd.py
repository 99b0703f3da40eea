"""Oracle -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this module; the product path never does.

Plain FP64 closed-shell RI-CCSD on the CPU, written for a reader to check by eye:
numpy ``einsum`` is used as the tensor-contraction primitive, with no blocking,
packing or fusion beyond the definitions.

Conventions
-----------
* ``B[Q][p][q]``: RI factors of the MO integrals, ``(pq|rs) = sum_Q B^Q_pq B^Q_rs``
  (eq. RIM); MOs occupied first.  ``v^{pq}_{rs} = (pr|qs)`` (eq. eri).
* ``t1[i][a] = t^a_i`` (eq. t1), ``t2[i][j][a][b] = t^{ab}_{ij}`` (eq. t2, with the
  factor 1/2 of the doubles operator); pair symmetry ``t2[i,j,a,b] = t2[j,i,b,a]``.
* Fock matrix ``f = diag(eps)`` (canonical HF orbitals); the bare one-electron
  Hamiltonian follows from it, ``h_pq = eps_p delta_pq - sum_k [2(pq|kk) - (pk|kq)]``,
  and the reference energy is ``E_ref = sum_k (h_kk + eps_k)``.

The paper names the spin-adapted closed-shell equations it solves (Sec. II) but
does not print them.  The residual here is the T1-similarity-transformed
closed-shell form (integrals dressed by ``exp(-T1) H exp(T1)``), projected with
the biorthogonal basis in which the doubles part of the transformed Hamiltonian
acting on the reference is ``1/2 sum Omega_{aibj} E_ai E_bj |0>``.  It is pinned
by a determinant-space evaluation of eqs. ccsd-1..3 in the tests.
"""
from __future__ import annotations

import dataclasses

import numpy as np

_es = dict(optimize=True)


def eri(B1: np.ndarray, B2: np.ndarray) -> np.ndarray:
    """(pq|rs) = sum_Q B1^Q_pq B2^Q_rs (eq. RIM), returned as [p][q][r][s]."""
    return np.einsum("Qpq,Qrs->pqrs", B1, B2, **_es)


def core_hamiltonian(B: np.ndarray, eps: np.ndarray, o: int):
    """Bare one-electron Hamiltonian and reference energy for f = diag(eps).

    Returns (h, E_ref)."""
    Boo = B[:, :o, :o]
    J = np.einsum("Qpq,Qkk->pq", B, Boo, **_es)           # sum_k (pq|kk)
    K = np.einsum("Qpk,Qkq->pq", B[:, :, :o], B[:, :o, :], **_es)  # sum_k (pk|kq)
    h = np.diag(eps) - 2.0 * J + K
    e_ref = float(sum(h[k, k] + eps[k] for k in range(o)))
    return h, e_ref


def t1_operator(t1: np.ndarray, n: int) -> np.ndarray:
    """n x n matrix with t[a][k] = t^a_k (virtual row, occupied column)."""
    o, v = t1.shape
    t = np.zeros((n, n))
    t[o:, :o] = t1.T
    return t


def dress(B: np.ndarray, t1: np.ndarray) -> np.ndarray:
    """T1-dressed RI factors B~^Q = (1 - t) B^Q (1 + t)."""
    n = B.shape[1]
    t = t1_operator(t1, n)
    X = np.eye(n) - t
    Y = np.eye(n) + t
    return np.einsum("pr,Qrs,sq->Qpq", X, B, Y, **_es)


def dressed_fock(B: np.ndarray, h: np.ndarray, t1: np.ndarray, o: int):
    """F~_pq = h~_pq + sum_k [2 (pq|kk)~ - (pk|kq)~] with h~ = (1 - t) h (1 + t).

    Returns (F~, B~)."""
    n = B.shape[1]
    t = t1_operator(t1, n)
    hd = (np.eye(n) - t) @ h @ (np.eye(n) + t)
    Bd = dress(B, t1)
    J = np.einsum("Qpq,Qkk->pq", Bd, Bd[:, :o, :o], **_es)
    K = np.einsum("Qpk,Qkq->pq", Bd[:, :, :o], Bd[:, :o, :], **_es)
    return hd + 2.0 * J - K, Bd


def ppl(B_vv: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Ladder term sum_cd (ac|bd) tau^{cd}_{ij} (eq. pp-Ladder-0) -> [i][j][a][b].

    Forms the v^4 integral tensor; for small sizes only."""
    V = eri(B_vv, B_vv)  # [a][c][b][d]
    return np.einsum("acbd,ijcd->ijab", V, tau, **_es)


def ppl_paper_b(B_vv: np.ndarray, B_ov: np.ndarray, t1: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """The paper's ladder with t1-dressed integrals, eqs. pp-Ladder-0/-01/-1:

    b^{ab}_{cd} = v^{ab}_{cd} - sum_k v^{ak}_{cd} t^b_k - sum_k t^a_k v^{kb}_{cd},
    L^{ab}_{ij} = sum_cd b^{ab}_{cd} tau^{cd}_{ij},

    with v^{ab}_{cd} = (ac|bd), v^{ak}_{cd} = (ac|kd), v^{kb}_{cd} = (kc|bd).
    Small sizes only (forms v^4)."""
    v_abcd = eri(B_vv, B_vv)          # (ac|bd) as [a][c][b][d]
    v_akcd = eri(B_vv, B_ov)          # (ac|kd) as [a][c][k][d]
    v_kbcd = eri(B_ov, B_vv)          # (kc|bd) as [k][c][b][d]
    b = (np.einsum("acbd->abcd", v_abcd)
         - np.einsum("ackd,kb->abcd", v_akcd, t1, **_es)
         - np.einsum("ka,kcbd->abcd", t1, v_kbcd, **_es))
    return np.einsum("abcd,ijcd->ijab", b, tau, **_es)


def make_tau(t1: np.ndarray, t2: np.ndarray) -> np.ndarray:
    """tau^{ab}_{ij} = t^{ab}_{ij} + t^a_i t^b_j (eq. pp-Ladder-01)."""
    return t2 + np.einsum("ia,jb->ijab", t1, t1)


def ovov(B: np.ndarray, o: int) -> np.ndarray:
    """K[i][a][j][b] = (ia|jb) = v^{ij}_{ab}."""
    Bov = B[:, :o, o:]
    return eri(Bov, Bov)


def denominators(eps: np.ndarray, o: int):
    """D1[i][a] = e_i - e_a and D2[i][j][a][b] = e_i + e_j - e_a - e_b."""
    eo, ev = eps[:o], eps[o:]
    D1 = eo[:, None] - ev[None, :]
    D2 = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    return D1, D2


def energy(B: np.ndarray, o: int, t1: np.ndarray, t2: np.ndarray) -> float:
    """E_corr = sum_ijab (2 v^{ij}_{ab} - v^{ij}_{ba}) (t^{ab}_{ij} + t^a_i t^b_j)."""
    K = ovov(B, o)                                   # [i][a][j][b]
    L = 2.0 * K - K.transpose(0, 3, 2, 1)            # 2(ia|jb) - (ib|ja)
    return float(np.einsum("iajb,ijab->", L, make_tau(t1, t2), **_es))


def mp2(B: np.ndarray, eps: np.ndarray, o: int):
    """Iteration-0 guess: t1 = 0, t2 = (ia|jb) / D; returns (t1, t2, E_MP2)."""
    v = B.shape[1] - o
    K = ovov(B, o)
    _, D2 = denominators(eps, o)
    t2 = K.transpose(0, 2, 1, 3) / D2
    t1 = np.zeros((o, v))
    return t1, t2, energy(B, o, t1, t2)


def residual(B: np.ndarray, eps: np.ndarray, o: int, t1: np.ndarray, t2: np.ndarray,
             terms: bool = False):
    """CCSD residuals (Omega1 [i][a], Omega2 [i][j][a][b]).

    Omega2_{aibj} = (ai|bj)~ + A2 + B2 + P^{ab}_{ij} (C2 + D2 + E2),
    Omega1_{ai}   = sum u^{cd}_{ki} (ad|kc)~ - sum u^{ac}_{kl} (ki|lc)~
                    + sum u^{ac}_{ik} F~_kc + F~_ai,
    with u^{ab}_{ij} = 2 t^{ab}_{ij} - t^{ab}_{ji}, L_{pqrs} = 2(pq|rs) - (ps|rq),
    P^{ab}_{ij} X_{aibj} = X_{aibj} + X_{bjai}; "~" marks T1-dressed integrals.
    A2 is the particle-particle ladder with t2 (eq. pp-Ladder-0 evaluated on
    dressed factors).  With ``terms=True`` also returns the doubles terms.
    """
    h, _ = core_hamiltonian(B, eps, o)
    F, Bd = dressed_fock(B, h, t1, o)
    T = t2
    U = 2.0 * T - T.transpose(1, 0, 2, 3)            # u^{ab}_{ij} = 2t^{ab}_{ij} - t^{ab}_{ji}
    Boo, Bov, Bvo, Bvv = Bd[:, :o, :o], B[:, :o, o:], Bd[:, o:, :o], Bd[:, o:, o:]
    Fov, Fvo, Foo, Fvv = F[:o, o:], F[o:, :o], F[:o, :o], F[o:, o:]

    # integrals
    g_aibj = eri(Bvo, Bvo)                           # (ai|bj)~  [a][i][b][j]
    g_kilj = eri(Boo, Boo)                           # (ki|lj)~  [k][i][l][j]
    g_kcld = eri(Bov, Bov)                           # (kc|ld)   [k][c][l][d]
    g_kiac = eri(Boo, Bvv)                           # (ki|ac)~  [k][i][a][c]
    g_aikc = eri(Bvo, Bov)                           # (ai|kc)~  [a][i][k][c]
    g_adkc = eri(Bvv, Bov)                           # (ad|kc)~  [a][d][k][c]
    g_kilc = eri(Boo, Bov)                           # (ki|lc)~  [k][i][l][c]

    I2 = g_aibj.transpose(1, 3, 0, 2)                # -> [i][j][a][b]
    A2 = ppl(Bvv, T)
    W = g_kilj + np.einsum("kcld,ijcd->kilj", g_kcld, T, **_es)
    B2 = np.einsum("klab,kilj->ijab", T, W, **_es)

    Z = g_kiac - 0.5 * np.einsum("liad,kdlc->kiac", T, g_kcld, **_es)
    C2 = (-0.5 * np.einsum("kjbc,kiac->ijab", T, Z, **_es)
          - np.einsum("kibc,kjac->ijab", T, Z, **_es))

    Lt = 2.0 * g_aikc - g_kiac.transpose(2, 1, 0, 3)   # L~_{aikc} = 2(ai|kc)~ - (ac|ki)~
    L_ldkc = 2.0 * g_kcld - g_kcld.transpose(0, 3, 2, 1)  # L_{ldkc} = 2(ld|kc) - (lc|kd)
    Y = Lt + 0.5 * np.einsum("ilad,ldkc->aikc", U, L_ldkc, **_es)
    D2 = 0.5 * np.einsum("jkbc,aikc->ijab", U, Y, **_es)

    Gv = Fvv - np.einsum("klbd,ldkc->bc", U, g_kcld, **_es)
    Go = Foo + np.einsum("ljcd,kdlc->kj", U, g_kcld, **_es)
    E2 = (np.einsum("ijac,bc->ijab", T, Gv, **_es)
          - np.einsum("ikab,kj->ijab", T, Go, **_es))

    X = C2 + D2 + E2
    PX = X + X.transpose(1, 0, 3, 2)
    Om2 = I2 + A2 + B2 + PX

    Om1 = (np.einsum("kicd,adkc->ia", U, g_adkc, **_es)
           - np.einsum("klac,kilc->ia", U, g_kilc, **_es)
           + np.einsum("ikac,kc->ia", U, Fov, **_es)
           + Fvo.T)
    if terms:
        return Om1, Om2, dict(I2=I2, A2=A2, B2=B2, C2=C2, D2=D2, E2=E2)
    return Om1, Om2


class DIIS:
    """Pulay extrapolation over stored (Jacobi output, Jacobi step) pairs.

    With error vectors e_k (the Jacobi steps) and Gram matrix B_kl = <e_k, e_l>,
    solve [[B, 1], [1^T, 0]] [c, lam] = [0, 1] and return sum_k c_k (t_k + e_k).
    The Gram block is divided by its largest diagonal element before the solve.
    When the system is singular the oldest vector is dropped and the solve retried.
    """

    def __init__(self, size: int):
        self.size = size
        self.vecs: list[np.ndarray] = []
        self.errs: list[np.ndarray] = []

    def push(self, vec: np.ndarray, err: np.ndarray):
        self.vecs.append(vec.copy())
        self.errs.append(err.copy())
        if len(self.vecs) > self.size:
            self.vecs.pop(0)
            self.errs.pop(0)

    def extrapolate(self) -> np.ndarray | None:
        while len(self.vecs) >= 2:
            m = len(self.vecs)
            Bm = np.empty((m + 1, m + 1))
            for k in range(m):
                for l in range(m):
                    Bm[k, l] = float(np.dot(self.errs[k], self.errs[l]))
            # the solution is invariant under scaling of the Gram block; scale it to O(1)
            # so the singularity test is not dominated by the bordering ones
            Bm[:m, :m] /= np.max(np.abs(np.diag(Bm)[:m]))
            Bm[m, :m] = 1.0
            Bm[:m, m] = 1.0
            Bm[m, m] = 0.0
            rhs = np.zeros(m + 1)
            rhs[m] = 1.0
            c = _solve_partial_pivot(Bm, rhs)
            if c is None:
                self.vecs.pop(0)
                self.errs.pop(0)
                continue
            return sum(c[k] * self.vecs[k] for k in range(m))
        return None


def _solve_partial_pivot(A: np.ndarray, b: np.ndarray, rcond: float = 1e-14):
    """Gaussian elimination with partial pivoting; None when (near) singular."""
    A = A.astype(np.float64).copy()
    b = b.astype(np.float64).copy()
    n = len(b)
    scale = np.max(np.abs(A))
    for col in range(n):
        piv = col + int(np.argmax(np.abs(A[col:, col])))
        if abs(A[piv, col]) <= rcond * scale:
            return None
        if piv != col:
            A[[col, piv]] = A[[piv, col]]
            b[[col, piv]] = b[[piv, col]]
        for r in range(col + 1, n):
            f = A[r, col] / A[col, col]
            A[r, col:] -= f * A[col, col:]
            b[r] -= f * b[col]
    x = np.zeros(n)
    for r in range(n - 1, -1, -1):
        x[r] = (b[r] - A[r, r + 1:] @ x[r + 1:]) / A[r, r]
    return x


@dataclasses.dataclass
class Result:
    t1: np.ndarray
    t2: np.ndarray
    e_corr: float
    e_mp2: float
    iterations: int
    converged: bool
    residual_inf: float
    history: list


def solve(B: np.ndarray, eps: np.ndarray, o: int, max_iter: int = 100, tol: float = 1e-10,
          tol_energy: float = 1e-10, diis_size: int = 6, diis_start: int = 2,
          t1: np.ndarray | None = None, t2: np.ndarray | None = None) -> Result:
    """Jacobi iterations t += Omega / D with DIIS, from the MP2 guess unless
    (t1, t2) are given.  Converged when ||Omega||_inf <= tol and |dE| <= tol_energy,
    both measured on the current amplitudes before they are updated.  After each
    update t2 is replaced by its pair-symmetric part."""
    D1, D2 = denominators(eps, o)
    _, t2_mp2, e_mp2 = mp2(B, eps, o)
    if t2 is None:
        t1 = np.zeros_like(D1)
        t2 = t2_mp2
    elif t1 is None:
        t1 = np.zeros_like(D1)
    e_prev = None
    e = energy(B, o, t1, t2)
    diis = DIIS(diis_size) if diis_size >= 2 else None
    hist = []
    conv = False
    rinf = float("inf")
    it = 0
    nt1 = t1.size
    for it in range(max_iter):
        Om1, Om2 = residual(B, eps, o, t1, t2)
        rinf = max(np.max(np.abs(Om1)), np.max(np.abs(Om2)))
        hist.append((it, e, rinf))
        if rinf <= tol and e_prev is not None and abs(e - e_prev) <= tol_energy:
            conv = True
            break
        t1n = t1 + Om1 / D1
        t2n = t2 + Om2 / D2
        step = np.concatenate([(t1n - t1).ravel(), (t2n - t2).ravel()])
        new = np.concatenate([t1n.ravel(), t2n.ravel()])
        if diis is not None:
            diis.push(new, step)
            if it + 1 >= diis_start:
                ex = diis.extrapolate()
                if ex is not None:
                    new = ex
        t1 = new[:nt1].reshape(t1.shape)
        t2 = new[nt1:].reshape(t2.shape)
        # only the pair-symmetric part of t2 enters T2 (E_ai and E_bj commute, eq. t2);
        # the other part is an unstable mode of the iteration, so it is removed
        t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
        e_prev = e
        e = energy(B, o, t1, t2)
    return Result(t1=t1, t2=t2, e_corr=e, e_mp2=e_mp2, iterations=it, converged=conv,
                  residual_inf=rinf, history=hist)


def fci_two_electron(B: np.ndarray, eps: np.ndarray) -> float:
    """Exact correlation energy of a one-occupied-orbital (two-electron) system.

    Singlet spatial wavefunction Psi = sum_pq C_pq phi_p(1) phi_q(2), C symmetric;
    H_{pq,rs} = h_pr d_qs + d_pr h_qs + (pr|qs).  Returns E_FCI - E_ref for the
    lowest singlet root (the one dominated by the reference)."""
    n = B.shape[1]
    h, e_ref = core_hamiltonian(B, eps, 1)
    g = eri(B, B)                                    # (pr|qs) as [p][r][q][s]
    I = np.eye(n)
    H = (np.einsum("pr,qs->pqrs", h, I) + np.einsum("pr,qs->pqrs", I, h)
         + g.transpose(0, 2, 1, 3)).reshape(n * n, n * n)
    # orthonormal basis of symmetric C
    cols = []
    for p in range(n):
        for q in range(p, n):
            c = np.zeros((n, n))
            if p == q:
                c[p, p] = 1.0
            else:
                c[p, q] = c[q, p] = 1.0 / np.sqrt(2.0)
            cols.append(c.ravel())
    S = np.array(cols).T
    Hs = S.T @ H @ S
    w, vecs = np.linalg.eigh(Hs)
    ref = np.zeros(Hs.shape[0])
    ref[0] = 1.0                                     # (p, q) = (0, 0)
    k = int(np.argmax(np.abs(vecs.T @ ref)))
    return float(w[k] - e_ref)


def triples(B: np.ndarray, eps: np.ndarray, o: int, t1: np.ndarray, t2: np.ndarray) -> float:
    """Perturbative triples energy E_(T) of the closed-shell formula of Sec. II.A:

        E_(T) = sum_{ijk} sum_{abc} (4 W^{abc}_{ijk} + W^{bca}_{ijk} + W^{cab}_{ijk})
                                     (V^{abc}_{ijk} - V^{cba}_{ijk}) / (3 D^{abc}_{ijk}),
        W^{abc}_{ijk} = P^{abc}_{ijk} ( sum_d v^{ba}_{di} t^{cd}_{kj} - sum_l v^{cj}_{kl} t^{ab}_{il} ),
        V^{abc}_{ijk} = W^{abc}_{ijk} + v^{bc}_{jk} t^a_i + v^{ac}_{ik} t^b_j + v^{ab}_{ij} t^c_k,
        D^{abc}_{ijk} = e_i + e_j + e_k - e_a - e_b - e_c,

    with v^{pq}_{rs} = (pr|qs) and P^{abc}_{ijk} the sum over the six simultaneous
    permutations of the column pairs (i, a), (j, b), (k, c).  Full o^3 v^3 arrays:
    for small systems only."""
    v = t1.shape[1]
    g = eri(B, B)
    O, V = slice(0, o), slice(o, o + v)
    g_vvvo = g[V, V, V, O]  # (bd|ai) at [b][d][a][i]
    g_vooo = g[V, O, O, O]  # (ck|jl) at [c][k][j][l]
    g_ovov = g[O, V, O, V]  # (ia|jb) at [i][a][j][b]
    # X(ijk, abc) = sum_d v^{ba}_{di} t^{cd}_{kj} - sum_l v^{cj}_{kl} t^{ab}_{il}
    #             = sum_d (bd|ai) t2[k,j,c,d]   - sum_l (ck|jl) t2[i,l,a,b]
    X = (np.einsum("bdai,kjcd->ijkabc", g_vvvo, t2, **_es)
         - np.einsum("ckjl,ilab->ijkabc", g_vooo, t2, **_es))
    # P: f(ijk,abc) + f(ikj,acb) + f(kij,cab) + f(kji,cba) + f(jki,bca) + f(jik,bac)
    W = (X + np.einsum("ikjacb->ijkabc", X) + np.einsum("kijcab->ijkabc", X)
         + np.einsum("kjicba->ijkabc", X) + np.einsum("jkibca->ijkabc", X) + np.einsum("jikbac->ijkabc", X))
    # v^{bc}_{jk} = (bj|ck) = (jb|kc)
    Vt = (W + np.einsum("jbkc,ia->ijkabc", g_ovov, t1) + np.einsum("iakc,jb->ijkabc", g_ovov, t1)
          + np.einsum("iajb,kc->ijkabc", g_ovov, t1))
    e_o, e_v = eps[:o], eps[o:]
    D = (e_o[:, None, None, None, None, None] + e_o[None, :, None, None, None, None]
         + e_o[None, None, :, None, None, None] - e_v[None, None, None, :, None, None]
         - e_v[None, None, None, None, :, None] - e_v[None, None, None, None, None, :])
    W_bca = np.einsum("ijkbca->ijkabc", W)  # W^{bca}_{ijk} as an array over (a, b, c)
    W_cab = np.einsum("ijkcab->ijkabc", W)
    V_cba = np.einsum("ijkcba->ijkabc", Vt)
    return float(np.sum((4.0 * W + W_bca + W_cab) * (Vt - V_cba) / (3.0 * D)))
