"""Determinant-space (tier-0) second quantization for small closed-shell systems.

TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product path; only
the tests, the smoke check and the benchmark's CPU baseline may use the
``oracle`` package.

Everything in this module follows operator definitions, not working
equations: CI vectors are arrays C[alpha_string, beta_string]; the singlet
excitation operator E_pq = sum_sigma a+_{p sigma} a_{q sigma} acts on them
through signed string maps; H = sum h_pq E_pq + 1/2 sum g_pqrs e_pqrs with
e_pqrs = E_pq E_rs - delta_qr E_ps (Mulliken g_pqrs = (pq|rs)); the cluster
operator is T = sum t_ai E_ai + 1/2 sum t_aibj E_ai E_bj (Sec. II A); the
coupled-cluster residual is Omega_mu = <mu~| e^-T H e^T |HF> with the
biorthonormal dual <mu~| of |mu> = tau_mu |HF>.

Conventions (shared with the closed-shell oracle):
* orbitals 0..o-1 occupied, o..n-1 virtual;
* t1[i, a] = t_ai, t2[i, j, a, b] = t_aibj with t2[i,j,a,b] == t2[j,i,b,a];
* the doubles parameters are the unique pairs (ai) <= (bj) with compound
  index P = i*v + a; tau_(ai,bj) = E_ai E_bj for (ai) < (bj) and
  1/2 E_ai E_ai on the diagonal, so T2 = sum_mu t_mu tau_mu.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


class DetSpace:
    """CI space of o alpha and o beta electrons in n spatial orbitals."""

    def __init__(self, n: int, o: int):
        self.n, self.o, self.v = n, o, n - o
        self.strings = list(itertools.combinations(range(n), o))
        self.index = {s: k for k, s in enumerate(self.strings)}
        ns = self.ns = len(self.strings)
        self.A = [[None] * n for _ in range(n)]
        for p in range(n):
            for q in range(n):
                rows, cols, vals = [], [], []
                for k, s in enumerate(self.strings):
                    if q not in s or (p != q and p in s):
                        continue
                    rest = [x for x in s if x != q]
                    sign = (-1) ** sum(1 for x in s if x < q)
                    sign *= (-1) ** sum(1 for x in rest if x < p)
                    rows.append(self.index[tuple(sorted(rest + [p]))])
                    cols.append(k)
                    vals.append(float(sign))
                self.A[p][q] = sp.csr_matrix((vals, (rows, cols)), shape=(ns, ns))

    # ------------------------------------------------------------------ basics
    def hf(self) -> np.ndarray:
        C = np.zeros((self.ns, self.ns))
        k = self.index[tuple(range(self.o))]
        C[k, k] = 1.0
        return C

    def E(self, p: int, q: int, C: np.ndarray) -> np.ndarray:
        """E_pq C (alpha part acts on rows, beta part on columns)."""
        A = self.A[p][q]
        return A @ C + (A @ C.T).T

    def all_E(self, C: np.ndarray) -> np.ndarray:
        n = self.n
        return np.array([[self.E(p, q, C) for q in range(n)] for p in range(n)])

    def H(self, h: np.ndarray, g: np.ndarray, C: np.ndarray) -> np.ndarray:
        """(sum h_pq E_pq + 1/2 sum g_pqrs (E_pq E_rs - delta_qr E_ps)) C."""
        n = self.n
        D = self.all_E(C)
        k = h - 0.5 * np.einsum("prrq->pq", g)
        out = np.tensordot(k, D, axes=([0, 1], [0, 1]))
        Y = np.tensordot(g, D, axes=([2, 3], [0, 1]))
        for p in range(n):
            for q in range(n):
                out += 0.5 * self.E(p, q, Y[p, q])
        return out

    # ------------------------------------------------------- cluster operators
    def excite(self, x1: np.ndarray, x2: np.ndarray, C: np.ndarray,
               transpose: bool = False) -> np.ndarray:
        """X C with X = sum x1_ai E_ai + 1/2 sum x2_aibj E_ai E_bj, or X^T C."""
        o, v = self.o, self.v
        if transpose:
            Eop = lambda a, i, Z: self.E(i, o + a, Z)   # noqa: E731  E_ia
        else:
            Eop = lambda a, i, Z: self.E(o + a, i, Z)   # noqa: E731  E_ai
        Z = np.array([[Eop(b, j, C) for b in range(v)] for j in range(o)])
        out = np.zeros_like(C)
        for i in range(o):
            for a in range(v):
                W = x1[i, a] * C + 0.5 * np.tensordot(x2[i, :, a, :], Z,
                                                      axes=([0, 1], [0, 1]))
                out += Eop(a, i, W)
        return out

    def exp_excite(self, x1, x2, C, sign: float = 1.0, transpose: bool = False):
        """exp(sign * X) C by the (terminating) Taylor series."""
        out = C.copy()
        term = C.copy()
        for k in range(1, 2 * self.o + 2):
            term = sign * self.excite(x1, x2, term, transpose) / k
            if not np.any(term):
                break
            out += term
        return out

    def kappa_op(self, kappa: np.ndarray, C: np.ndarray) -> np.ndarray:
        """kappa C with kappa = sum_ai kappa_ai (E_ai - E_ia), kappa[i, a]."""
        o, v = self.o, self.v
        out = np.zeros_like(C)
        for i in range(o):
            for a in range(v):
                if kappa[i, a] != 0.0:
                    out += kappa[i, a] * (self.E(o + a, i, C) - self.E(i, o + a, C))
        return out

    def exp_kappa(self, kappa, C, sign: float = 1.0, tol: float = 1e-18):
        out = C.copy()
        term = C.copy()
        for k in range(1, 200):
            term = sign * self.kappa_op(kappa, term) / k
            out += term
            if np.abs(term).max() < tol:
                break
        return out

    # -------------------------------------------------- excitation manifold
    def pairs(self):
        o, v = self.o, self.v
        npair = o * v
        return [(P, Q) for P in range(npair) for Q in range(P, npair)]

    def basis(self):
        """Columns |mu> = tau_mu |HF> (singles then unique doubles), and S."""
        o, v = self.o, self.v
        hf = self.hf()
        cols = []
        for i in range(o):
            for a in range(v):
                cols.append(self.E(o + a, i, hf).ravel())
        single = {(i, a): self.E(o + a, i, hf) for i in range(o) for a in range(v)}
        for P, Q in self.pairs():
            i, a = divmod(P, v)
            j, b = divmod(Q, v)
            vec = self.E(o + a, i, single[(j, b)])
            if P == Q:
                vec = 0.5 * vec
            cols.append(vec.ravel())
        M = np.array(cols).T
        return M, M.T @ M

    def project(self, w: np.ndarray, M=None, S=None) -> np.ndarray:
        """<mu~|w> for all mu (biorthonormal dual coefficients)."""
        if M is None:
            M, S = self.basis()
        return np.linalg.solve(S, M.T @ w.ravel())

    def dual_vector(self, L: np.ndarray, M=None, S=None) -> np.ndarray:
        """CI coefficients of the bra sum_mu L_mu <mu~|."""
        if M is None:
            M, S = self.basis()
        return (M @ np.linalg.solve(S, L)).reshape(self.ns, self.ns)

    def ket_vector(self, x: np.ndarray, M=None) -> np.ndarray:
        """CI coefficients of sum_mu x_mu tau_mu |HF>."""
        if M is None:
            M, _ = self.basis()
        return (M @ x).reshape(self.ns, self.ns)

    # ------------------------------------------------------ CC by definition
    def cc_residual(self, h, g, t1, t2, M=None, S=None):
        """(E, Omega) with E = <HF|e^-T H e^T|HF>, Omega_mu = <mu~|...|HF>."""
        hf = self.hf()
        w = self.exp_excite(t1, t2, hf)
        w = self.H(h, g, w)
        w = self.exp_excite(t1, t2, w, sign=-1.0)
        E = float(np.sum(hf * w))
        return E, self.project(w, M, S)

    def hamiltonian_matrix(self, h, g) -> np.ndarray:
        ns = self.ns
        Hm = np.zeros((ns * ns, ns * ns))
        for k in range(ns * ns):
            e = np.zeros(ns * ns)
            e[k] = 1.0
            Hm[:, k] = self.H(h, g, e.reshape(ns, ns)).ravel()
        return Hm


def pack(t1: np.ndarray, t2: np.ndarray) -> np.ndarray:
    """Singles then unique doubles (P <= Q, P = i*v + a)."""
    o, v = t1.shape
    X = t2.transpose(0, 2, 1, 3).reshape(o * v, o * v)
    iu = np.triu_indices(o * v)
    return np.concatenate([t1.ravel(), X[iu]])


def unpack(x: np.ndarray, o: int, v: int):
    nov = o * v
    t1 = x[:nov].reshape(o, v).copy()
    X = np.zeros((nov, nov))
    iu = np.triu_indices(nov)
    X[iu] = x[nov:]
    X = X + X.T - np.diag(np.diag(X))
    t2 = X.reshape(o, v, o, v).transpose(0, 2, 1, 3).copy()
    return t1, t2


def two_electron_fci(h: np.ndarray, g: np.ndarray):
    """Singlet spectrum of a two-electron Hamiltonian (one alpha, one beta).

    The spatial wavefunction C[p, q] of a singlet is symmetric; H acts as
    h (x) 1 + 1 (x) h + g with (H C)[p,q] = sum_r h_pr C_rq + sum_s h_qs C_ps
    + sum_rs (pr|qs) C_rs.  Returns ascending eigenvalues and eigenvectors
    (columns, in the full n*n basis).
    """
    n = h.shape[0]
    I = np.eye(n)
    Hm = (np.einsum("pr,qs->pqrs", h, I) + np.einsum("pr,qs->pqrs", I, h)
          + g.transpose(0, 2, 1, 3)).reshape(n * n, n * n)
    # symmetric-subspace basis
    cols = []
    for p in range(n):
        for q in range(p, n):
            e = np.zeros((n, n))
            e[p, q] = e[q, p] = 1.0
            cols.append(e.ravel() / np.linalg.norm(e))
    U = np.array(cols).T
    w, V = np.linalg.eigh(U.T @ Hm @ U)
    return w, U @ V
