"""Closed-shell CCSD residual, energy and ground-state solver (fp64, CPU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The residual Omega_mu = <mu~| exp(-T) H exp(T) |HF> (Sec. II A) is evaluated in
the T1-transformed form: with Hhat = exp(-T1) H exp(T1) the singles and
doubles projections are written in terms of the transformed integrals hhat,
ghat and the transformed Fock matrix Fhat, and T1 only enters through the
transformation.  The paper does not print the closed-shell working equations;
those below are the standard spin-adapted T1-transformed CCSD equations
(Koch et al.), restated here and pinned against the determinant-space
definition in ``oracle.detspace`` (tests/test_oracle_ccsd.py).

Fock matrix (Sec. II A, with Coulomb and exchange in Mulliken order):
f_pq = h_pq + sum_k (2 g_pqkk - g_pkkq).

Layouts: t1[i, a] = t_ai; t2[i, j, a, b] = t_aibj (symmetric under
(i,a) <-> (j,b)); h[p, q]; g[p, q, r, s] = (pq|rs).  Occupied orbitals come
first.  Everything is torch.float64 on the CPU so that the Jacobians of the
method can be taken by automatic differentiation.
"""
from __future__ import annotations

import numpy as np
import torch

DT = torch.float64


def as_t(x):
    if isinstance(x, torch.Tensor):
        return x.to(DT)
    return torch.as_tensor(np.asarray(x), dtype=DT)


def fock(h, g, o: int):
    """f_pq = h_pq + sum_k (2 g_pqkk - g_pkkq)."""
    J = torch.einsum("pqkk->pq", g[:, :, :o, :o])
    K = torch.einsum("pkkq->pq", g[:, :o, :o, :])
    return h + 2.0 * J - K


def hamiltonian_from_eps(eps, g, o: int):
    """One-electron integrals that make the Fock matrix equal diag(eps)."""
    eps = as_t(eps)
    J = torch.einsum("pqkk->pq", g[:, :, :o, :o])
    K = torch.einsum("pkkq->pq", g[:, :o, :o, :])
    return torch.diag(eps) - 2.0 * J + K


def eri_from_factor(B):
    """(pq|rs) = sum_P B[P,p,q] B[P,r,s]."""
    B = as_t(B)
    return torch.einsum("Ppq,Prs->pqrs", B, B)


def t1_transform(h, g, t1, o: int):
    """hhat = X h Y^T and ghat_pqrs = X_pp' Y_qq' X_rr' Y_ss' g_p'q'r's'.

    exp(-T1) a+_p exp(T1) = sum_r a+_r X_rp with X = 1 - t~ and
    exp(-T1) a_q exp(T1) = sum_s a_s Y_sq with Y = 1 + t~^T, where
    t~[a, i] = t_ai is the virtual-occupied block.
    """
    n = h.shape[0]
    v = n - o
    tt = torch.nn.functional.pad(t1.T, (0, v, o, 0))   # tt[a, i] = t_ai
    X = torch.eye(n, dtype=DT) - tt
    Y = torch.eye(n, dtype=DT) + tt.T
    hh = X @ h @ Y.T
    gg = torch.einsum("pP,PQRS->pQRS", X, g)
    gg = torch.einsum("qQ,pQRS->pqRS", Y, gg)
    gg = torch.einsum("rR,pqRS->pqrS", X, gg)
    gg = torch.einsum("sS,pqrS->pqrs", Y, gg)
    return hh, gg


def residual(t1, t2, h, g):
    """(Omega1[i,a], Omega2[i,j,a,b]) of closed-shell CCSD for (h, g)."""
    o, v = t1.shape
    hh, gg = t1_transform(h, g, t1, o)
    F = fock(hh, gg, o)
    O, V = slice(0, o), slice(o, o + v)
    u = 2.0 * t2 - t2.transpose(2, 3)                   # u_ij^ab = 2t_ij^ab - t_ij^ba

    g_vvov = gg[V, V, O, V]
    g_ooov = gg[O, O, O, V]
    g_ovov = gg[O, V, O, V]
    # singles
    om1 = torch.einsum("kicd,adkc->ia", u, g_vvov)
    om1 = om1 - torch.einsum("klac,kilc->ia", u, g_ooov)
    om1 = om1 + torch.einsum("ikac,kc->ia", u, F[O, V])
    om1 = om1 + F[V, O].T
    # doubles: A2 + B2
    om2 = gg[V, O, V, O].permute(1, 3, 0, 2).clone()
    om2 = om2 + torch.einsum("ijcd,acbd->ijab", t2, gg[V, V, V, V])
    W = gg[O, O, O, O] + torch.einsum("ijcd,kcld->kilj", t2, g_ovov)
    om2 = om2 + torch.einsum("klab,kilj->ijab", t2, W)
    # C2
    Xc = gg[O, O, V, V] - 0.5 * torch.einsum("liad,kdlc->kiac", t2, g_ovov)
    P = -0.5 * torch.einsum("kjbc,kiac->ijab", t2, Xc)
    P = P - torch.einsum("kibc,kjac->ijab", t2, Xc)
    # D2
    L_voov = 2.0 * gg[V, O, O, V] - gg[V, V, O, O].permute(0, 3, 2, 1)
    L_ovov = 2.0 * g_ovov - g_ovov.permute(0, 3, 2, 1)
    Xd = L_voov + 0.5 * torch.einsum("ilad,ldkc->aikc", u, L_ovov)
    P = P + 0.5 * torch.einsum("jkbc,aikc->ijab", u, Xd)
    # E2
    Ev = F[V, V] - torch.einsum("klbd,ldkc->bc", u, g_ovov)
    Eo = F[O, O] + torch.einsum("ljcd,kdlc->kj", u, g_ovov)
    P = P + torch.einsum("ijac,bc->ijab", t2, Ev)
    P = P - torch.einsum("ikab,kj->ijab", t2, Eo)
    om2 = om2 + P + P.permute(1, 0, 3, 2)
    return om1, om2


def energy(t1, t2, h, g):
    """E = <HF| exp(-T) H exp(T) |HF> (total electronic energy, no nuclei)."""
    o, v = t1.shape
    hh, gg = t1_transform(h, g, t1, o)
    O, V = slice(0, o), slice(o, o + v)
    e_ref = 2.0 * torch.einsum("ii->", hh[O, O])
    e_ref = e_ref + 2.0 * torch.einsum("iijj->", gg[O, O, O, O])
    e_ref = e_ref - torch.einsum("ijji->", gg[O, O, O, O])
    g_ovov = gg[O, V, O, V]
    L = 2.0 * g_ovov - g_ovov.permute(0, 3, 2, 1)
    return e_ref + torch.einsum("ijab,iajb->", t2, L)


# ---------------------------------------------------------------- packing
def pair_index(o: int, v: int):
    iu = np.triu_indices(o * v)
    return torch.as_tensor(iu[0]), torch.as_tensor(iu[1])


def pack(t1, t2):
    """Singles (i*v + a) then unique doubles (P <= Q, P = i*v + a)."""
    o, v = t1.shape
    X = t2.permute(0, 2, 1, 3).reshape(o * v, o * v)
    r, c = pair_index(o, v)
    return torch.cat([t1.reshape(-1), X[r, c]])


def unpack(x, o: int, v: int):
    nov = o * v
    t1 = x[:nov].reshape(o, v)
    r, c = pair_index(o, v)
    X = torch.zeros((nov, nov), dtype=DT)
    X = X.index_put((r, c), x[nov:])
    X = X + X.T - torch.diag(torch.diag(X))
    t2 = X.reshape(o, v, o, v).permute(0, 2, 1, 3)
    return t1, t2


def dim(o: int, v: int) -> int:
    nov = o * v
    return nov + nov * (nov + 1) // 2


def dot_bio(x, y):
    """Biorthonormal inner product sum_mu x_mu y_mu of packed vectors."""
    return torch.dot(x, y)


# ---------------------------------------------------------------- solver
def orbital_denominators(f, o: int):
    eo = torch.diag(f)[:o]
    ev = torch.diag(f)[o:]
    d1 = ev[None, :] - eo[:, None]
    d2 = (ev[None, None, :, None] + ev[None, None, None, :]
          - eo[:, None, None, None] - eo[None, :, None, None])
    return d1, d2


def solve_ground(h, g, o: int, tol: float = 1e-11, maxit: int = 200,
                 diis_dim: int = 8, t_init=None):
    """Jacobi steps t <- t - Omega/D accelerated by DIIS, from t = 0 (MP2 first).

    Returns (t1, t2, E, iterations).  Raises if not converged.
    """
    h = as_t(h)
    g = as_t(g)
    n = h.shape[0]
    v = n - o
    f = fock(h, g, o)
    d1, d2 = orbital_denominators(f, o)
    if t_init is None:
        t1 = torch.zeros((o, v), dtype=DT)
        t2 = torch.zeros((o, o, v, v), dtype=DT)
    else:
        t1, t2 = (as_t(x).clone() for x in t_init)
    vecs, errs = [], []
    for it in range(1, maxit + 1):
        om1, om2 = residual(t1, t2, h, g)
        err = max(float(om1.abs().max()), float(om2.abs().max()))
        if err < tol:
            return t1, t2, float(energy(t1, t2, h, g)), it
        t1 = t1 - om1 / d1
        t2 = t2 - om2 / d2
        vecs.append(torch.cat([t1.reshape(-1), t2.reshape(-1)]))
        errs.append(torch.cat([(om1 / d1).reshape(-1), (om2 / d2).reshape(-1)]))
        if len(vecs) > diis_dim:
            vecs.pop(0)
            errs.pop(0)
        m = len(vecs)
        if m >= 2:
            Bm = torch.zeros((m + 1, m + 1), dtype=DT)
            E = torch.stack(errs)
            Bm[:m, :m] = E @ E.T
            Bm[:m, m] = -1.0
            Bm[m, :m] = -1.0
            rhs = torch.zeros(m + 1, dtype=DT)
            rhs[m] = -1.0
            c = torch.linalg.lstsq(Bm, rhs.unsqueeze(1)).solution.squeeze(1)[:m]
            x = c @ torch.stack(vecs)
            t1 = x[: o * v].reshape(o, v)
            t2 = x[o * v:].reshape(o, o, v, v)
            t2 = 0.5 * (t2 + t2.permute(1, 0, 3, 2))
    raise RuntimeError(f"CCSD not converged in {maxit} iterations (max|Omega|={err:.3e})")
