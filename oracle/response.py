"""EOM states, Lagrangian multipliers, densities and the derivative coupling.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Every derivative object of the method is taken here from its definition by
automatic differentiation (torch.func, fp64) of the residual and energy in
``oracle.ccsd``:

* Jacobian A_mu,nu = <mu~|[Hbar, tau_nu]|HF> = dOmega_mu/dt_nu (Sec. II B);
* eta_nu = <HF|[Hbar, tau_nu]|HF> = dE/dt_nu, which fixes the reference
  weight R0 = eta.R / omega of a right EOM state;
* F-matrix transform (F(gamma) R)_sigma = d/dt_sigma [gamma . A(t) R] (Sec. II B);
* the orbital-rotation derivatives under H -> exp(kappa) H exp(-kappa)
  (Sec. II A), i.e. integrals rotated by U = exp(K);
* the effective densities as derivatives of the (linear) Hamiltonian
  functional with respect to h and g.

Packed vectors: singles (i*v + a) then unique doubles (P <= Q, P = i*v + a);
the biorthonormal inner product of two packed vectors is their plain dot
product (``ccsd.dot_bio``).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import torch
from torch.func import grad, jvp, vjp, vmap

from . import ccsd, iterative
from .ccsd import DT, as_t


# ------------------------------------------------------------- packed maps
def omega_vec(x, h, g, o, v):
    t1, t2 = ccsd.unpack(x, o, v)
    return ccsd.pack(*ccsd.residual(t1, t2, h, g))


def energy_vec(x, h, g, o, v):
    t1, t2 = ccsd.unpack(x, o, v)
    return ccsd.energy(t1, t2, h, g)


def right_transform(x, R, h, g, o, v):
    """A(t) R."""
    return jvp(lambda y: omega_vec(y, h, g, o, v), (x,), (R,))[1]


def left_transform(x, L, h, g, o, v):
    """L^T A(t)."""
    _, f = vjp(lambda y: omega_vec(y, h, g, o, v), x)
    return f(L)[0]


def eta(x, h, g, o, v):
    return grad(lambda y: energy_vec(y, h, g, o, v))(x)


def dense_jacobian(x, h, g, o, v, chunk: int = 128):
    n = x.numel()
    f = lambda R: right_transform(x, R, h, g, o, v)  # noqa: E731
    cols = []
    I = torch.eye(n, dtype=DT)
    for s in range(0, n, chunk):
        cols.append(vmap(f)(I[s:s + chunk]))
    return torch.cat(cols, 0).T.contiguous()


# ----------------------------------------------------------------- EOM
def gauge_right(R: np.ndarray) -> np.ndarray:
    """dot_bio(R, R) = 1 and the largest-magnitude component positive
    (ties resolved towards the lowest packed index)."""
    R = R / np.linalg.norm(R)
    k = int(np.argmax(np.abs(R)))
    return R if R[k] > 0 else -R


def eom_dense(A: np.ndarray, nroots: int, imag_tol: float = 1e-8):
    """Lowest nroots (by Re omega) right and left eigenpairs of A.

    Returns (omega[nroots], R[nroots, dim], L[nroots, dim]) with R gauged by
    ``gauge_right`` and L biorthonormal to R (L R^T = 1).
    """
    w, vl, vr = scipy.linalg.eig(A, left=True, right=True)
    order = np.argsort(w.real)[:nroots]
    if np.abs(w[order].imag).max() > imag_tol:
        raise ValueError("complex EOM root among the requested states")
    om = w[order].real
    R = np.array([gauge_right(vr[:, k].real) for k in order])
    L = np.array([vl[:, k].real for k in order])
    L = np.linalg.solve(L @ R.T, L)
    return om, R, L


# ------------------------------------------------------- state overlaps
def outer(x1, y1):
    """(x (x) y)_aibj = x_ai y_bj as a [i, j, a, b] tensor."""
    return torch.einsum("ia,jb->ijab", x1, y1)


def overlap(dT, L, R0, R, o, v):
    """<HF| L_i exp(-T0) (R0 + R_j) exp(T0 + dT) |HF> for L0 = 0 (Sec. II A).

    Exact in the CC parameterisation: L holds only single and double
    de-excitations, so only the singles and doubles of
    (R0 + R)(1 + dT + dT^2/2)|HF> contribute.
    """
    d1, d2 = ccsd.unpack(dT, o, v)
    r1, r2 = ccsd.unpack(R, o, v)
    s1 = R0 * d1 + r1
    s2 = R0 * (d2 + outer(d1, d1)) + r2 + outer(d1, r1) + outer(r1, d1)
    return torch.dot(L, ccsd.pack(s1, s2))


def reference_transition_density(x, R0, R, o, v, n):
    """D_pq = <HF| exp(-T) E_pq (R0 + R) exp(T) |HF> (the reference row of a
    bra, L0 = 1): R0 E(h1) + eta(h1).R for the one-electron operator h1,
    differentiated with respect to h1."""
    g0 = torch.zeros((n, n, n, n), dtype=DT)

    def functional(h1):
        return R0 * energy_vec(x, h1, g0, o, v) + torch.dot(eta(x, h1, g0, o, v), R)

    return grad(functional)(torch.zeros((n, n), dtype=DT))


def transition_density(x, L, R0, R, o, v, n):
    """D_pq = <HF| L exp(-T) E_pq (R0 + R) exp(T) |HF> (L0 = 0).

    With a one-electron operator h1 and Hbar1 = exp(-T) h1 exp(T):
    <L| Hbar1 (R0 + R) |HF> = R0 L.Omega(h1) + L.(A(h1) R) + E(h1) L.R
    + L2 . (R1 (x) Omega1(h1) + Omega1(h1) (x) R1), all linear in h1;
    D is its gradient with respect to h1.
    """
    g0 = torch.zeros((n, n, n, n), dtype=DT)
    r1, _ = ccsd.unpack(R, o, v)
    nov = o * v

    def functional(h1):
        om = omega_vec(x, h1, g0, o, v)
        ar = right_transform(x, R, h1, g0, o, v)
        e1 = energy_vec(x, h1, g0, o, v)
        om1 = om[:nov].reshape(o, v)
        z = torch.zeros((o, v), dtype=DT)
        x2 = ccsd.pack(z, outer(r1, om1) + outer(om1, r1))
        return (R0 * torch.dot(L, om) + torch.dot(L, ar) + e1 * torch.dot(L, R)
                + torch.dot(L, x2))

    return grad(functional)(torch.zeros((n, n), dtype=DT))


# ------------------------------------------------------ orbital rotation
def kappa_matrix(kappa, o, v):
    """K with K_ai = kappa_ai, K_ia = -kappa_ai (kappa[i, a])."""
    lower = torch.nn.functional.pad(kappa.T, (0, v, o, 0))
    return lower - lower.T


def rotate(h, g, kappa, o, v):
    """Integrals of exp(kappa) H exp(-kappa): U h U^T and U^(x4) g, U = exp(K)."""
    U = torch.linalg.matrix_exp(kappa_matrix(kappa, o, v))
    hr = U @ h @ U.T
    gr = torch.einsum("pP,PQRS->pQRS", U, g)
    gr = torch.einsum("qQ,pQRS->pqRS", U, gr)
    gr = torch.einsum("rR,pqRS->pqrS", U, gr)
    gr = torch.einsum("sS,pqrS->pqrs", U, gr)
    return hr, gr


def fock_ai(h, g, o):
    """Brillouin vector F_ai in [i, a] layout."""
    return ccsd.fock(h, g, o)[o:, :o].T


def hf_hessian(h, g, o, v):
    """A^HF[(ai), (bj)] = dF_ai / dkappa_bj at kappa = 0."""
    f = lambda k: fock_ai(*rotate(h, g, k.reshape(o, v), o, v), o).reshape(-1)  # noqa: E731
    k0 = torch.zeros(o * v, dtype=DT)
    I = torch.eye(o * v, dtype=DT)
    cols = vmap(lambda e: jvp(f, (k0,), (e,))[1])(I)
    return cols.T.contiguous()


# ------------------------------------------------------------ multipliers
GROUND = -1   # index of the CC ground state when it is the right state of a pair


def solve_zeta(st: dict, eta_t):
    """zeta with A^T zeta = -eta_t (eq. amplituderelax): a dense solve with
    the dense Jacobian, or GMRES on the left transform for a state solved
    iteratively (``ground_and_eom_iterative``)."""
    o, v, h, g, x = st["o"], st["v"], st["h"], st["g"], st["x"]
    if st.get("iterative"):
        return iterative.krylov_solve(lambda y: left_transform(x, y, h, g, o, v), -eta_t,
                                      iterative.orbital_diagonal(h, g, o), tol=st["lin_tol"])
    A = st.get("A")
    if A is None:
        A = dense_jacobian(x, h, g, o, v)
        st["A"] = A
    return torch.linalg.solve(A.T, -eta_t)


def solve_kappa(st: dict, eta_k):
    """kappa_bar with (A^HF)^T kappa_bar = -eta_kappa (eq. orbitalrelax): a
    dense solve with the orbital Hessian, or, for a state solved iteratively,
    GMRES on its transpose applied by a reverse derivative of F_ai through the
    orbital rotation."""
    o, v, h, g = st["o"], st["v"], st["h"], st["g"]
    if st.get("iterative"):
        f = lambda k: fock_ai(*rotate(h, g, k.reshape(o, v), o, v), o).reshape(-1)  # noqa: E731
        _, pull = vjp(f, torch.zeros(o * v, dtype=DT))
        f0 = ccsd.fock(h, g, o)
        d = (torch.diag(f0)[o:][None, :] - torch.diag(f0)[:o][:, None]).reshape(-1)
        x = iterative.krylov_solve(lambda y: pull(y)[0], -eta_k.reshape(-1), d, tol=st["lin_tol"])
        return x.reshape(o, v)
    AHF = st.get("AHF")
    if AHF is None:
        AHF = hf_hessian(h, g, o, v)
        st["AHF"] = AHF
    return torch.linalg.solve(AHF.T, -eta_k.reshape(-1)).reshape(o, v)


def ground_left(st: dict):
    """Lambda of the ground-state left state <psi_0^L| = <HF| (1 + Lambda)
    exp(-T): the left eigenvector of the Jacobian bordered by the reference
    row [[0, eta], [0, A]] with eigenvalue 0, (1, Lambda), so that
    A^T Lambda = -eta (Sec. II C, eq. nac with i = 0).  Cached in st."""
    if "Lambda" not in st:
        st["Lambda"] = solve_zeta(st, eta(st["x"], st["h"], st["g"], st["o"], st["v"]))
    return st["Lambda"]


def right_state(st: dict, j: int):
    """(omega_j, R0_j, R_j) of the right state j of a pair.  The ground state
    exp(T)|HF> (Sec. II C, j = 0) has R0 = 1, R = 0 and no EOM condition, so
    every gamma term of the Lagrangian vanishes with it."""
    if j == GROUND:
        return 0.0, 1.0, torch.zeros_like(st["x"])
    return st["omega"][j], st["R0"][j], st["R"][j]


def lagrangian_hamiltonian_part(x, gamma, zeta, Rj, h, g, o, v, gamma0=0.0):
    """gamma . A(t; h, g) R_j + zeta . Omega(t; h, g) (+ gamma0 eta(t; h, g).R_j,
    the reference row of the excited-state condition, for a ground-state bra)."""
    val = (torch.dot(gamma, right_transform(x, Rj, h, g, o, v))
           + torch.dot(zeta, omega_vec(x, h, g, o, v)))
    if gamma0:
        val = val + gamma0 * torch.dot(eta(x, h, g, o, v), Rj)
    return val


def multipliers(st: dict, i: int, j: int, relaxed: bool = True) -> dict:
    """Multipliers of the ordered pair (i, j): i != j excited, j = GROUND
    (i excited), or i = GROUND (j excited).

    gamma = L_i/(omega_j - omega_i) and xi = -omega_j gamma.R_j (Sec. II B);
    t-stationarity A^T zeta = -eta_t with
    eta_t = d/dt <L_i| exp(-T0) (R0 + R_j) exp(T) |HF> + F(gamma) R_j;
    kappa-stationarity (A^HF)^T kappa_bar = -eta_kappa with
    eta_kappa = d/dkappa [O + zeta.Omega + gamma.(A R_j)] under
    H -> exp(kappa) H exp(-kappa) and |psi_j^R> -> exp(-kappa) |psi_j^R>.

    i = GROUND: the bra is <HF| (1 + Lambda) exp(-T) (``ground_left``,
    omega_0 = 0).  Its reference weight makes R0_j enter the overlap, so the
    excited-state condition keeps its reference row eta.R_j - omega_j R0_j,
    whose multiplier is gamma0 = 1/omega_j (stationarity in R0_j); gamma =
    Lambda/omega_j then satisfies the R_j condition because Lambda A = -eta,
    and xi = -(R0_j + Lambda.R_j) = -<psi_0^L|psi_j^R> = 0.
    """
    o, v, h, g, x = st["o"], st["v"], st["h"], st["g"], st["x"]
    n = o + v
    om, L = st["omega"], st["L"]
    wj, R0j, Rj = right_state(st, j)
    if i == GROUND:
        Li, wi = ground_left(st), 0.0
        gamma0 = 1.0 / wj
    else:
        Li, wi = L[i], om[i]
        gamma0 = 0.0
    gamma = torch.zeros_like(Li) if j == GROUND else Li / (wj - wi)
    xi = -wj * (torch.dot(gamma, Rj) + gamma0 * R0j)
    # eta_t
    zero = torch.zeros_like(x)
    eta_o = grad(lambda d: overlap(d, Li, R0j, Rj, o, v))(zero)
    eta_f = grad(lambda y: lagrangian_hamiltonian_part(
        y, gamma, torch.zeros_like(y), Rj, h, g, o, v, gamma0))(x)
    eta_t = eta_o + eta_f
    zeta = solve_zeta(st, eta_t)
    out = dict(gamma=gamma, gamma0=gamma0, xi=xi, eta_t=eta_t, eta_t_overlap=eta_o, zeta=zeta)
    D = transition_density(x, Li, R0j, Rj, o, v, n)
    if i == GROUND:
        D = D + reference_transition_density(x, R0j, Rj, o, v, n)
    out["D"] = D
    if relaxed:
        k1 = -(D[o:, :o].T - D[:o, o:])
        k0 = torch.zeros((o, v), dtype=DT)
        k23 = grad(lambda k: lagrangian_hamiltonian_part(
            x, gamma, zeta, Rj, *rotate(h, g, k, o, v), o, v, gamma0))(k0)
        eta_k = k1 + k23
        kbar = solve_kappa(st, eta_k)
        out.update(eta_kappa=eta_k, eta_kappa_overlap=k1, kappa_bar=kbar)
    else:
        out["kappa_bar"] = torch.zeros((o, v), dtype=DT)
    return out


# ----------------------------------------------------------- coupling
def coupling_direct(st: dict, mult: dict, j: int, dh, dg) -> float:
    """F^q = gamma.(A(t; H^q) R_j) + zeta.Omega(t; H^q) + kappa_bar.F^q_ai (Sec. II C),
    plus gamma0 eta(t; H^q).R_j for a ground-state bra."""
    o, v, x = st["o"], st["v"], st["x"]
    dh, dg = as_t(dh), as_t(dg)
    val = lagrangian_hamiltonian_part(x, mult["gamma"], mult["zeta"], right_state(st, j)[2],
                                      dh, dg, o, v, mult.get("gamma0", 0.0))
    val = val + torch.sum(mult["kappa_bar"] * fock_ai(dh, dg, o))
    return float(val)


def effective_densities(st: dict, mult: dict, j: int):
    """(D_eff[n,n], d_eff[n,n,n,n]) with F^q = sum D_eff dh + 1/2 sum d_eff dg.

    Gradient of the Hamiltonian-linear part of the Lagrangian,
    gamma.A(t;h,g)R_j + zeta.Omega(t;h,g) + kappa_bar.F_ai(h,g), with respect
    to h and g; d_eff is symmetrised over the 8-fold permutation group of
    real two-electron integrals.
    """
    o, v, x = st["o"], st["v"], st["x"]
    n = o + v

    def functional(h, g):
        val = lagrangian_hamiltonian_part(x, mult["gamma"], mult["zeta"],
                                          right_state(st, j)[2], h, g, o, v,
                                          mult.get("gamma0", 0.0))
        return val + torch.sum(mult["kappa_bar"] * fock_ai(h, g, o))

    h0 = torch.zeros((n, n), dtype=DT)
    g0 = torch.zeros((n, n, n, n), dtype=DT)
    Dh, Dg = grad(functional, argnums=(0, 1))(h0, g0)
    Dh = 0.5 * (Dh + Dh.T)
    d = 2.0 * Dg
    d = 0.5 * (d + d.permute(2, 3, 0, 1))
    d = 0.5 * (d + d.permute(1, 0, 2, 3))
    d = 0.5 * (d + d.permute(0, 1, 3, 2))
    return Dh, d


def coupling_from_densities(D, d, dh, dg) -> float:
    return float(torch.sum(D * as_t(dh)) + 0.5 * torch.sum(d * as_t(dg)))


# ------------------------------------------ state energies and their gradients
def energy_lagrangian_part(x, Lj, zeta, Rj, h, g, o, v):
    """E0(t; h, g) + L_j . A(t; h, g) R_j + zeta . Omega(t; h, g); the L_j term
    is absent for the ground state (Lj None).  At the solution this equals
    E_j = E0 + omega_j, because L_j . R_j = 1 and A R_j = omega_j R_j."""
    val = energy_vec(x, h, g, o, v) + torch.dot(zeta, omega_vec(x, h, g, o, v))
    if Lj is not None:
        val = val + torch.dot(Lj, right_transform(x, Rj, h, g, o, v))
    return val


def gradient_multipliers(st: dict, j: int, relaxed: bool = True) -> dict:
    """Multipliers of the energy of state j (j = GROUND: E0; else E0 + omega_j)
    as a Lagrangian in the same stationarity conditions as the coupling
    (Sec. II B): A^T zeta = -(dE0/dt + d/dt [L_j . A(t) R_j]) and
    (A^HF)^T kappa_bar = -d/dkappa [E0 + L_j . A R_j + zeta . Omega]."""
    o, v, h, g, x = st["o"], st["v"], st["h"], st["g"], st["x"]
    if j == GROUND:
        Lj = Rj = None
        eta_t = eta(x, h, g, o, v)
    else:
        Lj, Rj = st["L"][j], st["R"][j]
        eta_t = eta(x, h, g, o, v) + grad(
            lambda y: torch.dot(Lj, right_transform(y, Rj, h, g, o, v)))(x)
    zeta = solve_zeta(st, eta_t)
    out = dict(L=Lj, R=Rj, eta_t=eta_t, zeta=zeta)
    if relaxed:
        k0 = torch.zeros((o, v), dtype=DT)
        eta_k = grad(lambda k: energy_lagrangian_part(
            x, Lj, zeta, Rj, *rotate(h, g, k, o, v), o, v))(k0)
        kbar = solve_kappa(st, eta_k)
        out.update(eta_kappa=eta_k, kappa_bar=kbar)
    else:
        out["kappa_bar"] = torch.zeros((o, v), dtype=DT)
    return out


def energy_gradient(st: dict, mult: dict, dh, dg) -> float:
    """dE_j/dlam along (dh, dg): the Hamiltonian-linear part of the energy
    Lagrangian evaluated with (dh, dg), plus kappa_bar . F^q_ai."""
    o, v, x = st["o"], st["v"], st["x"]
    dh, dg = as_t(dh), as_t(dg)
    val = energy_lagrangian_part(x, mult["L"], mult["zeta"], mult["R"], dh, dg, o, v)
    return float(val + torch.sum(mult["kappa_bar"] * fock_ai(dh, dg, o)))


def gradient_densities(st: dict, mult: dict):
    """(D[n,n], d[n,n,n,n]) with dE_j/dlam = sum D dh + 1/2 sum d dg."""
    o, v, x = st["o"], st["v"], st["x"]
    n = o + v

    def functional(h, g):
        val = energy_lagrangian_part(x, mult["L"], mult["zeta"], mult["R"], h, g, o, v)
        return val + torch.sum(mult["kappa_bar"] * fock_ai(h, g, o))

    Dh, Dg = grad(functional, argnums=(0, 1))(torch.zeros((n, n), dtype=DT),
                                              torch.zeros((n, n, n, n), dtype=DT))
    Dh = 0.5 * (Dh + Dh.T)
    d = 2.0 * Dg
    d = 0.5 * (d + d.permute(2, 3, 0, 1))
    d = 0.5 * (d + d.permute(1, 0, 2, 3))
    d = 0.5 * (d + d.permute(0, 1, 3, 2))
    return Dh, d


# -------------------------------------------------------------- pipeline
def ground_and_eom(h, g, o: int, nroots: int, tol: float = 1e-11, t_init=None):
    """Solve CCSD and the lowest nroots right/left EOM states (dense)."""
    h, g = as_t(h), as_t(g)
    n = h.shape[0]
    v = n - o
    t1, t2, E0, it = ccsd.solve_ground(h, g, o, tol=tol, t_init=t_init)
    x = ccsd.pack(t1, t2)
    A = dense_jacobian(x, h, g, o, v)
    om, R, L = eom_dense(A.numpy(), nroots)
    R, L = torch.as_tensor(R), torch.as_tensor(L)
    et = eta(x, h, g, o, v)
    R0 = torch.stack([torch.dot(et, R[k]) / om[k] for k in range(nroots)])
    return dict(o=o, v=v, h=h, g=g, x=x, t1=t1, t2=t2, E0=E0, iters=it, A=A,
                omega=torch.as_tensor(om), R=R, L=L, R0=R0, eta=et)


def ground_and_eom_iterative(h, g, o: int, nroots: int, tol: float = 1e-11,
                             eom_tol: float = 1e-10, lin_tol: float = 1e-12):
    """As ``ground_and_eom`` without the dense Jacobian: the right and left
    EOM states by Davidson on the right and left transforms (residual norms
    below eom_tol), gauged and biorthonormalised the same way; the zeta
    equations of the multipliers are then solved by GMRES (relative residual
    lin_tol)."""
    h, g = as_t(h), as_t(g)
    n = h.shape[0]
    v = n - o
    t1, t2, E0, it = ccsd.solve_ground(h, g, o, tol=tol)
    x = ccsd.pack(t1, t2)
    diag = iterative.orbital_diagonal(h, g, o)
    wr, Rr, _ = iterative.davidson(lambda y: right_transform(x, y, h, g, o, v), diag, nroots,
                                   tol=eom_tol)
    wl, Ll, _ = iterative.davidson(lambda y: left_transform(x, y, h, g, o, v), diag, nroots,
                                   tol=eom_tol)
    if np.abs(wr - wl).max() > 1e-8:
        raise RuntimeError("left and right Davidson roots differ")
    R = torch.stack([torch.as_tensor(gauge_right(Rr[k].numpy())) for k in range(nroots)])
    L = torch.linalg.solve(Ll @ R.T, Ll)
    et = eta(x, h, g, o, v)
    R0 = torch.stack([torch.dot(et, R[k]) / wr[k] for k in range(nroots)])
    return dict(o=o, v=v, h=h, g=g, x=x, t1=t1, t2=t2, E0=E0, iters=it, A=None,
                omega=torch.as_tensor(wr), R=R, L=L, R0=R0, eta=et, iterative=True,
                lin_tol=lin_tol)


def system_hamiltonian(eps, B, o):
    """(h, g) of a synthetic system: g from the DF factor, h such that the
    Fock matrix is diag(eps) (canonical Hartree-Fock reference)."""
    g = ccsd.eri_from_factor(B)
    h = ccsd.hamiltonian_from_eps(eps, g, o)
    return h, g
