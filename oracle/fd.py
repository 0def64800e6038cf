"""Finite-difference derivative couplings (the plain definition of F_ij).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

F_ij^q = d/dlam <psi_i^L(0)|psi_j^R(lam)> at lam = 0 (Sec. II A, eq. nac),
for H(lam) = (h + lam dh, g + lam dg) in the fixed orbital basis, by central
differences.  The right state at lam is normalised by the Lagrangian's own
constraint <L_j(0)|R_j(lam)> = 1 (Sec. II A); for i != j any smooth
normalisation gives the same derivative because <psi_i^L|psi_j^R> = 0.

* ``fd_unrelaxed``: the reference determinant stays the lam = 0 one; the
  overlap is evaluated exactly in the CC parameterisation.
* ``fd_relaxed``: Hartree-Fock is re-solved at lam (orbital rotation kappa with
  H -> exp(kappa) H exp(-kappa)); the right state
  exp(-kappa) (R0 + R) exp(T) |HF> is built as a CI vector in determinant
  space and projected on the CI bra <HF| L_i exp(-T0).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import torch
from torch.func import jacfwd

from . import ccsd, response
from .ccsd import DT, as_t
from .detspace import DetSpace


def _right_state_at(st, j, h, g, t_init):
    o, v = st["o"], st["v"]
    t1, t2, _, _ = ccsd.solve_ground(h, g, o, tol=1e-12, t_init=t_init)
    x = ccsd.pack(t1, t2)
    if j == response.GROUND:      # exp(T)|HF>, intermediate normalisation
        return t1, t2, x, 1.0, torch.zeros_like(x)
    A = response.dense_jacobian(x, h, g, o, v).numpy()
    w, vr = scipy.linalg.eig(A)
    k = int(np.argmin(np.abs(w - float(st["omega"][j]))))
    R = torch.as_tensor(vr[:, k].real.copy())
    R = R / torch.dot(st["L"][j], R)
    R0 = torch.dot(response.eta(x, h, g, o, v), R) / float(w[k].real)
    return t1, t2, x, R0, R


def richardson(fn, delta):
    """(4 F(delta) - F(2 delta)) / 3: removes the O(delta^2) error of a
    central difference."""
    return (4.0 * fn(delta) - fn(2.0 * delta)) / 3.0


def fd_unrelaxed(st, i, j, dh, dg, delta=1e-4):
    """i = GROUND: the bra <HF| (1 + Lambda) exp(-T0), whose reference part
    projects (R0 + R) exp(T) |HF> on R0."""
    o, v = st["o"], st["v"]
    dh, dg = as_t(dh), as_t(dg)
    Li = response.ground_left(st) if i == response.GROUND else st["L"][i]
    vals = []
    for lam in (delta, -delta):
        h = st["h"] + lam * dh
        g = st["g"] + lam * dg
        _, _, x, R0, R = _right_state_at(st, j, h, g, (st["t1"], st["t2"]))
        val = float(response.overlap(x - st["x"], Li, R0, R, o, v))
        if i == response.GROUND:
            val += float(R0)
        vals.append(val)
    return (vals[0] - vals[1]) / (2.0 * delta)


def solve_hf(h, g, o, v, tol=1e-13, maxit=50):
    """kappa[i, a] with F_ai(exp(kappa) H exp(-kappa)) = 0, by Newton from 0."""
    f = lambda k: response.fock_ai(*response.rotate(h, g, k.reshape(o, v), o, v), o).reshape(-1)  # noqa: E731
    k = torch.zeros(o * v, dtype=DT)
    for _ in range(maxit):
        r = f(k)
        if float(r.abs().max()) < tol:
            return k.reshape(o, v)
        J = jacfwd(f)(k)
        k = k - torch.linalg.solve(J, r)
    raise RuntimeError("Hartree-Fock did not converge")


class CIStates:
    """CI vectors of the CC bra and ket states of a solved system."""

    def __init__(self, st):
        self.st = st
        o, v = st["o"], st["v"]
        self.ds = DetSpace(o + v, o)
        self.M, self.S = self.ds.basis()

    def ket(self, t1, t2, R0, R, kappa=None):
        o, v = self.st["o"], self.st["v"]
        ds = self.ds
        c = ds.exp_excite(t1.numpy(), t2.numpy(), ds.hf())
        r1, r2 = ccsd.unpack(R, o, v)
        c = float(R0) * c + ds.excite(r1.numpy(), r2.numpy(), c)
        if kappa is not None:
            c = ds.exp_kappa(kappa.numpy(), c, sign=-1.0)
        return c

    def bra(self, i):
        """<HF| L_i exp(-T0) as a CI vector; i = GROUND: <HF| (1 + Lambda) exp(-T0)."""
        st, ds = self.st, self.ds
        if i == response.GROUND:
            ell = ds.hf() + ds.dual_vector(response.ground_left(st).numpy(), self.M, self.S)
        else:
            ell = ds.dual_vector(st["L"][i].numpy(), self.M, self.S)
        return ds.exp_excite(st["t1"].numpy(), st["t2"].numpy(), ell, sign=-1.0,
                             transpose=True)

    def ket0(self, j):
        st = self.st
        _, R0, R = response.right_state(st, j)
        return self.ket(st["t1"], st["t2"], R0, R)


def fd_relaxed(st, i, j, dh, dg, delta=1e-4, ci: CIStates | None = None):
    o, v = st["o"], st["v"]
    dh, dg = as_t(dh), as_t(dg)
    ci = ci or CIStates(st)
    b = ci.bra(i)
    vals = []
    for lam in (delta, -delta):
        h = st["h"] + lam * dh
        g = st["g"] + lam * dg
        kappa = solve_hf(h, g, o, v)
        hr, gr = response.rotate(h, g, kappa, o, v)
        t1, t2, _, R0, R = _right_state_at(st, j, hr, gr, (st["t1"], st["t2"]))
        vals.append(float(np.sum(b * ci.ket(t1, t2, R0, R, kappa))))
    return (vals[0] - vals[1]) / (2.0 * delta)


def transition_density_ci(st, i, j, ci: CIStates | None = None):
    """D_pq = <psi_i^L| E_pq |psi_j^R> by brute force on CI vectors."""
    ci = ci or CIStates(st)
    b, c = ci.bra(i), ci.ket0(j)
    n = st["o"] + st["v"]
    D = np.zeros((n, n))
    for p in range(n):
        for q in range(n):
            D[p, q] = np.sum(b * ci.ds.E(p, q, c))
    return D


def hellmann_feynman_two_electron(st, i, j, dh, dg, ci: CIStates | None = None):
    """For exact (o = 1) states: <psi_i^L| H^q |psi_j^R> / (omega_j - omega_i)
    (omega = 0 for the ground state)."""
    ci = ci or CIStates(st)
    b, c = ci.bra(i), ci.ket0(j)
    Hc = ci.ds.H(np.asarray(dh), np.asarray(dg), c)
    wj = response.right_state(st, j)[0]
    wi = 0.0 if i == response.GROUND else float(st["omega"][i])
    return float(np.sum(b * Hc)) / float(wj - wi)


def _state_energy_at(st, j, h, g):
    """E_j = E0 + omega_j (E0 for the ground state) of the system (h, g),
    the root nearest omega_j(0)."""
    o, v = st["o"], st["v"]
    t1, t2, E0, _ = ccsd.solve_ground(h, g, o, tol=1e-12, t_init=(st["t1"], st["t2"]))
    if j == response.GROUND:
        return E0
    x = ccsd.pack(t1, t2)
    w = scipy.linalg.eigvals(response.dense_jacobian(x, h, g, o, v).numpy())
    k = int(np.argmin(np.abs(w - float(st["omega"][j]))))
    return E0 + float(w[k].real)


def fd_energy_gradient(st, j, dh, dg, delta=1e-4, relaxed=True):
    """Central difference of E_j along (dh, dg); relaxed: Hartree-Fock
    re-solved at lam (the energy is invariant to the orbital rotation)."""
    o, v = st["o"], st["v"]
    dh, dg = as_t(dh), as_t(dg)
    vals = []
    for lam in (delta, -delta):
        h = st["h"] + lam * dh
        g = st["g"] + lam * dg
        if relaxed:
            h, g = response.rotate(h, g, solve_hf(h, g, o, v), o, v)
        vals.append(_state_energy_at(st, j, h, g))
    return (vals[0] - vals[1]) / (2.0 * delta)

