"""Pins of the closed-shell CCSD oracle against its definition
Omega_mu = <mu~| exp(-T) H exp(T) |HF> in determinant space, the MP2 closed
form and two-electron FCI (CCSD is exact for two electrons)."""
import numpy as np
import pytest
import torch

import synth
from oracle import ccsd
from oracle import response as rs
from oracle.detspace import DetSpace, two_electron_fci


def T(x):
    return torch.as_tensor(np.asarray(x), dtype=torch.float64)


@pytest.mark.parametrize("o,v", [(1, 3), (2, 3), (2, 4), (3, 3)])
def test_residual_and_energy_match_definition(o, v):
    """Random non-Brillouin h, random g and random amplitudes."""
    n = o + v
    h, B = synth.random_hamiltonian(n, 2 * n, seed=7 + 10 * o + v, sigma=0.3)
    g = np.einsum("Ppq,Prs->pqrs", B, B)
    t1, t2 = synth.random_amplitudes(o, v, seed=11, scale=0.2)
    ds = DetSpace(n, o)
    E, Om = ds.cc_residual(h, g, t1, t2)
    om1, om2 = ccsd.residual(T(t1), T(t2), T(h), T(g))
    Ec = float(ccsd.energy(T(t1), T(t2), T(h), T(g)))
    assert abs(E - Ec) < 1e-12 * max(1.0, abs(E))
    assert np.abs(Om - ccsd.pack(om1, om2).numpy()).max() < 1e-12


def test_residual_is_linear_in_hamiltonian():
    o, v = 2, 4
    n = o + v
    h1, B1 = synth.random_hamiltonian(n, 2 * n, seed=1)
    h2, B2 = synth.random_hamiltonian(n, 2 * n, seed=2)
    g1, g2 = (np.einsum("Ppq,Prs->pqrs", B, B) for B in (B1, B2))
    t1, t2 = (T(x) for x in synth.random_amplitudes(o, v, seed=3, scale=0.2))
    a = ccsd.pack(*ccsd.residual(t1, t2, T(h1 + 2 * h2), T(g1 + 2 * g2)))
    b = (ccsd.pack(*ccsd.residual(t1, t2, T(h1), T(g1)))
         + 2 * ccsd.pack(*ccsd.residual(t1, t2, T(h2), T(g2))))
    assert torch.abs(a - b).max() < 1e-13


def test_first_iterate_is_mp2():
    """From t = 0 one Jacobi step gives t2 = (ia|jb)/(e_i + e_j - e_a - e_b)
    and t1 = 0 for a canonical Hartree-Fock reference."""
    o, v, naux = 3, 7, 30
    sysd = synth.make_system(o, v, naux, seed=12)
    h, g = rs.system_hamiltonian(sysd["eps"], sysd["B"], o)
    z1 = torch.zeros((o, v), dtype=torch.float64)
    z2 = torch.zeros((o, o, v, v), dtype=torch.float64)
    om1, om2 = ccsd.residual(z1, z2, h, g)
    f = ccsd.fock(h, g, o)
    assert torch.abs(f - torch.diag(T(sysd["eps"]))).max() < 1e-12
    d1, d2 = ccsd.orbital_denominators(f, o)
    t2 = -om2 / d2
    e = T(sysd["eps"])
    eo, ev = e[:o], e[o:]
    mp2 = g[:o, o:, :o, o:].permute(0, 2, 1, 3) / (
        eo[:, None, None, None] + eo[None, :, None, None]
        - ev[None, None, :, None] - ev[None, None, None, :])
    assert torch.abs(om1).max() < 1e-13
    assert torch.abs(t2 - mp2).max() < 1e-13


@pytest.mark.parametrize("v", [3, 5, 8, 12, 20])
def test_ccsd_equals_fci_for_two_electrons(v):
    """Exact-check set: o = 1, naux = 3(o+v); CCSD energy = lowest singlet FCI."""
    o = 1
    n = o + v
    sysd = synth.make_system(o, v, 3 * n, synth.exact_check_seed(o, v))
    h, g = rs.system_hamiltonian(sysd["eps"], sysd["B"], o)
    t1, t2, E, it = ccsd.solve_ground(h, g, o)
    w, _ = two_electron_fci(h.numpy(), g.numpy())
    assert abs(E - w[0]) < 1e-10
