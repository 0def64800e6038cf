"""Pins of the determinant-space layer against operator algebra and a
textbook two-electron Hamiltonian (no working equations involved)."""
import numpy as np
import pytest

import synth
from oracle.detspace import DetSpace, pack, two_electron_fci, unpack


def _rand_ci(ds, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(ds.ns, ds.ns))


def test_excitation_operator_commutator():
    ds = DetSpace(5, 2)
    C = _rand_ci(ds, 1)
    n = ds.n
    rng = np.random.default_rng(2)
    for _ in range(20):
        p, q, r, s = rng.integers(0, n, 4)
        lhs = ds.E(p, q, ds.E(r, s, C)) - ds.E(r, s, ds.E(p, q, C))
        rhs = (q == r) * ds.E(p, s, C) - (p == s) * ds.E(r, q, C)
        assert np.abs(lhs - rhs).max() < 1e-12


def test_number_operator_counts_electrons():
    ds = DetSpace(6, 2)
    C = _rand_ci(ds, 3)
    N = sum(ds.E(p, p, C) for p in range(ds.n))
    assert np.abs(N - 4 * C).max() < 1e-12


def test_hf_energy_with_mulliken_fock():
    """<HF|H|HF> = sum_i (h_ii + f_ii) holds with f_pq = h_pq + sum_k
    (2 g_pqkk - g_pkkq) (Sec. II A Fock matrix, Coulomb/exchange in Mulliken
    order); the printed order (2 g_pkkq - g_pqkk) fails it."""
    o, v = 2, 3
    n = o + v
    h, B = synth.random_hamiltonian(n, 2 * n, seed=5, sigma=0.3)
    g = np.einsum("Ppq,Prs->pqrs", B, B)
    ds = DetSpace(n, o)
    hf = ds.hf()
    e_def = np.sum(hf * ds.H(h, g, hf))
    f = h + 2 * np.einsum("pqkk->pq", g[:, :, :o, :o]) - np.einsum("pkkq->pq", g[:, :o, :o, :])
    f_printed = h + 2 * np.einsum("pkkq->pq", g[:, :o, :o, :]) - np.einsum("pqkk->pq", g[:, :, :o, :o])
    e_fock = sum(h[i, i] + f[i, i] for i in range(o))
    e_bad = sum(h[i, i] + f_printed[i, i] for i in range(o))
    assert abs(e_def - e_fock) < 1e-12
    assert abs(e_def - e_bad) > 1e-3


def test_two_electron_fci_against_generic_determinant_hamiltonian():
    o, v = 1, 4
    n = o + v
    h, B = synth.random_hamiltonian(n, 3 * n, seed=9, sigma=0.3)
    g = np.einsum("Ppq,Prs->pqrs", B, B)
    w, _ = two_electron_fci(h, g)
    ds = DetSpace(n, o)
    full = np.linalg.eigvalsh(ds.hamiltonian_matrix(h, g))
    for e in w:   # every singlet level appears in the M_s = 0 spectrum
        assert np.min(np.abs(full - e)) < 1e-10


@pytest.mark.parametrize("o,v", [(1, 3), (2, 3), (3, 3)])
def test_dual_basis_and_packing(o, v):
    ds = DetSpace(o + v, o)
    M, S = ds.basis()
    assert np.linalg.matrix_rank(S) == S.shape[0]
    dual = np.linalg.solve(S, M.T)
    assert np.abs(dual @ M - np.eye(S.shape[0])).max() < 1e-12
    t1, t2 = synth.random_amplitudes(o, v, seed=4)
    x = pack(t1, t2)
    b1, b2 = unpack(x, o, v)
    assert np.abs(b1 - t1).max() == 0 and np.abs(b2 - t2).max() == 0
    # sum_mu t_mu tau_mu |HF> equals T|HF> with T2 = 1/2 sum t_aibj E_ai E_bj
    assert np.abs(ds.ket_vector(x, M) - ds.excite(t1, t2, ds.hf())).max() < 1e-12
