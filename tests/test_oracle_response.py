"""Pins of the response/coupling oracle: finite differences of the residual,
adjointness, exact two-electron limits, determinant-space brute force of
transition quantities, and finite-difference couplings (the plain definition
F_ij = d/dlam <psi_i^L(0)|psi_j^R(lam)>)."""
import numpy as np
import pytest
import scipy.linalg
import torch

from oracle import ccsd, fd
from oracle import response as rs
from oracle.detspace import two_electron_fci

from oracle_cases import directions, solved


def _rand(n, seed):
    return torch.as_tensor(np.random.default_rng(seed).normal(size=n))


@pytest.mark.parametrize("o,v", [(1, 4), (2, 3)])
def test_jacobian_matches_finite_difference(o, v):
    st = solved(o, v)
    x, h, g = st["x"], st["h"], st["g"]
    R = _rand(x.numel(), 1)
    eps = 1e-5
    fdv = (rs.omega_vec(x + eps * R, h, g, o, v) - rs.omega_vec(x - eps * R, h, g, o, v)) / (2 * eps)
    assert torch.abs(rs.right_transform(x, R, h, g, o, v) - fdv).max() < 1e-8


def test_left_transform_is_adjoint():
    o, v = 2, 3
    st = solved(o, v)
    x, h, g = st["x"], st["h"], st["g"]
    a, b = _rand(x.numel(), 2), _rand(x.numel(), 3)
    lhs = torch.dot(a, rs.right_transform(x, b, h, g, o, v))
    rhs = torch.dot(rs.left_transform(x, a, h, g, o, v), b)
    assert abs(float(lhs - rhs)) < 1e-12 * abs(float(lhs))


@pytest.mark.parametrize("v", [3, 6, 10])
def test_eom_spectrum_is_fci_for_two_electrons(v):
    st = solved(1, v)
    w, _ = two_electron_fci(st["h"].numpy(), st["g"].numpy())
    ev = np.sort(np.linalg.eigvals(st["A"].numpy()).real)
    assert ev.size == w.size - 1
    assert np.abs(ev - (w[1:] - w[0])).max() < 1e-9


@pytest.mark.parametrize("o,v", [(1, 6), (3, 9)])
def test_left_right_biorthonormal_and_eigenvalues_agree(o, v):
    st = solved(o, v)
    A = st["A"].numpy()
    k = st["omega"].numel()
    assert np.abs((st["L"] @ st["R"].T).numpy() - np.eye(k)).max() < 1e-10
    wl = np.sort(scipy.linalg.eigvals(A.T).real)[:k]
    assert np.abs(wl - st["omega"].numpy()).max() < 1e-10
    for m in range(k):
        L, R, w = st["L"][m].numpy(), st["R"][m].numpy(), float(st["omega"][m])
        assert np.abs(A @ R - w * R).max() < 1e-9
        assert np.abs(L @ A - w * L).max() < 1e-9


def test_right_state_is_exact_eigenvector_for_two_electrons():
    """Pins R0 = eta.R/omega: (R0 + R) exp(T)|HF> must be an eigenvector of H."""
    st = solved(1, 5)
    ci = fd.CIStates(st)
    for j in range(st["omega"].numel()):
        c = ci.ket0(j)
        Hc = ci.ds.H(st["h"].numpy(), st["g"].numpy(), c)
        assert np.abs(Hc - (st["E0"] + float(st["omega"][j])) * c).max() < 1e-9


def test_reference_weight_equals_minus_lambda_dot_r():
    o, v = 2, 4
    st = solved(o, v)
    lam = torch.linalg.solve(st["A"].T, -st["eta"])
    for j in range(st["omega"].numel()):
        assert abs(float(st["R0"][j] + torch.dot(lam, st["R"][j]))) < 1e-10


@pytest.mark.parametrize("o,v", [(1, 4), (2, 3)])
def test_transition_quantities_match_ci(o, v):
    st = solved(o, v)
    ci = fd.CIStates(st)
    M = ci.M
    for (i, j) in [(0, 1), (1, 0)]:
        D = rs.transition_density(st["x"], st["L"][i], st["R0"][j], st["R"][j], o, v, o + v)
        assert np.abs(D.numpy() - fd.transition_density_ci(st, i, j, ci)).max() < 1e-12
        m = rs.multipliers(st, i, j, relaxed=False)
        b, c = ci.bra(i), ci.ket0(j)
        # eta_t first term: <psi_i^L| tau_sigma |psi_j^R> (tau_sigma commutes with T)
        brute = []
        for s in range(M.shape[1]):
            e = np.zeros(M.shape[1])
            e[s] = 1.0
            x1, x2 = ccsd.unpack(torch.as_tensor(e), o, v)
            brute.append(np.sum(b * ci.ds.excite(x1.numpy(), x2.numpy(), c)))
        assert np.abs(m["eta_t_overlap"].numpy() - np.array(brute)).max() < 1e-12
        # first singles term of eta_t is the vo block of D (Sec. III A)
        assert torch.abs(m["eta_t_overlap"][: o * v].reshape(o, v) - D[o:, :o].T).max() < 1e-12


def test_f_matrix_is_symmetric():
    o, v = 2, 3
    st = solved(o, v)
    x, h, g = st["x"], st["h"], st["g"]
    gam = _rand(x.numel(), 5)
    a, b = _rand(x.numel(), 6), _rand(x.numel(), 7)

    def F(y):
        return torch.func.grad(lambda z: torch.dot(gam, rs.right_transform(z, y, h, g, o, v)))(x)

    assert abs(float(torch.dot(a, F(b)) - torch.dot(b, F(a)))) < 1e-12 * float(torch.abs(F(b)).max()) * 10


def test_gamma_xi_closed_form():
    st = solved(2, 3)
    for (i, j) in [(0, 1), (1, 2), (2, 0)]:
        m = rs.multipliers(st, i, j, relaxed=False)
        w = st["omega"]
        assert torch.abs(m["gamma"] - st["L"][i] / (w[j] - w[i])).max() == 0
        assert abs(float(m["xi"])) < 1e-12


@pytest.mark.parametrize("v", [3, 7])
def test_orbital_response_vanishes_for_two_electrons(v):
    """o = 1: CCSD is exact for any reference, so kappa-stationarity holds
    with kappa_bar = 0; this fixes the sign of the overlap term of eta_kappa
    relative to the Hamiltonian terms (H -> exp(kappa) H exp(-kappa))."""
    st = solved(1, v)
    for (i, j) in [(0, 1), (1, 0), (0, 2)]:
        m = rs.multipliers(st, i, j, relaxed=True)
        assert float(m["eta_kappa_overlap"].abs().max()) > 1e-3
        assert float(m["eta_kappa"].abs().max()) < 1e-9
        assert float(m["kappa_bar"].abs().max()) < 1e-9


def test_hf_hessian_matches_finite_difference():
    o, v = 2, 4
    st = solved(o, v)
    h, g = st["h"], st["g"]
    AHF = rs.hf_hessian(h, g, o, v)
    k = _rand(o * v, 8).reshape(o, v)
    eps = 1e-5
    fp = rs.fock_ai(*rs.rotate(h, g, eps * k, o, v), o)
    fm = rs.fock_ai(*rs.rotate(h, g, -eps * k, o, v), o)
    fdv = ((fp - fm) / (2 * eps)).reshape(-1)
    assert torch.abs(AHF @ k.reshape(-1) - fdv).max() < 1e-8


@pytest.mark.parametrize("o,v,relaxed", [(2, 3, True), (3, 9, True), (3, 9, False)])
def test_density_route_equals_direct_route(o, v, relaxed):
    st = solved(o, v)
    for (i, j) in [(0, 1), (1, 0)]:
        m = rs.multipliers(st, i, j, relaxed=relaxed)
        D, d = rs.effective_densities(st, m, j)
        for dh, dg in directions(st, 2):
            a = rs.coupling_direct(st, m, j, dh, dg)
            b = rs.coupling_from_densities(D, d, dh, dg)
            assert abs(a - b) < 1e-12 * max(1.0, abs(a))


def test_two_electron_closed_form_coupling():
    """Exact states: F_ij = <psi_i^L|H^q|psi_j^R>/(omega_j - omega_i)."""
    st = solved(1, 6)
    ci = fd.CIStates(st)
    for (i, j) in [(0, 1), (2, 1), (3, 0)]:
        m = rs.multipliers(st, i, j, relaxed=True)
        for dh, dg in directions(st, 2):
            F = rs.coupling_direct(st, m, j, dh, dg)
            assert abs(F - fd.hellmann_feynman_two_electron(st, i, j, dh, dg, ci)) < 1e-9


@pytest.mark.parametrize("o,v", [(1, 3), (1, 10), (1, 20), (3, 9)])
def test_unrelaxed_coupling_matches_finite_difference(o, v):
    """Exact-check set: central difference at lam = +-1e-4, and its Richardson
    extrapolation, which removes the O(lam^2) truncation error that dominates
    for strongly coupled (small-gap) pairs."""
    st = solved(o, v)
    pairs = [(0, 1), (1, 0)] if o == 3 else [(0, 1), (1, 0), (2, 3)]
    for dh, dg in directions(st, 3 if o == 1 else 1):
        for (i, j) in pairs:
            m = rs.multipliers(st, i, j, relaxed=False)
            F = rs.coupling_direct(st, m, j, dh, dg)
            Ffd = fd.fd_unrelaxed(st, i, j, dh, dg, delta=1e-4)
            assert abs(F - Ffd) < 1e-5 * max(1.0, abs(F))
            Fr = fd.richardson(lambda d: fd.fd_unrelaxed(st, i, j, dh, dg, delta=d), 1e-4)
            assert abs(F - Fr) < 1e-7 * max(1.0, abs(F))


@pytest.mark.parametrize("o,v", [(1, 4), (2, 3), (3, 9)])
def test_relaxed_coupling_matches_finite_difference(o, v):
    """Hartree-Fock re-solved along lam; CI vectors in determinant space."""
    st = solved(o, v)
    ci = fd.CIStates(st)
    (dh, dg), = directions(st, 1)
    for (i, j) in [(0, 1), (1, 0)]:
        m = rs.multipliers(st, i, j, relaxed=True)
        F = rs.coupling_direct(st, m, j, dh, dg)
        Fr = fd.richardson(lambda d: fd.fd_relaxed(st, i, j, dh, dg, delta=d, ci=ci), 1e-4)
        assert abs(F - Fr) < 1e-7 * max(1.0, abs(F))


def test_gauge_invariant_product_two_electrons():
    """F_ij F_ji <= 0 for exact states and the same direction."""
    st = solved(1, 8)
    (dh, dg), = directions(st, 1)
    mij = rs.multipliers(st, 0, 1)
    mji = rs.multipliers(st, 1, 0)
    assert rs.coupling_direct(st, mij, 1, dh, dg) * rs.coupling_direct(st, mji, 0, dh, dg) <= 0


# ----------------------------------------------- ground-state right state
GROUND = rs.GROUND


@pytest.mark.parametrize("o,v", [(1, 5), (2, 3), (3, 9)])
def test_ground_pair_zeta_closed_form(o, v):
    """j = ground state: the solved t-multipliers equal -L_i / omega_i
    (= L_i / (E0 - E_i)); only kappa-bar needs a solve."""
    st = solved(o, v)
    for i in range(2):
        m = rs.multipliers(st, i, GROUND, relaxed=True)
        ref = -st["L"][i] / st["omega"][i]
        assert torch.abs(m["zeta"] - ref).max() < 1e-10 * max(1.0, float(ref.abs().max()))
        assert torch.abs(m["gamma"]).max() == 0.0


def test_ground_pair_two_electron_closed_form():
    """Exact states: F_i0 = <psi_i^L|H^q|psi_0^R>/(E0 - E_i), and the orbital
    response vanishes for two electrons."""
    st = solved(1, 6)
    ci = fd.CIStates(st)
    for i in range(3):
        m = rs.multipliers(st, i, GROUND, relaxed=True)
        assert torch.abs(m["kappa_bar"]).max() < 1e-10
        for dh, dg in directions(st, 2):
            F = rs.coupling_direct(st, m, GROUND, dh, dg)
            assert abs(F - fd.hellmann_feynman_two_electron(st, i, GROUND, dh, dg, ci)) < 1e-9


@pytest.mark.parametrize("o,v", [(1, 10), (3, 9)])
def test_ground_pair_unrelaxed_matches_finite_difference(o, v):
    st = solved(o, v)
    (dh, dg), = directions(st, 1)
    for i in range(2):
        m = rs.multipliers(st, i, GROUND, relaxed=False)
        F = rs.coupling_direct(st, m, GROUND, dh, dg)
        Fr = fd.richardson(lambda d: fd.fd_unrelaxed(st, i, GROUND, dh, dg, delta=d), 1e-4)
        assert abs(F - Fr) < 1e-7 * max(1.0, abs(F))


@pytest.mark.parametrize("o,v", [(2, 3), (3, 9)])
def test_ground_pair_relaxed_matches_finite_difference(o, v):
    st = solved(o, v)
    ci = fd.CIStates(st)
    (dh, dg), = directions(st, 1)
    m = rs.multipliers(st, 0, GROUND, relaxed=True)
    F = rs.coupling_direct(st, m, GROUND, dh, dg)
    Fr = fd.richardson(lambda d: fd.fd_relaxed(st, 0, GROUND, dh, dg, delta=d, ci=ci), 1e-4)
    assert abs(F - Fr) < 1e-7 * max(1.0, abs(F))
    D, d = rs.effective_densities(st, m, GROUND)
    assert abs(rs.coupling_from_densities(D, d, dh, dg) - F) < 1e-12 * max(1.0, abs(F))


# ------------------------------------------------ ground-state left state
@pytest.mark.parametrize("o,v", [(1, 6), (2, 3), (3, 9)])
def test_ground_bra_is_left_eigenvector_and_biorthogonal(o, v):
    """(1, Lambda) is the left eigenvector with eigenvalue 0 of the Jacobian
    bordered by the reference row, and the CI bra <HF| (1 + Lambda) exp(-T)
    is biorthonormal to the ground and excited CI kets (brute force in
    determinant space)."""
    st = solved(o, v)
    lam = rs.ground_left(st)
    et = rs.eta(st["x"], st["h"], st["g"], o, v)
    assert torch.abs(st["A"].T @ lam + et).max() < 1e-10 * max(1.0, float(et.abs().max()))
    ci = fd.CIStates(st)
    b = ci.bra(GROUND)
    assert abs(float(np.sum(b * ci.ket0(GROUND))) - 1.0) < 1e-10
    for j in range(st["omega"].numel()):
        assert abs(float(np.sum(b * ci.ket0(j)))) < 1e-9


def test_ground_bra_two_electron_closed_form():
    """Exact states: F_0j = <psi_0^L|H^q|psi_j^R>/(E_j - E0)."""
    st = solved(1, 6)
    ci = fd.CIStates(st)
    for j in range(3):
        m = rs.multipliers(st, GROUND, j, relaxed=True)
        assert torch.abs(m["kappa_bar"]).max() < 1e-10
        assert abs(m["xi"]) < 1e-10
        for dh, dg in directions(st, 2):
            F = rs.coupling_direct(st, m, j, dh, dg)
            assert abs(F - fd.hellmann_feynman_two_electron(st, GROUND, j, dh, dg, ci)) < 1e-9


@pytest.mark.parametrize("o,v", [(1, 10), (3, 9)])
def test_ground_bra_unrelaxed_matches_finite_difference(o, v):
    st = solved(o, v)
    (dh, dg), = directions(st, 1)
    for j in range(2):
        m = rs.multipliers(st, GROUND, j, relaxed=False)
        F = rs.coupling_direct(st, m, j, dh, dg)
        Fr = fd.richardson(lambda d: fd.fd_unrelaxed(st, GROUND, j, dh, dg, delta=d), 1e-4)
        assert abs(F - Fr) < 1e-7 * max(1.0, abs(F))


@pytest.mark.parametrize("o,v", [(2, 3), (3, 9)])
def test_ground_bra_relaxed_matches_finite_difference(o, v):
    st = solved(o, v)
    ci = fd.CIStates(st)
    (dh, dg), = directions(st, 1)
    m = rs.multipliers(st, GROUND, 0, relaxed=True)
    F = rs.coupling_direct(st, m, 0, dh, dg)
    Fr = fd.richardson(lambda d: fd.fd_relaxed(st, GROUND, 0, dh, dg, delta=d, ci=ci), 1e-4)
    assert abs(F - Fr) < 1e-7 * max(1.0, abs(F))
    D, d = rs.effective_densities(st, m, 0)
    assert abs(rs.coupling_from_densities(D, d, dh, dg) - F) < 1e-12 * max(1.0, abs(F))


# ------------------------------------------------ state-energy gradients
@pytest.mark.parametrize("o,v,relaxed", [(1, 6, True), (2, 3, True), (3, 9, True), (3, 9, False)])
def test_energy_gradient_matches_finite_difference(o, v, relaxed):
    """dE_j/dlam of the ground (j = GROUND) and excited states from the
    energy Lagrangian equals the Richardson-extrapolated central difference of
    the re-solved energies; density route = direct route."""
    st = solved(o, v)
    (dh, dg), = directions(st, 1)
    for j in (GROUND, 0, 1):
        m = rs.gradient_multipliers(st, j, relaxed=relaxed)
        G = rs.energy_gradient(st, m, dh, dg)
        Gr = fd.richardson(lambda d: fd.fd_energy_gradient(st, j, dh, dg, delta=d, relaxed=relaxed),
                           1e-4)
        assert abs(G - Gr) < 1e-7 * max(1.0, abs(G))
        D, d = rs.gradient_densities(st, m)
        assert abs(rs.coupling_from_densities(D, d, dh, dg) - G) < 1e-11 * max(1.0, abs(G))


def test_energy_gradient_is_hellmann_feynman_for_two_electrons():
    """CCSD is FCI for two electrons and orbital rotations are redundant:
    dE_j/dlam = <psi_j^L|H^q|psi_j^R> for the (exact) excited and ground states."""
    st = solved(1, 5)
    ci = fd.CIStates(st)
    for dh, dg in directions(st, 2):
        for j in (GROUND, 0, 2):
            m = rs.gradient_multipliers(st, j, relaxed=True)
            G = rs.energy_gradient(st, m, dh, dg)
            c = ci.ket0(j)
            if j == GROUND:
                b = ci.ds.exp_excite(st["t1"].numpy(), st["t2"].numpy(), ci.ds.hf(), sign=-1.0,
                                     transpose=True)
                lam = ci.ds.dual_vector(
                    -torch.linalg.solve(st["A"].T, st["eta"]).numpy(), ci.M, ci.S)
                b = b + ci.ds.exp_excite(st["t1"].numpy(), st["t2"].numpy(), lam, sign=-1.0,
                                         transpose=True)
            else:
                b = ci.bra(j)
            hf = float(np.sum(b * ci.ds.H(np.asarray(dh), np.asarray(dg), c)))
            assert abs(G - hf) < 1e-9 * max(1.0, abs(G))
