"""Pins of the oracle's iterative tier (Davidson and GMRES on its own
transforms) against its dense tier: the same EOM roots and states, the same
multipliers and couplings, on exact-check systems small enough for both."""
import numpy as np
import pytest
import torch

import synth
from oracle import response as rs

from oracle_cases import directions, solved


@pytest.mark.parametrize("o,v", [(1, 10), (3, 9)])
def test_iterative_states_equal_dense_states(o, v):
    st = solved(o, v)
    sysd = st["sys"]
    h, g = rs.system_hamiltonian(sysd["eps"], sysd["B"], o)
    it = rs.ground_and_eom_iterative(h, g, o, nroots=4)
    assert np.abs(it["omega"].numpy() - st["omega"].numpy()).max() < 1e-10
    assert torch.abs(it["R"] - st["R"]).max() < 1e-8
    assert torch.abs(it["L"] - st["L"]).max() < 1e-8
    assert torch.abs(it["L"] @ it["R"].T - torch.eye(4, dtype=torch.float64)).max() < 1e-10
    assert torch.abs(it["R0"] - st["R0"]).max() < 1e-9


@pytest.mark.parametrize("relaxed", [True, False])
def test_iterative_multipliers_and_coupling_equal_dense(relaxed):
    o, v = 3, 9
    st = solved(o, v)
    sysd = st["sys"]
    h, g = rs.system_hamiltonian(sysd["eps"], sysd["B"], o)
    it = rs.ground_and_eom_iterative(h, g, o, nroots=2)
    for (i, j) in [(0, 1), (1, 0)]:
        md = rs.multipliers(st, i, j, relaxed=relaxed)
        mi = rs.multipliers(it, i, j, relaxed=relaxed)
        assert torch.abs(mi["zeta"] - md["zeta"]).max() < 1e-8 * max(1.0, float(md["zeta"].abs().max()))
        assert torch.abs(mi["kappa_bar"] - md["kappa_bar"]).max() < 1e-8
        for dh, dg in directions(st, 2):
            Fd = rs.coupling_direct(st, md, j, dh, dg)
            Fi = rs.coupling_direct(it, mi, j, dh, dg)
            assert abs(Fi - Fd) < 1e-8 * max(1.0, abs(Fd))


def test_davidson_finds_lowest_roots_of_a_known_matrix():
    """A non-symmetric matrix with a known real spectrum (similarity transform
    of a diagonal): the lowest three eigenvalues and their eigenvectors."""
    from oracle import iterative
    rng = np.random.default_rng(4)
    n = 60
    d = np.sort(rng.uniform(0.5, 5.0, size=n))
    S = np.eye(n) + 0.05 * rng.normal(size=(n, n))
    A = S @ np.diag(d) @ np.linalg.inv(S)
    At = torch.as_tensor(A)
    w, X, _ = iterative.davidson(lambda x: At @ x, torch.as_tensor(np.diag(A).copy()), 3, tol=1e-11)
    assert np.abs(w - d[:3]).max() < 1e-10
    for k in range(3):
        assert float(torch.linalg.norm(At @ X[k] - w[k] * X[k])) < 1e-10


def test_krylov_solve_matches_dense_solve():
    from oracle import iterative
    rng = np.random.default_rng(5)
    n = 80
    A = np.diag(rng.uniform(1.0, 3.0, size=n)) + 0.1 * rng.normal(size=(n, n))
    b = rng.normal(size=n)
    At = torch.as_tensor(A)
    x = iterative.krylov_solve(lambda y: At @ y, torch.as_tensor(b), torch.as_tensor(np.diag(A).copy()))
    assert np.abs(x.numpy() - np.linalg.solve(A, b)).max() < 1e-10
