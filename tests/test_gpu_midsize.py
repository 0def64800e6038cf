"""GPU parity against a fully independent oracle run at a size beyond the
dense-Jacobian oracle: o = 8, v = 32, naux = 120 (the benchmark's
conditioning, naux sigma_B^2 v held at its o = 4, v = 12, naux = 48 value),
two roots, both ordered pairs, three perturbation directions.  The oracle
solves the ground state by DIIS, the EOM states by Davidson and the
multiplier equations by GMRES on its own transforms; nothing it uses comes
from the library.  Plain fp64 and the bf16-pair mode."""
import functools

import numpy as np
import pytest
import torch

import synth
from oracle import ccsd
from oracle import response as rs

from gpu_helpers import T, say, to_packed

pytestmark = pytest.mark.gpu

O, V = 8, 32
NAUX = 3 * (O + V)
SIGMA_B = 0.05 * (48 * 12 / (NAUX * V)) ** 0.5
SEED = synth.exact_check_seed(O, V)
NDIR, DIR_SEED = 3, 778


@pytest.fixture(scope="module")
def nm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_13264_amd as nm
    return nm


@functools.lru_cache(maxsize=None)
def oracle_run():
    say("[mid size] oracle: ground state, Davidson, multipliers, couplings")
    sysd = synth.make_system(O, V, NAUX, SEED, sigma_b=SIGMA_B)
    dirs = synth.make_directions(O + V, NAUX, DIR_SEED, NDIR, sigma_b=SIGMA_B)
    h, g = rs.system_hamiltonian(sysd["eps"], sysd["B"], O)
    st = rs.ground_and_eom_iterative(h, g, O, nroots=2)
    e_hf = float(ccsd.energy(torch.zeros(O, V, dtype=torch.float64),
                             torch.zeros(O, O, V, V, dtype=torch.float64), h, g))
    out = dict(sys=sysd, dirs=dirs, st=st, e_corr=st["E0"] - e_hf, mult={}, F={})
    dg = [np.einsum("Ppq,Prs->pqrs", dirs["dB"][q], dirs["dB"][q]) for q in range(NDIR)]
    for (i, j) in [(1, 2), (2, 1)]:
        m = rs.multipliers(st, i - 1, j - 1, relaxed=True)
        out["mult"][(i, j)] = m
        out["F"][(i, j)] = np.array([rs.coupling_direct(st, m, j - 1, dirs["dh"][q], dg[q])
                                     for q in range(NDIR)])
    return out


@pytest.mark.parametrize("prec", [0, 2])
def test_midsize_coupling_matches_iterative_oracle(nm, prec):
    ref = oracle_run()
    sysd, dirs, st = ref["sys"], ref["dirs"], ref["st"]
    say(f"[mid size] library, precision {prec}")
    ctx = nm.Context(O, V, NAUX, T(sysd["eps"]), T(sysd["B"]), nm.default_opts(precision=prec))
    e, _, rc = ctx.ground()
    assert rc == 0
    assert abs(e - ref["e_corr"]) < 1e-9
    w, _, rc = ctx.eom(nm.CC_BOTH, 2)
    assert rc == 0
    assert np.abs(np.array(w) - st["omega"].numpy()).max() < 1e-9
    Nf = O * V + (O * V) ** 2
    buf = torch.zeros(Nf, dtype=torch.float64, device="cuda")
    for k in range(2):
        R = to_packed(ctx.export(nm._lib.CC_R, k + 1, 0, buf).cpu().numpy(), O, V)
        L = to_packed(ctx.export(nm._lib.CC_L, k + 1, 0, buf).cpu().numpy(), O, V)
        assert np.abs(R - st["R"][k].numpy()).max() < 1e-7
        assert np.abs(L - st["L"][k].numpy()).max() < 1e-7 * max(1.0, np.abs(L).max())
    _, rc = ctx.multipliers([(1, 2), (2, 1)])
    assert rc == 0
    kb = torch.zeros(O * V, dtype=torch.float64, device="cuda")
    worst = 0.0
    for (i, j), m in ref["mult"].items():
        zeta = to_packed(ctx.export(nm._lib.CC_ZETA, i, j, buf).cpu().numpy(), O, V)
        assert np.abs(zeta - m["zeta"].numpy()).max() < 1e-7 * max(1.0, float(m["zeta"].abs().max()))
        kbar = ctx.export(nm._lib.CC_KAPPA, i, j, kb).cpu().numpy().reshape(O, V)
        assert np.abs(kbar - m["kappa_bar"].numpy()).max() < 1e-7 * max(1.0, float(m["kappa_bar"].abs().max()))
        ctx.densities(i, j)
        F = np.asarray(ctx.nacme(i, j, T(dirs["dh"]), T(dirs["dB"])))
        worst = max(worst, float(np.abs(F - ref["F"][(i, j)]).max()))
        assert np.abs(F - ref["F"][(i, j)]).max() < 1e-7 * max(1.0, np.abs(ref["F"][(i, j)]).max())
    say(f"[mid size] precision {prec}: max |F - F_oracle| = {worst:.2e}")
    assert worst < 1e-6
    ctx.close()
