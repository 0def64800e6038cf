"""GPU parity at the thymine-shaped size the benchmark runs (o = 33, v = 127,
naux = 640, same synthetic system and DF scale as bench.py): the residual and
both Jacobian transforms element by element against the fp64 oracle on the
host, and the EOM states' defining properties (biorthonormality, Rayleigh
quotients equal to the eigenvalues)."""
import numpy as np
import pytest
import torch

import synth
from oracle import ccsd
from oracle import response as rs

from gpu_helpers import T, say, to_full, to_packed

pytestmark = pytest.mark.gpu

O, V, NAUX, SEED = 33, 127, 640, 4301
SIGMA_B = 0.05 * (48 * 12 / (NAUX * V)) ** 0.5


@pytest.fixture(scope="module")
def nm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_13264_amd as nm
    return nm


@pytest.fixture(scope="module")
def system():
    sysd = synth.make_system(O, V, NAUX, SEED, sigma_b=SIGMA_B)
    torch.set_num_threads(16)
    h, g = rs.system_hamiltonian(sysd["eps"], sysd["B"], O)
    return sysd, h, g


def _rel(a, b):
    return float(np.abs(a - b).max() / max(1.0, np.abs(b).max()))


def test_residual_full_size(nm, system):
    sysd, h, g = system
    say("[full size] residual")
    t1, t2 = synth.random_amplitudes(O, V, seed=5, scale=0.01)
    om1, om2 = ccsd.residual(torch.as_tensor(t1), torch.as_tensor(t2), h, g)
    ref = np.concatenate([om1.numpy().ravel(), om2.numpy().ravel()])
    ctx = nm.Context(O, V, NAUX, T(sysd["eps"]), T(sysd["B"]))
    out = torch.zeros(ref.size, dtype=torch.float64, device="cuda")
    ctx.residual(T(np.concatenate([t1.ravel(), t2.ravel()])), out)
    torch.cuda.synchronize()
    assert _rel(out.cpu().numpy(), ref) < 1e-11
    ctx.close()


def test_transforms_and_eom_full_size(nm, system):
    sysd, h, g = system
    say("[full size] ground state and transforms")
    ctx = nm.Context(O, V, NAUX, T(sysd["eps"]), T(sysd["B"]))
    _, _, rc = ctx.ground()
    assert rc == 0
    N = O * V + (O * V) ** 2
    t = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.export(nm._lib.CC_T, 0, 0, t)
    x = torch.as_tensor(to_packed(t.cpu().numpy(), O, V))
    rng = np.random.default_rng(9)
    r = rng.normal(scale=1e-2, size=x.numel())
    y = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.apply_jacobian(nm.CC_RIGHT, T(to_full(r, O, V)), y)
    ref = rs.right_transform(x, torch.as_tensor(r), h, g, O, V).numpy()
    assert _rel(to_packed(y.cpu().numpy(), O, V), ref) < 1e-10
    ctx.apply_jacobian(nm.CC_LEFT, T(to_full(r, O, V)), y)
    ref = rs.left_transform(x, torch.as_tensor(r), h, g, O, V).numpy()
    assert _rel(to_packed(y.cpu().numpy(), O, V), ref) < 1e-10
    say("[full size] low-precision transforms")
    # the solvers' fp32 and bfloat16-pair operators at this size (split-K,
    # cached constant packs, padded K) against the fp64 ones: operand rounding
    # only, and not identical (the low-precision kernels ran)
    X = torch.stack([T(to_full(r, O, V)), T(to_full(rng.normal(scale=1e-2, size=x.numel()), O, V))])
    for side in (nm.CC_RIGHT, nm.CC_LEFT):
        Y64 = torch.zeros_like(X)
        ctx.apply_jacobian_block(side, X, Y64, precision=0)
        scale = Y64.abs().max().item()
        for prec, tol in [(1, 1e-5), (2, 1e-3)]:
            Ylp = torch.zeros_like(X)
            ctx.apply_jacobian_block(side, X, Ylp, precision=prec)
            d = (Ylp - Y64).abs().max().item()
            assert 0.0 < d < tol * scale, (side, prec, d, scale)
    say("[full size] EOM properties")
    w, _, rc = ctx.eom(nm.CC_BOTH, 2)
    assert rc == 0
    R = [to_packed(ctx.export(nm._lib.CC_R, k + 1, 0, y).cpu().numpy(), O, V) for k in range(2)]
    L = [to_packed(ctx.export(nm._lib.CC_L, k + 1, 0, y).cpu().numpy(), O, V) for k in range(2)]
    for k in range(2):
        for l in range(2):
            assert abs(float(L[k] @ R[l]) - (1.0 if k == l else 0.0)) < 1e-8
        ctx.apply_jacobian(nm.CC_RIGHT, T(to_full(R[k], O, V)), y)
        AR = to_packed(y.cpu().numpy(), O, V)
        assert abs(float(L[k] @ AR) - w[k]) < 1e-9
        # right eigen-residual from an independent transform
        assert np.linalg.norm(AR - w[k] * R[k]) < 1e-8
    ctx.close()
    say("[full size] EOM in the bf16-pair mode")
    # the split-precision solver's refined states: same eigenvalues, and the
    # fp64 operator's eigen-residual of its right states meets the same bound
    ctx = nm.Context(O, V, NAUX, T(sysd["eps"]), T(sysd["B"]),
                     nm.default_opts(precision=nm.CC_BF16X3_REFINE))
    _, _, rc = ctx.ground()
    assert rc == 0
    w16, _, rc = ctx.eom(nm.CC_BOTH, 2)
    assert rc == 0
    assert np.abs(np.array(w16) - np.array(w)).max() < 1e-9
    for k in range(2):
        Rk = to_packed(ctx.export(nm._lib.CC_R, k + 1, 0, y).cpu().numpy(), O, V)
        Lk = to_packed(ctx.export(nm._lib.CC_L, k + 1, 0, y).cpu().numpy(), O, V)
        assert abs(float(Lk @ Rk) - 1.0) < 1e-8
        ctx.apply_jacobian(nm.CC_RIGHT, T(to_full(Rk, O, V)), y)
        AR = to_packed(y.cpu().numpy(), O, V)
        assert np.linalg.norm(AR - w16[k] * Rk) < 1e-8
    ctx.close()


# ---------------------------------------------------------------------------
# The coupling of the benchmark workload (bf16 mode, both ordered pairs of the
# two roots, three of its perturbation directions) checked against the
# oracle's own definitions at full size: the oracle cannot run the iterative
# solvers there in test time, so every solution the library returns is put
# into the equation that defines it (Sec. II A-B) with the oracle's operators,
# and the oracle evaluates the coupling by its direct route (Sec. II C) from
# those solutions.  Residuals of the size checked here move F by far less
# than 1e-6 au.
NDIR_CHECK = 3


@pytest.fixture(scope="module")
def coupling_run(nm, system):
    sysd, h, g = system
    say("[full size] coupling run (bf16 mode)")
    dirs = synth.make_directions(O + V, NAUX, SEED, NDIR_CHECK, sigma_b=SIGMA_B)
    ctx = nm.Context(O, V, NAUX, T(sysd["eps"]), T(sysd["B"]),
                     nm.default_opts(precision=nm.CC_BF16X3_REFINE))
    _, _, rc = ctx.ground()
    assert rc == 0
    w, _, rc = ctx.eom(nm.CC_BOTH, 2)
    assert rc == 0
    pairs = [(1, 2), (2, 1)]
    _, rc = ctx.multipliers(pairs)
    assert rc == 0
    N = O * V + (O * V) ** 2
    y = torch.zeros(N, dtype=torch.float64, device="cuda")
    kb = torch.zeros(O * V, dtype=torch.float64, device="cuda")
    pk = lambda t: torch.as_tensor(to_packed(t.cpu().numpy(), O, V))  # noqa: E731
    out = dict(omega=w, x=pk(ctx.export(nm._lib.CC_T, 0, 0, y)),
               R=[pk(ctx.export(nm._lib.CC_R, k + 1, 0, y)) for k in range(2)],
               L=[pk(ctx.export(nm._lib.CC_L, k + 1, 0, y)) for k in range(2)],
               R0=[ctx.export_r0(k + 1) for k in range(2)], dirs=dirs, mult={}, F={})
    for (i, j) in pairs:
        zeta = pk(ctx.export(nm._lib.CC_ZETA, i, j, y))
        # |A^T zeta| (the t-equation's right-hand side norm, a tolerance
        # scale) by the library's left transform, which the transform test
        # above checks element by element against the oracle's
        az = torch.zeros(N, dtype=torch.float64, device="cuda")
        ctx.apply_jacobian(nm.CC_LEFT, T(to_full(zeta.numpy(), O, V)), az)
        out["mult"][(i, j)] = dict(
            zeta=zeta,
            kappa_bar=ctx.export(nm._lib.CC_KAPPA, i, j, kb).cpu().reshape(O, V).clone(),
            gamma=out["L"][i - 1] / (w[j - 1] - w[i - 1]),
            rhs_norm=float(np.linalg.norm(to_packed(az.cpu().numpy(), O, V))))
        ctx.densities(i, j)
        out["F"][(i, j)] = np.asarray(ctx.nacme(i, j, T(dirs["dh"]), T(dirs["dB"])))
    ctx.close()
    return out


def test_full_size_states_satisfy_oracle_equations(nm, system, coupling_run):
    """Amplitude equations, right and left eigen-equations, biorthonormality
    and the reference weight R0 = eta.R / omega with the oracle's residual,
    transforms and eta."""
    _, h, g = system
    r = coupling_run
    say("[full size] oracle: amplitude residual")
    x = r["x"]
    om = rs.omega_vec(x, h, g, O, V)
    assert float(om.abs().max()) < 1e-9
    say("[full size] oracle: eigen-equations")
    et = rs.eta(x, h, g, O, V)
    for k in range(2):
        Rk, Lk, wk = r["R"][k], r["L"][k], r["omega"][k]
        for l in range(2):
            assert abs(float(Lk @ r["R"][l]) - (1.0 if k == l else 0.0)) < 1e-8
        assert float(torch.linalg.norm(rs.right_transform(x, Rk, h, g, O, V) - wk * Rk)) < 1e-8
        assert float(torch.linalg.norm(rs.left_transform(x, Lk, h, g, O, V) - wk * Lk)) < 1e-8
        assert abs(float(et @ Rk) / wk - r["R0"][k]) < 1e-9


@pytest.mark.parametrize("pair,check_kappa", [((1, 2), True), ((2, 1), False)])
def test_full_size_multipliers_satisfy_oracle_equations(nm, system, coupling_run, pair, check_kappa):
    """Stationarity of the coupling Lagrangian at the library's multipliers,
    evaluated by the oracle: in t (A^T zeta + eta_t = 0, eq. amplituderelax)
    for both pairs, and in kappa ((A^HF)^T kappa_bar + eta_kappa = 0, eq.
    orbitalrelax) for the first (the oracle's reverse sweep through the
    orbital rotation costs minutes on the host at this size; the second pair
    runs the same code and its kappa-bar reaches the direct-route check)."""
    _, h, g = system
    r = coupling_run
    i, j = pair
    x, m = r["x"], r["mult"][pair]
    Li, Rj, R0j = r["L"][i - 1], r["R"][j - 1], r["R0"][j - 1]
    say(f"[full size] oracle: t-stationarity of pair {pair}")
    zero = torch.zeros_like(x)
    eta_o = torch.func.grad(lambda d: rs.overlap(d, Li, R0j, Rj, O, V))(zero)
    gt = torch.func.grad(lambda y: rs.lagrangian_hamiltonian_part(
        y, m["gamma"], m["zeta"], Rj, h, g, O, V))(x)
    # the solver's tolerance is 1e-9 relative to the norm of the right-hand
    # side eta_t = -A^T zeta
    scale_t = max(1.0, m["rhs_norm"])
    res_t = float(torch.linalg.norm(gt + eta_o))
    say(f"[full size] |dL/dt| = {res_t:.2e} (scale {scale_t:.2e})")
    assert res_t < 1e-8 * scale_t
    if not check_kappa:
        return
    say(f"[full size] oracle: kappa-stationarity of pair {pair}")
    D = rs.transition_density(x, Li, R0j, Rj, O, V, O + V)
    k1 = -(D[O:, :O].T - D[:O, O:])
    k0 = torch.zeros((O, V), dtype=torch.float64)

    def lag_k(k):
        hr, gr = rs.rotate(h, g, k, O, V)
        return (rs.lagrangian_hamiltonian_part(x, m["gamma"], m["zeta"], Rj, hr, gr, O, V)
                + torch.sum(m["kappa_bar"] * rs.fock_ai(hr, gr, O)))

    gk = torch.func.grad(lag_k)(k0)
    # relative to the right-hand side's norm, eta_kappa = -(A^HF)^T kappa_bar
    f_ai = lambda k: rs.fock_ai(*rs.rotate(h, g, k, O, V), O)  # noqa: E731
    _, pull = torch.func.vjp(f_ai, k0)
    scale_k = max(1.0, float(torch.linalg.norm(pull(m["kappa_bar"])[0])))
    res_k = float(torch.linalg.norm(gk + k1))
    say(f"[full size] |dL/dkappa| = {res_k:.2e} (scale {scale_k:.2e})")
    # quantities that vanish only at convergence (L_i . R_j, the eigen-equation
    # residuals, both held to ~1e-9) enter eta_kappa through
    # gamma = L_i / (omega_j - omega_i), amplified by 1/gap (~2e2 at this
    # pair's 0.0046 Ha); kappa-bar reaches F linearly through D_eff, so 1e-7
    # relative here stays far inside the 1e-6 au coupling bound checked below
    assert res_k < 1e-7 * scale_k


def test_full_size_coupling_matches_oracle_direct_route(nm, system, coupling_run):
    """F^q for three directions of pair (1, 2) and the first of pair (2, 1):
    the library's density route and contraction against the oracle's direct
    route (Sec. II C) at the library's multipliers, <= 1e-6 au each."""
    r = coupling_run
    st = dict(o=O, v=V, x=r["x"], omega=torch.as_tensor(r["omega"]), L=r["L"], R=r["R"],
              R0=torch.as_tensor(r["R0"]))
    worst = 0.0
    for q in range(NDIR_CHECK):
        dB = r["dirs"]["dB"][q]
        dg = torch.einsum("Ppq,Prs->pqrs", torch.as_tensor(dB), torch.as_tensor(dB))
        for (i, j), m in r["mult"].items():
            if (i, j) != (1, 2) and q > 0:
                continue
            say(f"[full size] oracle: direct-route coupling, pair {(i, j)} direction {q}")
            Fo = rs.coupling_direct(st, m, j - 1, r["dirs"]["dh"][q], dg)
            worst = max(worst, abs(r["F"][(i, j)][q] - Fo))
            assert abs(r["F"][(i, j)][q] - Fo) < 1e-6, ((i, j), q, r["F"][(i, j)][q], Fo)
        del dg
    say(f"[full size] max |F - F_oracle| = {worst:.2e}")
