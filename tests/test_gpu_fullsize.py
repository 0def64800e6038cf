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
