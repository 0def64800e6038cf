"""The aug-cc-pVDZ-shaped size (o = 33, v = 250, naux = 1100, the synthetic
system and DF scale of `bench.py --workload thymine_adz`).  The oracle cannot
run here within a test's budget (its dense n^4 integrals alone are 51 GB and
one residual takes hours on the host), so the library is checked by
properties that hold at any size: the amplitude equations converge, the
right transform equals a central difference of the residual, the left
transform is its adjoint in the biorthonormal product, and the bf16-pair
operator of the mixed mode stays within its rounding bound."""
import numpy as np
import pytest
import torch

import synth

from gpu_helpers import T, say

pytestmark = pytest.mark.gpu

O, V, NAUX, SEED = 33, 250, 1100, 6301
SIGMA_B = 0.05 * (48 * 12 / (NAUX * V)) ** 0.5
NOV = O * V
N = NOV + NOV * NOV


@pytest.fixture(scope="module")
def nm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_13264_amd as nm
    return nm


def _sym(x):
    """Amplitude-shaped vector with x2[i][j][a][b] = x2[j][i][b][a]."""
    x2 = x[NOV:].view(O, O, V, V)
    x2.copy_(0.5 * (x2 + x2.permute(1, 0, 3, 2)))
    return x


def _dot_bio(x, y):
    """Biorthonormal product of full-layout amplitude vectors: singles, half
    the doubles, plus half the diagonal doubles (the unique pairs once)."""
    x2, y2 = x[NOV:].view(O, O, V, V), y[NOV:].view(O, O, V, V)
    d = torch.einsum("iiaa,iiaa->", x2, y2)
    return float(torch.dot(x[:NOV], y[:NOV]) + 0.5 * torch.dot(x[NOV:], y[NOV:]) + 0.5 * d)


def test_adz_ground_state_and_transform_properties(nm):
    say("[adz] context and ground state")
    sysd = synth.make_system(O, V, NAUX, SEED, sigma_b=SIGMA_B)
    ctx = nm.Context(O, V, NAUX, T(sysd["eps"]), T(sysd["B"]))
    e, it, rc = ctx.ground()
    assert rc == 0 and np.isfinite(e)
    t = ctx.export(nm._lib.CC_T, 0, 0, torch.zeros(N, dtype=torch.float64, device="cuda"))
    om = torch.zeros_like(t)
    ctx.residual(t, om)
    assert float(om.abs().max()) < 1e-10
    g = torch.Generator(device="cuda").manual_seed(17)
    x = _sym(torch.randn(N, dtype=torch.float64, device="cuda", generator=g) * 1e-2)
    y = _sym(torch.randn(N, dtype=torch.float64, device="cuda", generator=g) * 1e-2)
    say("[adz] right transform against a central difference of the residual")
    Ax = torch.zeros(1, N, dtype=torch.float64, device="cuda")
    ctx.apply_jacobian_block(nm.CC_RIGHT, x.view(1, N), Ax)
    eps = 1e-3
    op, omm = torch.zeros_like(t), torch.zeros_like(t)
    ctx.residual(t + eps * x, op)
    ctx.residual(t - eps * x, omm)
    fd = (op - omm) / (2 * eps)
    del op, omm
    # the residual is a quartic polynomial in t: the central difference's
    # error is eps^2 / 6 times third derivatives of the size of the transform
    assert float(torch.linalg.norm(Ax[0] - fd)) < 1e-5 * float(torch.linalg.norm(Ax[0]))
    say("[adz] left transform is the adjoint")
    yA = torch.zeros(1, N, dtype=torch.float64, device="cuda")
    ctx.apply_jacobian_block(nm.CC_LEFT, y.view(1, N), yA)
    lhs, rhs = _dot_bio(y, Ax[0]), _dot_bio(yA[0], x)
    assert abs(lhs - rhs) < 1e-10 * max(abs(lhs), 1e-300) + 1e-14
    say("[adz] bf16-pair operator within its rounding bound")
    Ab = torch.zeros_like(Ax)
    ctx.apply_jacobian_block(nm.CC_RIGHT, x.view(1, N), Ab, precision=nm.CC_BF16X3_REFINE)
    err = float((Ab - Ax).abs().max()) / float(Ax.abs().max())
    assert 0.0 < err < 1e-3
    ctx.close()
