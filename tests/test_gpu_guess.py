"""GPU: the learned doubles guess (network kernels and the guess path) against
the fp64 reference in oracle/mlp.py, and what the trained network gains."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp

from gpu_helpers import T, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2301_13264_amd as nm
    return nm


def F32(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda")


@pytest.mark.parametrize("width,n", [(32, 3000), (256, 5000)])
def test_network_forward_gradient_and_adam_match_oracle(nm, width, n):
    say(f"[mlp] width={width} n={n}")
    net = nm.MLP(8, width, 1, seed=3)
    p = net.get_params(working=True)
    assert np.array_equal(p, mlp.bf16(net.get_params(working=False)))
    params = mlp.unflatten(p.astype(np.float64), 8, width, 1)
    rng = np.random.default_rng(width)
    X = rng.normal(size=(n, 8)).astype(np.float32)
    Tt = rng.normal(size=(n, 1)).astype(np.float32)
    Y = torch.zeros((n, 1), dtype=torch.float32, device="cuda")
    net.forward(F32(X), Y)
    yref, _ = mlp.forward(params, X.astype(np.float64))
    assert np.abs(Y.cpu().numpy() - yref).max() < 2e-4 * max(1.0, np.abs(yref).max())
    loss, g = net.loss_grad(F32(X), F32(Tt))
    lref, gref = mlp.loss_and_grad(params, X.astype(np.float64), Tt.astype(np.float64))
    gref = mlp.flatten(gref)
    assert abs(loss - lref) < 1e-4 * lref
    assert np.abs(g - gref).max() < 1e-3 * np.abs(gref).max()
    # first Adam step: zero moments give p - lr g / (|g| + eps)
    pm = net.get_params(working=False)
    net.adam_step(1e-3)
    pm1 = net.get_params(working=False)
    ref = pm - np.float32(1e-3) * g / (np.abs(g) + np.float32(1e-8))
    assert np.abs(pm1 - ref).max() < 1e-6
    assert np.array_equal(net.get_params(working=True), mlp.bf16(pm1))
    net.close()


def _inference_error_bound(params, X):
    """First-order bound on the fused inference's deviation from the fp64
    forward of the same (bfloat16-exact) weights: inputs and both hidden
    activations carried as bfloat16 pairs (2^-17 relative each, 2^-16 taken),
    fp32 accumulation of at most 256 terms (2^-16 relative to the sum of
    magnitudes), the fast SiLU within 2^-20 relative, |s'(u)| <= 1.1."""
    W1, b1, W2, b2, W3, b3 = params
    _, (_, u1, h1, u2, h2) = mlp.forward(params, X)
    aX, ah1, ah2 = np.abs(X), np.abs(h1), np.abs(h2)
    e1 = 2.0 ** -16 * (aX @ np.abs(W1))
    eh1 = 1.1 * e1 + (2.0 ** -16 + 2.0 ** -20) * ah1
    e2 = eh1 @ np.abs(W2) + 2.0 ** -16 * (ah1 @ np.abs(W2))
    eh2 = 1.1 * e2 + 2.0 ** -20 * ah2
    return eh2 @ np.abs(W3) + 2.0 ** -16 * (ah2 @ np.abs(W3))


@pytest.mark.parametrize("n_in,width,n_out,n", [(8, 256, 1, 100003), (5, 96, 3, 4099),
                                                (32, 32, 4, 777), (1, 64, 2, 31), (8, 160, 1, 0)])
def test_fused_inference_matches_oracle(nm, n_in, width, n_out, n):
    """mlp_forward's fused kernel (bf16 matrix cores, no intermediate rows)
    against the fp64 forward: several 32-row tiles and a ragged last tile,
    every width step of the kernel's range, one to four outputs, n = 0."""
    say(f"[mlp fused] {n_in}-{width}-{n_out}, rows {n}")
    net = nm.MLP(n_in, width, n_out, seed=7)
    params = mlp.unflatten(net.get_params(working=True).astype(np.float64), n_in, width, n_out)
    rng = np.random.default_rng(n + width)
    X = rng.normal(size=(n, n_in)).astype(np.float32)
    Y = torch.full((n + 1, n_out), np.nan, dtype=torch.float32, device="cuda")
    net.forward(F32(X), Y[:n])
    torch.cuda.synchronize()
    assert torch.isnan(Y[n:]).all()   # nothing written past the last row
    if n == 0:
        net.close()
        return
    Y = Y[:n]
    yref, _ = mlp.forward(params, X.astype(np.float64))
    bound = _inference_error_bound(params, X.astype(np.float64))
    err = np.abs(Y.cpu().numpy().astype(np.float64) - yref)
    assert np.isfinite(err).all()
    assert (err <= 4.0 * bound + 1e-30).all(), float((err / (bound + 1e-30)).max())
    net.close()


def test_training_fits_a_smooth_target(nm):
    say("[mlp] training")
    rng = np.random.default_rng(5)
    X = rng.normal(size=(20000, 8)).astype(np.float32)
    Tt = (np.sin(X[:, :1]) + 0.5 * X[:, 1:2] * X[:, 2:3]).astype(np.float32)
    net = nm.MLP(8, 256, 1, seed=1)
    Xd, Td = F32(X), F32(Tt)
    l0, _ = net.loss_grad(Xd, Td, want_grad=False)
    net.train(Xd, Td, batch=1024, steps=300, lr=3e-3, seed=2)
    l1, _ = net.loss_grad(Xd, Td, want_grad=False)
    assert l1 < 0.05 * l0
    net.close()


def test_features_and_target_match_oracle(nm):
    """Device features / targets / guess map equal the reference maps."""
    o, v, naux, seed = 3, 5, 24, 11
    sysd = synth.make_system(o, v, naux, seed)
    ctx = nm.Context(o, v, naux, T(sysd["eps"]), T(sysd["B"]))
    ctx.ground()
    g = np.einsum("Ppq,Prs->pqrs", sysd["B"], sysd["B"])
    ovov = g[:o, o:, :o, o:]
    mu = np.linspace(-0.5, 0.5, 8).astype(np.float32)
    sd = np.linspace(0.5, 2.0, 8).astype(np.float32)
    F = torch.zeros((o * o * v * v, 8), dtype=torch.float32, device="cuda")
    ctx.t2_features(F, mu, sd)
    Fref = (mlp.t2_features(sysd["eps"], ovov, o) - mu) / sd
    assert np.abs(F.cpu().numpy() - Fref).max() < 1e-5 * max(1.0, np.abs(Fref).max())
    N = o * v + (o * v) ** 2
    t = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx.export(nm._lib.CC_T, 0, 0, t)
    t2 = t.cpu().numpy()[o * v:]
    Z = torch.zeros(o * o * v * v, dtype=torch.float32, device="cuda")
    ctx.t2_target(Z, 0.01)
    zref = mlp.t2_target(t2, sysd["eps"], ovov, o) / 0.01
    assert np.abs(Z.cpu().numpy() - zref).max() < 1e-5 * max(1.0, np.abs(zref).max())
    ctx.close()


def _ground_iterations(nm, ctx):
    e, it, rc = ctx.ground()
    assert rc == 0, f"ground state not converged after {it} iterations"
    return e, it


def test_learned_guess_cuts_ground_iterations(nm):
    """Perturbed geometries of one system (orbital rotations, scale 0.01):
    a network trained on the converged doubles of 6 of them starts the
    amplitude solver of 2 held-out ones closer to the solution than MP2 does;
    the converged energy is the same."""
    o, v, naux, seed = 4, 12, 48, 2301
    base = synth.make_system(o, v, naux, seed)
    n4 = o * o * v * v
    feats, targs = [], []
    for k in range(6):
        Bk = synth.perturbed_factor(base["B"], 900 + k)
        ctx = nm.Context(o, v, naux, T(base["eps"]), T(Bk))
        ctx.ground()
        F = torch.zeros((n4, 8), dtype=torch.float32, device="cuda")
        Z = torch.zeros(n4, dtype=torch.float32, device="cuda")
        ctx.t2_features(F)
        ctx.t2_target(Z)
        feats.append(F.cpu().numpy())
        targs.append(Z.cpu().numpy())
        ctx.close()
    Fall = np.concatenate(feats)
    Zall = np.concatenate(targs)
    mu = Fall.mean(axis=0)
    sd = Fall.std(axis=0) + 1e-12
    zs = float(Zall.std())
    X = F32((Fall - mu) / sd)
    Y = F32((Zall / zs)[:, None])
    net = nm.MLP(8, 256, 1, seed=4)
    loss = net.train(X, Y, batch=2048, steps=600, lr=2e-3, seed=5)
    say(f"  training loss {loss:.3e} (target variance 0.5)")
    for k in range(2):
        Bk = synth.perturbed_factor(base["B"], 950 + k)
        ctx = nm.Context(o, v, naux, T(base["eps"]), T(Bk))
        e0, it0 = _ground_iterations(nm, ctx)
        ctx.guess_t2(net, mu, sd, zs)
        e1, it1 = _ground_iterations(nm, ctx)
        say(f"  held-out geometry {k}: MP2 start {it0} iterations, learned {it1}")
        assert abs(e1 - e0) < 1e-9
        assert it1 < it0
        ctx.close()
    net.close()


def test_eom_warm_start_from_neighbouring_geometry(nm):
    """EOM starting vectors (cc_set_guess with CC_R / CC_L) taken from the
    states of a neighbouring geometry: the same roots, in fewer iterations
    than the cold start from singles unit vectors."""
    o, v, naux, seed, nroots = 4, 12, 48, 2301, 2
    base = synth.make_system(o, v, naux, seed)
    N = o * v + (o * v) ** 2
    buf = torch.zeros(N, dtype=torch.float64, device="cuda")
    ctx = nm.Context(o, v, naux, T(base["eps"]), T(synth.perturbed_factor(base["B"], 960, scale=1e-3)))
    ctx.ground()
    ctx.eom(nm.CC_BOTH, nroots)
    R = [ctx.export(nm._lib.CC_R, k + 1, 0, buf).clone() for k in range(nroots)]
    L = [ctx.export(nm._lib.CC_L, k + 1, 0, buf).clone() for k in range(nroots)]
    ctx.close()
    ctx = nm.Context(o, v, naux, T(base["eps"]), T(synth.perturbed_factor(base["B"], 961, scale=1e-3)))
    ctx.ground()
    w0, itr0, rc = ctx.eom(nm.CC_RIGHT, nroots)
    assert rc == 0
    wl0, itl0, rc = ctx.eom(nm.CC_LEFT, nroots)
    assert rc == 0
    for k in range(nroots):
        ctx.set_guess(nm._lib.CC_R, k + 1, R[k])
        ctx.set_guess(nm._lib.CC_L, k + 1, L[k])
    w1, itr1, rc = ctx.eom(nm.CC_RIGHT, nroots)
    assert rc == 0
    wl1, itl1, rc = ctx.eom(nm.CC_LEFT, nroots)
    assert rc == 0
    say(f"  right: cold {itr0} iterations, warm {itr1}; left: from R {itl0}, warm {itl1}")
    assert np.abs(np.array(w1) - np.array(w0)).max() < 1e-9
    assert np.abs(np.array(wl1) - np.array(wl0)).max() < 1e-9
    assert itr1 < itr0
    # the guesses are used once: the next solve starts cold again
    w2, itr2, rc = ctx.eom(nm.CC_RIGHT, nroots)
    assert rc == 0 and itr2 > itr1
    with pytest.raises(nm.CCError) as e:
        ctx.set_guess(nm._lib.CC_R, 0, R[0])
    assert e.value.code == -1
    ctx.close()
