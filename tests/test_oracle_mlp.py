"""Pins of the learned-guess reference (oracle/mlp.py): gradients by central
finite differences, the activation against scipy's logistic function, the
bfloat16 rounding against torch's conversion, the feature map against the
amplitude solver's MP2 first iterate, and the first Adam step in closed form."""
import numpy as np
import pytest
import torch
from scipy.special import expit

import synth
from oracle import ccsd, mlp
from oracle import response as rs


def _net(n_in, width, n_out, seed):
    rng = np.random.default_rng(seed)
    return [rng.normal(scale=0.7, size=s) for s in mlp.shapes(n_in, width, n_out)]


@pytest.mark.parametrize("n_out", [1, 3])
def test_gradient_matches_central_differences(n_out):
    params = _net(8, 6, n_out, 1)
    rng = np.random.default_rng(2)
    X = rng.normal(size=(5, 8))
    T = rng.normal(size=(5, n_out))
    _, grads = mlp.loss_and_grad(params, X, T)
    g = mlp.flatten(grads)
    p0 = mlp.flatten(params)
    h = 1e-6
    fd = np.zeros_like(p0)
    for k in range(p0.size):
        pp, pm = p0.copy(), p0.copy()
        pp[k] += h
        pm[k] -= h
        lp, _ = mlp.loss_and_grad(mlp.unflatten(pp, 8, 6, n_out), X, T)
        lm, _ = mlp.loss_and_grad(mlp.unflatten(pm, 8, 6, n_out), X, T)
        fd[k] = (lp - lm) / (2 * h)
    assert np.abs(fd - g).max() < 1e-7 * max(1.0, np.abs(g).max())


def test_forward_is_silu_composition():
    """Width-1 identity weights: y = s(s(x)) with s(u) = u * logistic(u)."""
    params = [np.ones((1, 1)), np.zeros(1), np.ones((1, 1)), np.zeros(1), np.ones((1, 1)),
              np.zeros(1)]
    x = np.linspace(-6, 6, 25)[:, None]
    y, _ = mlp.forward(params, x)
    s = x * expit(x)
    ref = s * expit(s)
    assert np.abs(y - ref).max() < 1e-14


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=1000).astype(np.float32),
                        np.float32([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -1 - 2.0 ** -8])])
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16(x), ref)
    assert mlp.bf16(np.float32([1 + 2.0 ** -8]))[0] == 1.0           # tie to even
    assert mlp.bf16(np.float32([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6


def test_zero_correction_is_mp2_first_iterate():
    o, v, naux = 3, 5, 24
    sysd = synth.make_system(o, v, naux, seed=8)
    h, g = rs.system_hamiltonian(sysd["eps"], sysd["B"], o)
    ovov = g[:o, o:, :o, o:].numpy()
    t2 = mlp.t2_from_correction(np.zeros(o * o * v * v), sysd["eps"], ovov, o)
    z1 = torch.zeros((o, v), dtype=torch.float64)
    z2 = torch.zeros((o, o, v, v), dtype=torch.float64)
    _, om2 = ccsd.residual(z1, z2, h, g)
    _, d2 = ccsd.orbital_denominators(ccsd.fock(h, g, o), o)
    assert np.abs(t2 - (-om2 / d2).numpy()).max() < 1e-13
    # round trip through the target map
    t = np.random.default_rng(4).normal(size=(o, o, v, v))
    z = mlp.t2_target(t, sysd["eps"], ovov, o)
    assert np.abs(mlp.t2_from_correction(z, sysd["eps"], ovov, o) - t).max() < 1e-12


def test_first_adam_step_is_signed_lr():
    """With zero moments, the bias-corrected first step is lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p = np.zeros(3)
    m, v = np.zeros(3), np.zeros(3)
    mlp.adam_step(p, g, m, v, 1, 0.01)
    assert np.abs(p - (-0.01 * g / (np.abs(g) + 1e-8))).max() < 1e-15
