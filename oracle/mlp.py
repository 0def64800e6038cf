"""Learned initial guess for the doubles amplitudes: plain fp64 reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network is a three-layer perceptron y = W3^T s(W2^T s(W1^T x + b1) + b2)
+ b3 with the SiLU activation s(u) = u / (1 + exp(-u)), weights stored
row-major as W[in][out].  It maps per-element features of a doubles index
(i, j, a, b) to a correction z of the MP2 amplitude:

    t_ij^ab = -((ia|jb) + z_ijab) / D_ijab,   D_ijab = e_a + e_b - e_i - e_j,

so that z = 0 is the first-order (MP2) amplitude that the amplitude solver
reaches in one Jacobi step from t = 0, and z = -D t - (ia|jb) for the
converged CCSD amplitudes.  The loss is half the mean squared error over all
outputs.  Parameters are flattened in the order W1, b1, W2, b2, W3, b3.

The GPU trains the same network with bfloat16-rounded weights; ``bf16``
gives that rounding (nearest, ties to even) so both sides evaluate identical
weights.
"""
from __future__ import annotations

import numpy as np

N_FEATURES = 8


def bf16(x):
    """Round fp32 values to the nearest bfloat16 (ties to even), as fp32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).reshape(a.shape)


def shapes(n_in: int, width: int, n_out: int):
    return [(n_in, width), (width,), (width, width), (width,), (width, n_out), (n_out,)]


def unflatten(p, n_in, width, n_out):
    out, k = [], 0
    for s in shapes(n_in, width, n_out):
        m = int(np.prod(s))
        out.append(np.asarray(p[k:k + m], dtype=np.float64).reshape(s))
        k += m
    return out


def flatten(params):
    return np.concatenate([np.asarray(q, dtype=np.float64).ravel() for q in params])


def silu(u):
    return u / (1.0 + np.exp(-u))


def silu_grad(u):
    sg = 1.0 / (1.0 + np.exp(-u))
    return sg * (1.0 + u * (1.0 - sg))


def forward(params, X):
    """Returns the output [n][n_out] and the pre-activations for backward."""
    W1, b1, W2, b2, W3, b3 = params
    u1 = X @ W1 + b1
    h1 = silu(u1)
    u2 = h1 @ W2 + b2
    h2 = silu(u2)
    y = h2 @ W3 + b3
    return y, (X, u1, h1, u2, h2)


def loss_and_grad(params, X, T):
    """Half mean squared error over all n * n_out outputs and its gradient."""
    W1, b1, W2, b2, W3, b3 = params
    y, (X, u1, h1, u2, h2) = forward(params, X)
    r = y - T
    cnt = r.size
    loss = 0.5 * float(np.sum(r * r)) / cnt
    dy = r / cnt
    gW3 = h2.T @ dy
    gb3 = dy.sum(axis=0)
    dh2 = dy @ W3.T
    du2 = dh2 * silu_grad(u2)
    gW2 = h1.T @ du2
    gb2 = du2.sum(axis=0)
    dh1 = du2 @ W2.T
    du1 = dh1 * silu_grad(u1)
    gW1 = X.T @ du1
    gb1 = du1.sum(axis=0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of the flat parameters, in place."""
    m *= beta1
    m += (1.0 - beta1) * g
    v *= beta2
    v += (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    p -= lr * mh / (np.sqrt(vh) + eps)


# ---------------------------------------------------------------- features
def t2_features(eps, ovov, o: int):
    """Raw features [o*o*v*v][8] of every doubles index (i, j, a, b) in
    row-major order: e_i, e_j, e_a, e_b, D, (ia|jb), (ib|ja), -(ia|jb)/D.
    ovov[i][a][j][b] = (ia|jb)."""
    eps = np.asarray(eps, dtype=np.float64)
    eo, ev = eps[:o], eps[o:]
    v = ev.size
    ei = np.broadcast_to(eo[:, None, None, None], (o, o, v, v))
    ej = np.broadcast_to(eo[None, :, None, None], (o, o, v, v))
    ea = np.broadcast_to(ev[None, None, :, None], (o, o, v, v))
    eb = np.broadcast_to(ev[None, None, None, :], (o, o, v, v))
    D = ea + eb - ei - ej
    g = np.transpose(ovov, (0, 2, 1, 3))          # [i][j][a][b] = (ia|jb)
    k = np.transpose(ovov, (0, 2, 3, 1))          # [i][j][a][b] = (ib|ja)
    F = np.stack([ei, ej, ea, eb, D, g, k, -g / D], axis=-1)
    return F.reshape(-1, N_FEATURES)


def t2_target(t2, eps, ovov, o: int):
    """z = -D t - (ia|jb), flattened like the features."""
    F = t2_features(eps, ovov, o)
    D, g = F[:, 4], F[:, 5]
    return -D * np.asarray(t2, dtype=np.float64).reshape(-1) - g


def t2_from_correction(z, eps, ovov, o: int):
    """Amplitudes t = -((ia|jb) + z) / D as [o][o][v][v]."""
    F = t2_features(eps, ovov, o)
    D, g = F[:, 4], F[:, 5]
    v = np.asarray(eps).size - o
    return (-(g + np.asarray(z, dtype=np.float64).reshape(-1)) / D).reshape(o, o, v, v)
