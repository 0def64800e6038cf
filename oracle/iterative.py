"""Iterative eigen- and linear solvers on the oracle's own Jacobian transforms.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

For sizes where the dense Jacobian of ``oracle.response`` no longer fits, the
EOM eigenproblem and the zeta equation (Sec. II A-B) are solved by applying
the oracle's transforms (automatic derivatives of its residual) to vectors.
The paper does not say how these equations are solved; the methods here are
the textbook ones, written plainly and pinned against the dense routes in
``tests/test_oracle_iterative.py``:

* ``davidson`` - Davidson's method for the lowest eigenpairs (by real part)
  of a non-symmetric operator: Rayleigh-Ritz on a growing orthonormal
  subspace (dense eigensolver of the projected matrix each iteration), the
  subspace extended by the residuals divided by (omega - diagonal); no
  restarts.
* ``krylov_solve`` - GMRES (scipy) with a diagonal preconditioner.

Vectors are the oracle's packed vectors, whose biorthonormal inner product is
the plain dot product.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse.linalg as sla
import torch

from . import ccsd
from .ccsd import DT


def orbital_diagonal(h, g, o: int) -> torch.Tensor:
    """Packed orbital-energy differences e_a - e_i (singles) and
    e_a + e_b - e_i - e_j (doubles) from the Fock diagonal."""
    f = ccsd.fock(h, g, o)
    d1, d2 = ccsd.orbital_denominators(f, o)
    return ccsd.pack(d1, d2)


def davidson(apply, diag, nroots: int, tol: float = 1e-10, maxit: int = 400,
             extra: int = 2, imag_tol: float = 1e-8):
    """Lowest nroots eigenpairs (by real part) of the operator x -> apply(x).

    diag: diagonal used to precondition (torch vector of the problem's
    length).  Returns (omega[nroots], X[nroots, dim]) with unit-norm columns.
    Converged when every wanted residual norm ||A x - omega x|| < tol.
    """
    dim = diag.numel()
    nb = min(dim, nroots + extra)
    order = torch.argsort(diag)
    V = []
    for k in range(nb):
        e = torch.zeros(dim, dtype=DT)
        e[order[k]] = 1.0
        V.append(e)
    W = [apply(x) for x in V]
    for it in range(1, maxit + 1):
        Vm, Wm = torch.stack(V), torch.stack(W)
        G = (Vm @ Wm.T).numpy()               # G[a, b] = <V_a, A V_b>
        w, Y = scipy.linalg.eig(G)
        idx = np.argsort(w.real)[:nroots]
        # a complex Ritz pair of a poor subspace is expanded by the residual of
        # its real part; converged wanted roots are real (small real residual)
        cplx = np.abs(w[idx].imag).max() > imag_tol * max(1.0, np.abs(w[idx].real).max())
        omega = w[idx].real
        X, new = [], []
        worst = 0.0
        for k, col in enumerate(idx):
            y = torch.as_tensor(Y[:, col].real.copy())
            x = y @ Vm
            r = y @ Wm - omega[k] * x
            rn = float(torch.linalg.norm(r)) / float(torch.linalg.norm(x))
            worst = max(worst, rn)
            X.append(x / torch.linalg.norm(x))
            if rn >= tol:
                den = omega[k] - diag
                den = torch.where(den.abs() < 1e-8, torch.full_like(den, 1e-8), den)
                new.append(r / den)
        if worst < tol and not cplx:
            return omega, torch.stack(X), it
        added = 0
        for c in new:
            n0 = float(torch.linalg.norm(c))
            for _ in range(2):                   # Gram-Schmidt, twice
                c = c - (torch.stack(V) @ c) @ torch.stack(V)
            n1 = float(torch.linalg.norm(c))
            if n1 > 1e-10 * n0 and n1 > 1e-300:
                V.append(c / n1)
                W.append(apply(V[-1]))
                added += 1
        if added == 0:
            break
    if cplx:
        raise ValueError("complex EOM root among the requested states")
    raise RuntimeError(f"Davidson not converged (residual {worst:.3e})")


def krylov_solve(apply, b, diag, tol: float = 1e-12, maxit: int = 400):
    """x with apply(x) = b by GMRES, preconditioned by x -> x / diag."""
    n = b.numel()
    A = sla.LinearOperator((n, n), matvec=lambda x: apply(torch.as_tensor(x)).numpy(),
                           dtype=np.float64)
    d = diag.numpy()
    M = sla.LinearOperator((n, n), matvec=lambda x: x / d, dtype=np.float64)
    x, info = sla.gmres(A, b.numpy(), rtol=tol, atol=0.0, restart=min(n, 80), maxiter=maxit, M=M)
    if info != 0:
        raise RuntimeError(f"GMRES not converged (info {info})")
    return torch.as_tensor(x)
