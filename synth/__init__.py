"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and nothing else: it holds none of the
coupled-cluster arithmetic (no Fock build, no integral products, no
amplitudes).  Every array it returns is an *input* of the method.

Recipe (stand-in for the paper's thymine / cc-pVDZ and aug-cc-pVDZ workloads,
Sec. IV; no molecular integrals are used):

* orbital energies: occupied ~ U[-1.5, -0.3] Ha, virtual ~ U[0.1, 2.0] Ha,
  each block sorted ascending;
* density-fitting factor B[P, p, q] (Mulliken (pq|rs) = sum_P B[P,p,q] B[P,r,s]):
  upper triangle including the diagonal iid N(0, sigma_B^2), mirrored, so the
  two-electron integrals are positive semi-definite with 8-fold symmetry;
* one perturbation direction q: a one-electron derivative dh^q (symmetric,
  zero diagonal, off-diagonal N(0, 0.1^2)) and a factor dB^q drawn like B,
  which defines the two-electron derivative the same way as g is defined
  from B.

All generators use numpy's PCG64 (``default_rng``) and return float64 host
arrays in C order.
"""
from __future__ import annotations

import numpy as np

OCC_RANGE = (-1.5, -0.3)
VIR_RANGE = (0.1, 2.0)
SIGMA_B = 0.05
SIGMA_DH = 0.1

# Named workloads: (o, v, naux, roots, directions).  Seeds follow
# s0 = 2301 + 1000 k for the k-th named workload.
WORKLOADS = {
    "small": dict(o=4, v=12, naux=48, nroots=2, ndir=1, seed=2301),
    "thymine_dz": dict(o=33, v=127, naux=640, nroots=2, ndir=45, seed=4301),
    "thymine_adz": dict(o=33, v=250, naux=1100, nroots=4, ndir=45, seed=6301),
}


def orbital_energies(o: int, v: int, rng: np.random.Generator) -> np.ndarray:
    occ = np.sort(rng.uniform(OCC_RANGE[0], OCC_RANGE[1], size=o))
    vir = np.sort(rng.uniform(VIR_RANGE[0], VIR_RANGE[1], size=v))
    return np.concatenate([occ, vir]).astype(np.float64)


def symmetric_factor(naux: int, n: int, sigma: float,
                     rng: np.random.Generator) -> np.ndarray:
    """B[P] symmetric n x n, upper triangle (with diagonal) iid N(0, sigma^2)."""
    B = np.zeros((naux, n, n))
    iu = np.triu_indices(n)
    vals = rng.normal(0.0, sigma, size=(naux, iu[0].size))
    B[:, iu[0], iu[1]] = vals
    B[:, iu[1], iu[0]] = vals
    return B


def direction_one_electron(n: int, rng: np.random.Generator,
                           sigma: float = SIGMA_DH) -> np.ndarray:
    """Symmetric, zero-diagonal, off-diagonal N(0, sigma^2)."""
    D = np.zeros((n, n))
    iu = np.triu_indices(n, k=1)
    vals = rng.normal(0.0, sigma, size=iu[0].size)
    D[iu[0], iu[1]] = vals
    D[iu[1], iu[0]] = vals
    return D


def direction_seed(seed: int, q: int) -> int:
    return seed + 10007 * (q + 1)


def make_system(o: int, v: int, naux: int, seed: int,
                sigma_b: float = SIGMA_B) -> dict:
    """Orbital energies and DF factor of one synthetic closed-shell system."""
    rng = np.random.default_rng(seed)
    n = o + v
    eps = orbital_energies(o, v, rng)
    B = symmetric_factor(naux, n, sigma_b, rng)
    return dict(o=o, v=v, naux=naux, eps=eps, B=np.ascontiguousarray(B))


def make_direction(n: int, naux: int, seed: int, q: int, sigma_b: float = SIGMA_B) -> dict:
    """Perturbation direction q (dh^q, dB^q) of the set drawn from seed."""
    rng = np.random.default_rng(direction_seed(seed, q))
    dh = direction_one_electron(n, rng)
    dB = symmetric_factor(naux, n, sigma_b, rng)
    return dict(dh=dh, dB=dB)


def make_directions(n: int, naux: int, seed: int, ndir: int,
                    sigma_b: float = SIGMA_B) -> dict:
    """ndir independent perturbation directions (dh^q, dB^q)."""
    dh = np.zeros((ndir, n, n))
    dB = np.zeros((ndir, naux, n, n))
    for q in range(ndir):
        d = make_direction(n, naux, seed, q, sigma_b)
        dh[q] = d["dh"]
        dB[q] = d["dB"]
    return dict(dh=dh, dB=dB)


def exact_check_seed(o: int, v: int) -> int:
    """Seed of one member of the two-electron / small exact-check set."""
    return 3301 + 100 * v + o


def workload(name: str, ndir: int | None = None, **overrides) -> dict:
    cfg = dict(WORKLOADS[name])
    cfg.update(overrides)
    sysd = make_system(cfg["o"], cfg["v"], cfg["naux"], cfg["seed"],
                       cfg.get("sigma_b", SIGMA_B))
    nd = cfg["ndir"] if ndir is None else ndir
    sysd.update(make_directions(cfg["o"] + cfg["v"], cfg["naux"], cfg["seed"],
                                nd, cfg.get("sigma_b", SIGMA_B)))
    sysd["nroots"] = cfg["nroots"]
    sysd["seed"] = cfg["seed"]
    return sysd


def random_amplitudes(o: int, v: int, seed: int, scale: float = 0.05):
    """Random (t1[o,v], t2[o,o,v,v]) with t2[i,j,a,b] == t2[j,i,b,a]."""
    rng = np.random.default_rng(seed)
    t1 = rng.normal(0.0, scale, size=(o, v))
    t2 = rng.normal(0.0, scale, size=(o, o, v, v))
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    return t1, t2


def random_hamiltonian(n: int, naux: int, seed: int, sigma: float = 0.1):
    """A generic symmetric one-electron matrix and DF factor (no Brillouin
    condition) for residual tests away from canonical HF."""
    rng = np.random.default_rng(seed)
    h = rng.normal(0.0, sigma, size=(n, n))
    h = 0.5 * (h + h.T)
    B = symmetric_factor(naux, n, sigma, rng)
    return h, B


def perturbed_factor(B: np.ndarray, seed: int, scale: float = 0.01) -> np.ndarray:
    """A perturbed geometry of the learned-guess workload: the factor of an
    orbital rotation U = exp(K) of the same system, B[P] -> U^T B[P] U, with
    K antisymmetric and K_pq ~ N(0, scale^2) for p < q.  (A rotation of the
    auxiliary index alone would leave the integrals unchanged.)  The orbital
    energies stay as they are, so the perturbed system is again canonical."""
    from scipy.linalg import expm
    n = B.shape[1]
    rng = np.random.default_rng(seed)
    K = np.zeros((n, n))
    iu = np.triu_indices(n, 1)
    K[iu] = rng.normal(scale=scale, size=iu[0].size)
    K = K - K.T
    U = expm(K)
    out = np.einsum("pq,Ppr,rs->Pqs", U, B, U, optimize=True)
    return np.ascontiguousarray(0.5 * (out + out.transpose(0, 2, 1)))
