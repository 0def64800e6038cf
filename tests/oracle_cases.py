"""Solved oracle states shared by the CPU tests (cached per session)."""
import functools

import numpy as np

import synth
from oracle import response as rs


@functools.lru_cache(maxsize=None)
def solved(o, v, naux=None, nroots=4, seed=None):
    n = o + v
    naux = naux or 3 * n
    seed = synth.exact_check_seed(o, v) if seed is None else seed
    sysd = synth.make_system(o, v, naux, seed)
    h, g = rs.system_hamiltonian(sysd["eps"], sysd["B"], o)
    st = rs.ground_and_eom(h, g, o, nroots)
    st["sys"] = sysd
    return st


def directions(st, ndir=3, seed=777):
    n = st["o"] + st["v"]
    naux = st["sys"]["naux"]
    d = synth.make_directions(n, naux, seed, ndir)
    out = []
    for q in range(ndir):
        dB = d["dB"][q]
        out.append((d["dh"][q], np.einsum("Ppq,Prs->pqrs", dB, dB)))
    return out
