"""Shared helpers of the GPU parity tests (layout conversion, device arrays)."""
import functools
import sys

import numpy as np
import torch

import synth
from oracle import ccsd
from oracle import response as rs


def dev():
    return torch.device("cuda:0")


def T(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=dev())


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_full(x_packed, o, v):
    """Oracle packed vector -> library amplitude-shaped vector (numpy)."""
    t1, t2 = ccsd.unpack(torch.as_tensor(np.asarray(x_packed)), o, v)
    return np.concatenate([t1.numpy().ravel(), t2.numpy().ravel()])


def to_packed(y_full, o, v):
    y = np.asarray(y_full)
    nov = o * v
    t1 = torch.as_tensor(y[:nov].reshape(o, v))
    t2 = torch.as_tensor(y[nov:].reshape(o, o, v, v))
    return ccsd.pack(t1, t2).numpy()


@functools.lru_cache(maxsize=None)
def oracle_state(o, v, naux, seed, nroots):
    sysd = synth.make_system(o, v, naux, seed)
    h, g = rs.system_hamiltonian(sysd["eps"], sysd["B"], o)
    st = rs.ground_and_eom(h, g, o, nroots)
    st["sys"] = sysd
    return st
