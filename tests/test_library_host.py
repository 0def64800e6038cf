"""CPU-side checks of the built library: it loads, exports every symbol of
include/nacme.h, and its host-only subspace eigensolver is correct; and the
binding's bf16-pair layout helper."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    from paper_2301_13264_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libnacme.so not built")
    return _lib


def test_header_symbols_exported():
    _lib = _lib_or_skip()
    hdr = open(os.path.join(ROOT, "include", "nacme.h")).read()
    names = set(re.findall(r"^\w[\w\s\*]*?\b(\w+)\s*\(", hdr, flags=re.M))
    names.discard("defined")
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    assert set(_lib.EXPORTED) <= names


def test_host_eigensolver():
    _lib = _lib_or_skip()
    rng = np.random.default_rng(0)
    for m in (1, 2, 5, 17, 40):
        G = rng.normal(size=(m, m)) + np.diag(np.arange(m) * 3.0)
        wr, wi, V = _lib.eig_host(G)
        ref = np.linalg.eigvals(G)
        w = wr + 1j * wi
        assert max(np.min(np.abs(ref - x)) for x in w) < 1e-9
        assert max(np.min(np.abs(w - x)) for x in ref) < 1e-9
        for k in range(m):
            if abs(wi[k]) < 1e-12:
                assert np.abs(G @ V[k] - wr[k] * V[k]).max() < 1e-9 * max(1, abs(wr[k]))


def test_version():
    _lib = _lib_or_skip()
    assert b"gfx950" in _lib.lib().nm_version()


def test_pair_interleave_layout():
    """The bf16-pair operand layout of the GEMM surface: each group of 8 hi
    values of a row is followed by the group's 8 lo values, so element k sits
    at 2 (k - k % 8) + k % 8 (hi) and 8 further (lo)."""
    import torch

    from paper_2301_13264_amd import pair_interleave
    R, K = 3, 32
    hi = torch.arange(R * K, dtype=torch.float32).reshape(R, K)
    lo = -hi - 1
    P = pair_interleave(hi, lo)
    assert tuple(P.shape) == (R, 2 * K)
    for r in range(R):
        for k in range(K):
            assert P[r, 2 * (k - k % 8) + k % 8] == hi[r, k]
            assert P[r, 2 * (k - k % 8) + k % 8 + 8] == lo[r, k]
