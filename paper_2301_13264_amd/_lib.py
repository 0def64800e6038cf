"""ctypes binding of libnacme.so (argument marshalling only).

Device arrays are passed as raw pointers of torch tensors; every step of the
computation runs inside the library.  Importing this module never falls back
to anything else: if the library is missing it raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnacme.so")

CC_OK, CC_NOT_CONVERGED = 0, 1
CC_RIGHT, CC_LEFT, CC_BOTH = 1, 2, 3
CC_FP64, CC_FP32_REFINE = 0, 1
CC_T, CC_R, CC_L, CC_R0, CC_ZETA, CC_KAPPA, CC_D1, CC_ETA_T, CC_ETA_K, CC_DTRANS = range(1, 11)

ERRORS = {-1: "argument", -2: "call order", -3: "HIP", -4: "out of memory",
          -5: "numeric", -6: "complex root"}


class CCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)} error ({code}): {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("relaxed", ctypes.c_int),
                ("tol_ground", ctypes.c_double), ("tol_eom", ctypes.c_double),
                ("tol_mult", ctypes.c_double), ("maxit", ctypes.c_int),
                ("diis_dim", ctypes.c_int), ("davidson_block", ctypes.c_int),
                ("davidson_max", ctypes.c_int), ("mixed_min_flops", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        PI = ctypes.POINTER(ctypes.c_int)
        PD = ctypes.POINTER(ctypes.c_double)
        L64 = ctypes.POINTER(ctypes.c_int64)
        L.cc_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.cc_create.argtypes = [ctypes.POINTER(P), I, I, I, P, P, ctypes.POINTER(Opts), P]
        L.cc_ground.argtypes = [P, PD, PI]
        L.eom_solve.argtypes = [P, I, I, PD, PI]
        L.multipliers.argtypes = [P, I, I, PI]
        L.densities.argtypes = [P, I, I, P]
        L.nacme.argtypes = [P, I, I, I, P, P, PD]
        L.cc_apply_jacobian.argtypes = [P, I, P, P]
        L.cc_residual.argtypes = [P, P, P]
        L.cc_export.argtypes = [P, I, I, I, P]
        L.cc_set_guess.argtypes = [P, I, I, P]
        L.cc_last_error.argtypes = [P]
        L.cc_last_error.restype = ctypes.c_char_p
        L.cc_destroy.argtypes = [P]
        L.cc_destroy.restype = None
        L.nm_contract.argtypes = [ctypes.c_char_p, D, P, L64, P, L64, D, P, L64, I, P]
        L.nm_eig_host.argtypes = [I, PD, PD, PD, PD]
        L.nm_version.restype = ctypes.c_char_p
        L.cc_stats.argtypes = [P, PD, I]
        L.nm_gemm.argtypes = [I, I, I, I, I, I, D, P, ctypes.c_int64, P, ctypes.c_int64, D, P,
                              ctypes.c_int64, P]
        L.nm_gemm.restype = ctypes.c_int
        L.cc_stats.restype = ctypes.c_int
        L.cc_apply_jacobian_block.argtypes = [P, I, I, P, P, I]
        L.cc_apply_jacobian_block.restype = ctypes.c_int
        for name in ("cc_create", "cc_ground", "eom_solve", "multipliers", "densities", "nacme",
                     "cc_apply_jacobian", "cc_residual", "cc_export", "cc_set_guess",
                     "nm_contract", "nm_eig_host"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


EXPORTED = ["cc_default_opts", "cc_create", "cc_ground", "eom_solve", "multipliers",
            "densities", "nacme", "cc_apply_jacobian", "cc_residual", "cc_export",
            "cc_set_guess", "cc_last_error", "cc_destroy", "nm_contract", "nm_eig_host",
            "nm_version", "cc_stats", "nm_gemm", "cc_apply_jacobian_block"]


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().cc_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(t):
    if not t.is_cuda or t.dtype != __import__("torch").float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """One library context (one set of integrals) on one stream."""

    def __init__(self, o, v, naux, eps, B, opts: Opts | None = None, stream=None):
        self.o, self.v, self.naux, self.n = o, v, naux, o + v
        self.N = o * v + (o * v) ** 2
        self._stream = stream
        self._h = ctypes.c_void_p()
        rc = lib().cc_create(ctypes.byref(self._h), o, v, naux, _ptr(eps), _ptr(B),
                             ctypes.byref(opts) if opts is not None else None,
                             _stream_ptr(stream))
        if rc != CC_OK:
            raise CCError(rc, "cc_create failed")

    def _check(self, rc):
        if rc < 0:
            raise CCError(rc, lib().cc_last_error(self._h).decode())
        return rc

    def close(self):
        if self._h:
            lib().cc_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ground(self):
        e = ctypes.c_double()
        it = ctypes.c_int()
        rc = self._check(lib().cc_ground(self._h, ctypes.byref(e), ctypes.byref(it)))
        return e.value, it.value, rc

    def eom(self, side, nroots):
        w = (ctypes.c_double * nroots)()
        it = ctypes.c_int()
        rc = self._check(lib().eom_solve(self._h, side, nroots, w, ctypes.byref(it)))
        return list(w), it.value, rc

    def multipliers(self, i, j):
        it = (ctypes.c_int * 2)()
        rc = self._check(lib().multipliers(self._h, i, j, it))
        return list(it), rc

    def densities(self, i, j, D1=None):
        self._check(lib().densities(self._h, i, j, _ptr(D1) if D1 is not None else None))

    def nacme(self, i, j, dh, dB):
        nq = dh.shape[0]
        F = (ctypes.c_double * nq)()
        self._check(lib().nacme(self._h, i, j, nq, _ptr(dh), _ptr(dB), F))
        return list(F)

    def apply_jacobian(self, side, X, Y):
        self._check(lib().cc_apply_jacobian(self._h, side, _ptr(X), _ptr(Y)))

    def apply_jacobian_block(self, side, X, Y, precision=0):
        """Y[z] = A X[z] (or X[z]^T A) for the k rows of X ([k][N] device)."""
        if X.dim() != 2 or tuple(Y.shape) != tuple(X.shape):
            raise ValueError("X and Y must be [k][N]")
        self._check(lib().cc_apply_jacobian_block(self._h, side, X.shape[0], _ptr(X), _ptr(Y),
                                                  precision))

    def residual(self, t, out):
        self._check(lib().cc_residual(self._h, _ptr(t), _ptr(out)))

    def export(self, what, idx, jdx, out):
        self._check(lib().cc_export(self._h, what, idx, jdx, _ptr(out)))
        return out

    def export_r0(self, k):
        x = ctypes.c_double()
        self._check(lib().cc_export(self._h, CC_R0, k, 0, ctypes.byref(x)))
        return x.value

    def stats(self):
        out = (ctypes.c_double * 7)()
        self._check(lib().cc_stats(self._h, out, 7))
        keys = ["residuals", "right_transforms", "left_transforms", "gemm_flops",
                "peak_bytes", "reserved_bytes", "lowp_flops"]
        return dict(zip(keys, list(out)))

    def set_guess(self, what, idx, src):
        self._check(lib().cc_set_guess(self._h, what, idx, _ptr(src)))


def contract(spec: str, alpha, A, B, beta, C, stream=None, precision=0):
    dims = lambda t: (ctypes.c_int64 * max(t.dim(), 1))(*t.shape)  # noqa: E731
    rc = lib().nm_contract(spec.encode(), alpha, _ptr(A), dims(A), _ptr(B), dims(B), beta,
                           _ptr(C), dims(C), precision, _stream_ptr(stream))
    if rc != CC_OK:
        raise CCError(rc, f"nm_contract({spec})")
    return C


def gemm(precision, A, B, C, alpha=1.0, beta=0.0, stream=None):
    """One matrix-core GEMM launch C = alpha A B + beta C (2-D row-major
    device tensors; A, B float64 for precision 0, float32 for precision 1)."""
    import torch
    want = torch.float64 if precision == 0 else torch.float32
    for t in (A, B):
        if not t.is_cuda or t.dtype != want or not t.is_contiguous():
            raise ValueError("bad GEMM operand")
    M, K = A.shape
    K2, N = B.shape
    if K2 != K or tuple(C.shape) != (M, N):
        raise ValueError("GEMM shape mismatch")
    rc = lib().nm_gemm(precision, 0, 0, M, N, K, alpha, ctypes.c_void_p(A.data_ptr()), K,
                       ctypes.c_void_p(B.data_ptr()), N, beta, _ptr(C), N, _stream_ptr(stream))
    if rc != CC_OK:
        raise CCError(rc, "nm_gemm")
    return C


def eig_host(G):
    import numpy as np
    G = np.ascontiguousarray(G, dtype=np.float64)
    m = G.shape[0]
    wr, wi, V = np.zeros(m), np.zeros(m), np.zeros((m, m))
    pd = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    rc = lib().nm_eig_host(m, pd(G), pd(wr), pd(wi), pd(V))
    if rc != CC_OK:
        raise CCError(rc, "nm_eig_host")
    return wr, wi, V
