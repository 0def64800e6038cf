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
CC_FP64, CC_FP32_REFINE, CC_BF16X3_REFINE = 0, 1, 2
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
        L.multipliers.argtypes = [P, I, PI, PI]
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
        L.nm_gemm_tiled.argtypes = [I, I, I, I, I, I, I, D, P, ctypes.c_int64, P, ctypes.c_int64, D, P,
                                    ctypes.c_int64, P]
        L.nm_gemm_tiled.restype = ctypes.c_int
        L.cc_stats.restype = ctypes.c_int
        L.cc_apply_jacobian_block.argtypes = [P, I, I, P, P, I]
        L.cc_apply_jacobian_block.restype = ctypes.c_int
        PF = ctypes.POINTER(ctypes.c_float)
        F = ctypes.c_float
        U64 = ctypes.c_uint64
        L.mlp_create.argtypes = [ctypes.POINTER(P), I, I, I, U64, P]
        L.mlp_num_params.argtypes = [P]
        L.mlp_num_params.restype = ctypes.c_int64
        L.mlp_dims.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]
        L.mlp_set_params.argtypes = [P, PF]
        L.mlp_get_params.argtypes = [P, PF, I]
        L.mlp_forward.argtypes = [P, ctypes.c_int64, P, P]
        L.mlp_forward_noalloc.argtypes = [P, ctypes.c_int64, P, P]
        L.mlp_loss_grad.argtypes = [P, ctypes.c_int64, P, P, PD, PF]
        L.mlp_adam_step.argtypes = [P, F]
        L.mlp_train.argtypes = [P, ctypes.c_int64, P, P, ctypes.c_int64, I, F, U64, PD]
        L.mlp_last_error.argtypes = [P]
        L.mlp_last_error.restype = ctypes.c_char_p
        L.mlp_destroy.argtypes = [P]
        L.mlp_destroy.restype = None
        L.cc_t2_features.argtypes = [P, PF, PF, P]
        L.cc_t2_target.argtypes = [P, F, P]
        L.cc_guess_t2.argtypes = [P, P, PF, PF, F]
        for name in ("mlp_create", "mlp_dims", "mlp_set_params", "mlp_get_params", "mlp_forward",
                     "mlp_forward_noalloc",
                     "mlp_loss_grad", "mlp_adam_step", "mlp_train", "cc_t2_features",
                     "cc_t2_target", "cc_guess_t2"):
            getattr(L, name).restype = ctypes.c_int
        for name in ("cc_create", "cc_ground", "eom_solve", "multipliers", "densities", "nacme",
                     "cc_apply_jacobian", "cc_residual", "cc_export", "cc_set_guess",
                     "nm_contract", "nm_eig_host"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


EXPORTED = ["cc_default_opts", "cc_create", "cc_ground", "eom_solve", "multipliers",
            "densities", "nacme", "cc_apply_jacobian", "cc_residual", "cc_export",
            "cc_set_guess", "cc_last_error", "cc_destroy", "nm_contract", "nm_eig_host",
            "nm_version", "cc_stats", "nm_gemm", "nm_gemm_tiled", "cc_apply_jacobian_block",
            "mlp_create",
            "mlp_num_params", "mlp_dims", "mlp_set_params", "mlp_get_params", "mlp_forward",
            "mlp_forward_noalloc",
            "mlp_loss_grad", "mlp_adam_step", "mlp_train", "mlp_last_error", "mlp_destroy",
            "cc_t2_features", "cc_t2_target", "cc_guess_t2"]


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


def _fptr(t):
    if not t.is_cuda or t.dtype != __import__("torch").float32 or not t.is_contiguous():
        raise ValueError("expected a contiguous float32 device tensor")
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

    def multipliers(self, pairs):
        """Multipliers of the ordered pairs [(i, j), ...], solved together;
        returns ([[zeta iterations, kappa iterations] per pair], status)."""
        pairs = [(int(i), int(j)) for i, j in pairs]
        flat = (ctypes.c_int * (2 * len(pairs)))(*[x for p in pairs for x in p])
        it = (ctypes.c_int * (2 * len(pairs)))()
        rc = self._check(lib().multipliers(self._h, len(pairs), flat, it))
        return [[it[2 * p], it[2 * p + 1]] for p in range(len(pairs))], rc

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

    def t2_features(self, F, mu=None, sd=None):
        """F (device float32 [o^2 v^2][8]) <- standardised doubles features."""
        self._check(lib().cc_t2_features(self._h, _fvec(mu), _fvec(sd), _fptr(F)))
        return F

    def t2_target(self, Z, scale=1.0):
        """Z (device float32 [o^2 v^2]) <- (-D t - (ia|jb)) / scale."""
        self._check(lib().cc_t2_target(self._h, scale, _fptr(Z)))
        return Z

    def guess_t2(self, net, mu=None, sd=None, scale=1.0):
        """Start the next ground-state solve from the network's amplitudes."""
        self._check(lib().cc_guess_t2(self._h, net._h, _fvec(mu), _fvec(sd), scale))

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


def pair_interleave(hi, lo):
    """[R][K] hi and lo halves (K a multiple of 8) -> the library's pair
    layout [R][2K]: each chunk of 8 hi values followed by its 8 lo values."""
    import torch
    R, K = hi.shape
    return torch.stack([hi.reshape(R, K // 8, 8), lo.reshape(R, K // 8, 8)], dim=2).reshape(R, 2 * K)


def gemm(precision, A, B, C, alpha=1.0, beta=0.0, stream=None, tile=-1):
    """One matrix-core GEMM launch C = alpha A B + beta C (2-D row-major
    device tensors; A, B float64 for precision 0, float32 for precision 1).
    Precision 2: A [M][2K] and Bt [N][2K] bfloat16 pairs with B given
    transposed, hi and lo interleaved in chunks of 8 (pair_interleave), K a
    multiple of 32; tile selects the kernel's workgroup tile (nm_gemm_tiled,
    -1 = the library's choice)."""
    import torch
    if precision == 2:
        for t in (A, B):
            if not t.is_cuda or t.dtype != torch.bfloat16 or not t.is_contiguous() or t.dim() != 2:
                raise ValueError("bad GEMM operand")
        M, K2a = A.shape
        N, K2b = B.shape
        if K2a != K2b or K2a % 2 or tuple(C.shape) != (M, N):
            raise ValueError("GEMM shape mismatch")
        K = K2a // 2
        rc = lib().nm_gemm_tiled(2, tile, 0, 1, M, N, K, alpha, ctypes.c_void_p(A.data_ptr()), 2 * K,
                                 ctypes.c_void_p(B.data_ptr()), 2 * K, beta, _ptr(C), N,
                                 _stream_ptr(stream))
        if rc != CC_OK:
            raise CCError(rc, "nm_gemm")
        return C
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


def _fvec(x):
    if x is None:
        return None
    arr = (ctypes.c_float * len(x))(*[float(v) for v in x])
    return ctypes.cast(arr, ctypes.POINTER(ctypes.c_float))


class MLP:
    """Three-layer SiLU perceptron trained on the GPU (include/nacme.h)."""

    def __init__(self, n_in, width, n_out, seed=0, stream=None):
        self._h = ctypes.c_void_p()
        rc = lib().mlp_create(ctypes.byref(self._h), n_in, width, n_out, seed, _stream_ptr(stream))
        if rc != CC_OK:
            raise CCError(rc, "mlp_create failed")
        self.n_in, self.width, self.n_out = n_in, width, n_out
        self.num_params = int(lib().mlp_num_params(self._h))

    def _check(self, rc):
        if rc < 0:
            raise CCError(rc, lib().mlp_last_error(self._h).decode())
        return rc

    def get_params(self, working=False):
        import numpy as np
        out = np.zeros(self.num_params, dtype=np.float32)
        self._check(lib().mlp_get_params(
            self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(working)))
        return out

    def set_params(self, p):
        import numpy as np
        arr = np.ascontiguousarray(p, dtype=np.float32)
        if arr.size != self.num_params:
            raise ValueError("parameter count mismatch")
        self._check(lib().mlp_set_params(self._h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def forward(self, X, Y):
        self._check(lib().mlp_forward(self._h, X.shape[0], _fptr(X), _fptr(Y)))
        return Y

    def forward_noalloc(self, X, Y):
        """As forward, through the library's fixed work area (no allocation)."""
        self._check(lib().mlp_forward_noalloc(self._h, X.shape[0], _fptr(X), _fptr(Y)))
        return Y

    def loss_grad(self, X, T, want_grad=True):
        import numpy as np
        loss = ctypes.c_double()
        g = np.zeros(self.num_params, dtype=np.float32) if want_grad else None
        gp = g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if want_grad else None
        self._check(lib().mlp_loss_grad(self._h, X.shape[0], _fptr(X), _fptr(T), ctypes.byref(loss),
                                        gp))
        return loss.value, g

    def adam_step(self, lr):
        self._check(lib().mlp_adam_step(self._h, lr))

    def train(self, X, T, batch, steps, lr, seed=0):
        loss = ctypes.c_double()
        self._check(lib().mlp_train(self._h, X.shape[0], _fptr(X), _fptr(T), batch, steps, lr, seed,
                                    ctypes.byref(loss)))
        return loss.value

    def close(self):
        if self._h:
            lib().mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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
