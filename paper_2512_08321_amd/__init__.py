"""Ozaki-II emulation of complex GEMM on MI355X INT8 matrix cores.

Thin ctypes binding of ``libozc.so`` (C-ABI declared in ``include/ozc.h``):
argument marshalling only; every step of the computation runs in the HIP
kernels of the library.  PyTorch is used for device memory and streams.

Low level: ``Handle`` mirrors the C functions (``ozc_zgemm``, ``ozc_cgemm``,
``ozc_inspect``, ...) on raw device pointers.  High level: ``gemm(A, B, ...)``
takes torch tensors.

The library must have been built (``python -m paper_2512_08321_amd.build``
or ``__graft_entry__.build()``); importing the binding without it raises.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["Handle", "OzcError", "gemm", "lib", "OP", "MODE", "ALGO", "MAX_K", "NOALLOC_WORKSPACE",
           "MIN_MODULI", "MAX_MODULI", "EXP_ZERO", "EXP_NONFINITE", "library_path"]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.environ.get("OZC_LIBRARY") or os.path.join(_HERE, "libozc.so")

OP = {"N": 0, "T": 1, "C": 2}
MODE = {"fast": 0, "accurate": 1}
ALGO = {"karatsuba": 0, "4m": 1}
MAX_K = 131072
NOALLOC_WORKSPACE = 64 << 20   # bytes of the fixed workspace of ozc_zgemm_noalloc
MIN_MODULI, MAX_MODULI = 2, 24
EXP_ZERO, EXP_NONFINITE = -32768, 32767

STATUS = {0: "success", 1: "invalid value", 2: "not supported", 3: "device allocation failed",
          4: "HIP runtime error", 5: "non-finite input", 6: "invalid handle", 7: "verification failed"}


class OzcError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)} (status {status})")
        self.status = status


class Info(ctypes.Structure):
    _fields_ = [("num_moduli", ctypes.c_int), ("mode", ctypes.c_int), ("algo", ctypes.c_int),
                ("nonfinite", ctypes.c_int), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("k", ctypes.c_int64), ("workspace", ctypes.c_size_t), ("int8_ops", ctypes.c_double),
                ("verified", ctypes.c_int), ("escalations", ctypes.c_int),
                ("verify_failed_rows", ctypes.c_int64), ("verify_ratio", ctypes.c_double)]


class BatchPolicy(ctypes.Structure):
    _fields_ = [("tile_threshold", ctypes.c_int), ("moduli_group", ctypes.c_int),
                ("use_graph", ctypes.c_int)]


class Profile(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int), ("scale_ms", ctypes.c_double), ("split_ms", ctypes.c_double),
                ("gemm_ms", ctypes.c_double), ("crt_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]


_lib = None
_VP, _I64, _INT = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
_D2 = ctypes.c_double * 2
_F2 = ctypes.c_float * 2

EXPORTS = {
    "ozc_create": [ctypes.POINTER(_VP), _INT],
    "ozc_destroy": [_VP],
    "ozc_set_stream": [_VP, _VP],
    "ozc_set_config": [_VP, _INT, _INT, _INT],
    "ozc_workspace_size": [_VP, _INT, _INT, _I64, _I64, _I64, ctypes.POINTER(ctypes.c_size_t)],
    "ozc_set_workspace": [_VP, _VP, ctypes.c_size_t],
    "ozc_zgemm": [_VP, _INT, _INT, _I64, _I64, _I64, _D2, _VP, _I64, _VP, _I64, _D2, _VP, _I64],
    "ozc_cgemm": [_VP, _INT, _INT, _I64, _I64, _I64, _F2, _VP, _I64, _VP, _I64, _F2, _VP, _I64],
    "ozc_zgemm_noalloc": [_VP, _INT, _INT, _I64, _I64, _I64, _D2, _VP, _I64, _VP, _I64, _D2, _VP,
                          _I64],
    "ozc_zgemm_dd": [_VP, _INT, _INT, _I64, _I64, _I64, _VP, _I64, _VP, _I64, _VP, _VP, _I64],
    "ozc_dgemm": [_VP, _INT, _INT, _I64, _I64, _I64, ctypes.POINTER(ctypes.c_double), _VP, _I64,
                  _VP, _I64, ctypes.POINTER(ctypes.c_double), _VP, _I64],
    "ozc_sgemm": [_VP, _INT, _INT, _I64, _I64, _I64, ctypes.POINTER(ctypes.c_float), _VP, _I64,
                  _VP, _I64, ctypes.POINTER(ctypes.c_float), _VP, _I64],
    "ozc_inspect": [_VP, _INT, _INT, _INT, _I64, _I64, _I64, _VP, _I64, _VP, _I64, _VP, _VP, _VP,
                    _VP, _VP, _VP, _VP, _I64],
    "ozc_last_info": [_VP, ctypes.POINTER(Info)],
    "ozc_set_profiling": [_VP, _INT],
    "ozc_profile_read": [_VP, ctypes.POINTER(Profile)],
    "ozc_set_verify": [_VP, _INT, ctypes.c_double, _INT, ctypes.c_uint64],
    "ozc_debug_inject": [_VP, _INT],
    "ozc_zgemm_vbatched": [_VP, _INT, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                           _VP, _VP],
    "ozc_cgemm_vbatched": [_VP, _INT, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                           _VP, _VP],
    "ozc_set_batch_policy": [_VP, ctypes.POINTER(BatchPolicy)],
    "ozc_get_batch_policy": [_VP, ctypes.POINTER(BatchPolicy)],
    "ozc_batch_tune": [_VP, _INT, _INT, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                       ctypes.POINTER(BatchPolicy)],
    "ozc_features": [_VP, _INT, _INT, _INT, _I64, _I64, _I64, _VP, _I64, _VP, _I64, _VP],
    "ozc_mlp_set_params": [_VP, _VP, _INT],
    "ozc_mlp_get_params": [_VP, _VP, _INT],
    "ozc_mlp_save": [_VP, ctypes.c_char_p],
    "ozc_mlp_load": [_VP, ctypes.c_char_p],
    "ozc_mlp_forward": [_VP, _VP, _INT, _VP],
    "ozc_mlp_predict": [_VP, _VP, _INT, _VP],
    "ozc_mlp_grad": [_VP, _VP, _VP, _INT, _VP, _VP],
    "ozc_mlp_train": [_VP, _VP, _VP, _INT, _INT, _INT, ctypes.c_float, ctypes.c_uint64, _INT, _VP],
    "ozc_set_auto_moduli": [_VP, _INT, _INT],
    "ozc_predict_moduli": [_VP, _INT, _INT, _INT, _I64, _I64, _I64, _VP, _I64, _VP, _I64,
                           ctypes.POINTER(_INT)],
    "ozc_status_string": [_INT],
}

MLP_FEATURES, MLP_HIDDEN, MLP_CLASSES, MLP_MIN_N = 20, 64, 20, 6
MLP_PARAMS = (MLP_HIDDEN * MLP_FEATURES + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN
              + MLP_CLASSES * MLP_HIDDEN + MLP_CLASSES + 2 * MLP_FEATURES)


def lib():
    """The loaded libozc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise ImportError(f"{library_path} is missing: build it with "
                              "`python -m paper_2512_08321_amd.build`")
        L = ctypes.CDLL(library_path)
        for name, args in EXPORTS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name == "ozc_status_string" else ctypes.c_int
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != 0:
        raise OzcError(status, where)


def _ptr(x) -> int | None:
    """Device pointer of a torch tensor (or an int / None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


class Handle:
    """One ozc handle bound to a device; calls enqueue on torch's current stream."""

    def __init__(self, device: int = 0, num_moduli: int = 14, mode: str = "fast",
                 algo: str = "karatsuba"):
        self._h = _VP()
        _check(lib().ozc_create(ctypes.byref(self._h), device), "ozc_create")
        self.device = device
        self.set_config(num_moduli, mode, algo)

    def close(self):
        if self._h:
            lib().ozc_destroy(self._h)
            self._h = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_config(self, num_moduli: int, mode: str = "fast", algo: str = "karatsuba"):
        """num_moduli = 0 selects the learned per-call choice (ozc_zgemm)."""
        _check(lib().ozc_set_config(self._h, int(num_moduli), MODE[mode], ALGO[algo]), "ozc_set_config")
        self.num_moduli, self.mode, self.algo = int(num_moduli), mode, algo

    def set_stream(self, stream: int | None = None):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().ozc_set_stream(self._h, stream or None), "ozc_set_stream")

    def workspace_size(self, transa, transb, m, n, k) -> int:
        b = ctypes.c_size_t()
        _check(lib().ozc_workspace_size(self._h, OP[transa], OP[transb], m, n, k, ctypes.byref(b)),
               "ozc_workspace_size")
        return b.value

    def set_workspace(self, ptr, nbytes: int):
        _check(lib().ozc_set_workspace(self._h, _ptr(ptr), int(nbytes)), "ozc_set_workspace")

    def zgemm(self, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
        self.set_stream(stream)
        a, b = complex(alpha), complex(beta)
        _check(lib().ozc_zgemm(self._h, OP[transa], OP[transb], m, n, k, _D2(a.real, a.imag),
                               _ptr(A), lda, _ptr(B), ldb, _D2(b.real, b.imag), _ptr(C), ldc),
               "ozc_zgemm")

    def zgemm_noalloc(self, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                      stream=None):
        """ozc_zgemm_noalloc: ozc_zgemm on the library's fixed device workspace."""
        self.set_stream(stream)
        a, b = complex(alpha), complex(beta)
        _check(lib().ozc_zgemm_noalloc(self._h, OP[transa], OP[transb], m, n, k,
                                       _D2(a.real, a.imag), _ptr(A), lda, _ptr(B), ldb,
                                       _D2(b.real, b.imag), _ptr(C), ldc), "ozc_zgemm_noalloc")

    def cgemm(self, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
        self.set_stream(stream)
        a, b = complex(alpha), complex(beta)
        _check(lib().ozc_cgemm(self._h, OP[transa], OP[transb], m, n, k, _F2(a.real, a.imag),
                               _ptr(A), lda, _ptr(B), ldb, _F2(b.real, b.imag), _ptr(C), ldc),
               "ozc_cgemm")

    def zgemm_dd(self, transa, transb, m, n, k, A, lda, B, ldb, C_hi, C_lo, ldc, stream=None):
        """ozc_zgemm_dd: op(A) op(B) as the double-double pair C_hi + C_lo."""
        self.set_stream(stream)
        _check(lib().ozc_zgemm_dd(self._h, OP[transa], OP[transb], m, n, k, _ptr(A), lda, _ptr(B),
                                  ldb, _ptr(C_hi), _ptr(C_lo), ldc), "ozc_zgemm_dd")

    def dgemm(self, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
        """ozc_dgemm (real float64 operands)."""
        self.set_stream(stream)
        a, b = ctypes.c_double(float(alpha)), ctypes.c_double(float(beta))
        _check(lib().ozc_dgemm(self._h, OP[transa], OP[transb], m, n, k, ctypes.byref(a), _ptr(A),
                               lda, _ptr(B), ldb, ctypes.byref(b), _ptr(C), ldc), "ozc_dgemm")

    def sgemm(self, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
        """ozc_sgemm (real float32 operands)."""
        self.set_stream(stream)
        a, b = ctypes.c_float(float(alpha)), ctypes.c_float(float(beta))
        _check(lib().ozc_sgemm(self._h, OP[transa], OP[transb], m, n, k, ctypes.byref(a), _ptr(A),
                               lda, _ptr(B), ldb, ctypes.byref(b), _ptr(C), ldc), "ozc_sgemm")

    def inspect(self, single, transa, transb, m, n, k, A, lda, B, ldb, mu=None, nu=None,
                resA=None, resB=None, prods=None, eprime=None, C=None, ldc=1, stream=None):
        """ozc_inspect; ``single``: element kind (False/0 complex128, True/1 complex64,
        2 float64, 3 float32)."""
        self.set_stream(stream)
        _check(lib().ozc_inspect(self._h, int(single), OP[transa], OP[transb], m, n, k,
                                 _ptr(A), lda, _ptr(B), ldb, _ptr(mu), _ptr(nu), _ptr(resA),
                                 _ptr(resB), _ptr(prods), _ptr(eprime), _ptr(C), ldc),
               "ozc_inspect")

    def set_verify(self, enable: bool = True, rel: float = 0.0, escalate: bool = True,
                   seed: int = 0x5EED):
        _check(lib().ozc_set_verify(self._h, int(bool(enable)), float(rel), int(bool(escalate)),
                                    int(seed)), "ozc_set_verify")

    def debug_inject(self, fault: int):
        _check(lib().ozc_debug_inject(self._h, int(fault)), "ozc_debug_inject")

    def gemm_vbatched(self, problems, single: bool = False, stream=None):
        """Batched ozc_zgemm_vbatched / ozc_cgemm_vbatched.  ``problems``: list of dicts
        with keys transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc
        (A, B, C device tensors or pointers)."""
        self.set_stream(stream)
        b = _BatchArgs(problems, single)
        fn = lib().ozc_cgemm_vbatched if single else lib().ozc_zgemm_vbatched
        _check(fn(self._h, b.count, b.ta, b.tb, b.m, b.n, b.k, b.alpha, b.A, b.lda, b.B, b.ldb,
                  b.beta, b.C, b.ldc), "ozc_gemm_vbatched")

    def set_batch_policy(self, tile_threshold: int = 1024, moduli_group: int = 1,
                         use_graph: bool = True):
        p = BatchPolicy(int(tile_threshold), int(moduli_group), int(bool(use_graph)))
        _check(lib().ozc_set_batch_policy(self._h, ctypes.byref(p)), "ozc_set_batch_policy")

    def batch_policy(self) -> dict:
        p = BatchPolicy()
        _check(lib().ozc_get_batch_policy(self._h, ctypes.byref(p)), "ozc_get_batch_policy")
        return _policy_dict(p)

    def batch_tune(self, problems, single: bool = False, stream=None) -> dict:
        """ozc_batch_tune on the A/B operands of ``problems``; returns the chosen policy."""
        self.set_stream(stream)
        b = _BatchArgs(problems, single, with_c=False)
        p = BatchPolicy()
        _check(lib().ozc_batch_tune(self._h, int(bool(single)), b.count, b.ta, b.tb, b.m, b.n, b.k,
                                    b.A, b.lda, b.B, b.ldb, ctypes.byref(p)), "ozc_batch_tune")
        return _policy_dict(p)

    # ---------------------------------------------------------- moduli-count predictor
    def features(self, transa, transb, m, n, k, A, lda, B, ldb, out, single=False, stream=None):
        """ozc_features into ``out`` (device float32 tensor of MLP_FEATURES entries)."""
        self.set_stream(stream)
        _check(lib().ozc_features(self._h, int(bool(single)), OP[transa], OP[transb], m, n, k,
                                  _ptr(A), lda, _ptr(B), ldb, _ptr(out)), "ozc_features")

    def mlp_set_params(self, params):
        import numpy as np

        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().ozc_mlp_set_params(self._h, p.ctypes.data, p.size), "ozc_mlp_set_params")

    def mlp_get_params(self):
        import numpy as np

        p = np.zeros(MLP_PARAMS, np.float32)
        _check(lib().ozc_mlp_get_params(self._h, p.ctypes.data, p.size), "ozc_mlp_get_params")
        return p

    def mlp_save(self, path):
        _check(lib().ozc_mlp_save(self._h, os.fsencode(path)), "ozc_mlp_save")

    def mlp_load(self, path):
        _check(lib().ozc_mlp_load(self._h, os.fsencode(path)), "ozc_mlp_load")

    def mlp_forward(self, X, rows, logits, stream=None):
        self.set_stream(stream)
        _check(lib().ozc_mlp_forward(self._h, _ptr(X), int(rows), _ptr(logits)), "ozc_mlp_forward")

    def mlp_predict(self, X, rows, classes, stream=None):
        """ozc_mlp_predict: classes (device int32, rows) of feature rows X."""
        self.set_stream(stream)
        _check(lib().ozc_mlp_predict(self._h, _ptr(X), int(rows), _ptr(classes)), "ozc_mlp_predict")

    def mlp_grad(self, X, y, rows, grad, stream=None) -> float:
        self.set_stream(stream)
        loss = ctypes.c_float()
        _check(lib().ozc_mlp_grad(self._h, _ptr(X), _ptr(y), int(rows), _ptr(grad),
                                  ctypes.byref(loss)), "ozc_mlp_grad")
        return loss.value

    def mlp_train(self, X, y, rows, epochs, batch=256, lr=1e-3, seed=1, init=True, stream=None):
        import numpy as np

        self.set_stream(stream)
        losses = np.zeros(max(1, epochs), np.float32)
        _check(lib().ozc_mlp_train(self._h, _ptr(X), _ptr(y), int(rows), int(epochs), int(batch),
                                   float(lr), int(seed), int(bool(init)), losses.ctypes.data),
               "ozc_mlp_train")
        return losses[:epochs]

    def set_auto_moduli(self, fallback=18, margin=0):
        _check(lib().ozc_set_auto_moduli(self._h, int(fallback), int(margin)), "ozc_set_auto_moduli")

    def predict_moduli(self, transa, transb, m, n, k, A, lda, B, ldb, single=False,
                       stream=None) -> int:
        self.set_stream(stream)
        N = _INT()
        _check(lib().ozc_predict_moduli(self._h, int(bool(single)), OP[transa], OP[transb], m, n, k,
                                        _ptr(A), lda, _ptr(B), ldb, ctypes.byref(N)),
               "ozc_predict_moduli")
        return N.value

    def set_profiling(self, enable: bool):
        _check(lib().ozc_set_profiling(self._h, int(bool(enable))), "ozc_set_profiling")

    def profile_read(self) -> dict:
        prof = Profile()
        _check(lib().ozc_profile_read(self._h, ctypes.byref(prof)), "ozc_profile_read")
        return {f: getattr(prof, f) for f, _ in Profile._fields_}

    def last_info(self, raise_nonfinite: bool = False) -> dict:
        info = Info()
        st = lib().ozc_last_info(self._h, ctypes.byref(info))
        if st not in (0, 5) or (st == 5 and raise_nonfinite):
            _check(st, "ozc_last_info")
        return {f: getattr(info, f) for f, _ in Info._fields_}


def _arr(ctype, values):
    a = (ctype * max(1, len(values)))(*values)
    return a


class _BatchArgs:
    """Host arrays of one batched call (kept alive for the duration of the call)."""

    def __init__(self, problems, single: bool, with_c: bool = True):
        cnt = len(problems)
        self.count = cnt
        get = lambda key, default=None: [p.get(key, default) for p in problems]
        self.ta = _arr(_INT, [OP[t] for t in get("transa", "N")])
        self.tb = _arr(_INT, [OP[t] for t in get("transb", "N")])
        self.m = _arr(_I64, get("m"))
        self.n = _arr(_I64, get("n"))
        self.k = _arr(_I64, get("k"))
        self.lda = _arr(_I64, get("lda"))
        self.ldb = _arr(_I64, get("ldb"))
        self.A = _arr(_VP, [_ptr(x) for x in get("A")])
        self.B = _arr(_VP, [_ptr(x) for x in get("B")])
        if with_c:
            real = ctypes.c_float if single else ctypes.c_double
            al, be = [], []
            for p in problems:
                a, b = complex(p.get("alpha", 1.0)), complex(p.get("beta", 0.0))
                al += [a.real, a.imag]
                be += [b.real, b.imag]
            self.alpha = _arr(real, al)
            self.beta = _arr(real, be)
            self.C = _arr(_VP, [_ptr(x) for x in get("C")])
            self.ldc = _arr(_I64, get("ldc"))


def _policy_dict(p: BatchPolicy) -> dict:
    return {f: getattr(p, f) for f, _ in BatchPolicy._fields_}


_handles: dict = {}


def default_handle(device: int = 0) -> Handle:
    if device not in _handles:
        _handles[device] = Handle(device)
    return _handles[device]


def gemm(A, B, C=None, alpha=1.0, beta=0.0, num_moduli: int = 14, mode: str = "fast",
         algo: str = "karatsuba", handle: Handle | None = None):
    """alpha * A @ B + beta * C for row-major torch tensors on the GPU.

    complex128 -> ozc_zgemm, complex64 -> ozc_cgemm, float64 -> ozc_dgemm,
    float32 -> ozc_sgemm (real: real alpha and beta).  Row-major C = A B is
    computed as the column-major product C^T = B^T A^T (no copies); the
    scheme treats rows of A and columns of B symmetrically, so the result is
    the same bit for bit.
    """
    import torch

    calls = {torch.complex128: "zgemm", torch.complex64: "cgemm", torch.float64: "dgemm",
             torch.float32: "sgemm"}
    if A.dtype != B.dtype or A.dtype not in calls:
        raise TypeError("A and B must both be complex128, complex64, float64 or float32")
    if A.dim() != 2 or B.dim() != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("shape mismatch")
    m, k = A.shape
    n = B.shape[1]
    A = A.contiguous()
    B = B.contiguous()
    if C is None:
        C = torch.empty((m, n), dtype=A.dtype, device=A.device)
        beta = 0.0
    elif not C.is_contiguous() or C.shape != (m, n) or C.dtype != A.dtype:
        raise ValueError("C must be a contiguous (m, n) tensor of the same dtype")
    h = handle or default_handle(A.device.index or 0)
    if (h.num_moduli, h.mode, h.algo) != (num_moduli, mode, algo):
        h.set_config(num_moduli, mode, algo)
    call = getattr(h, calls[A.dtype])
    call("N", "N", n, m, k, alpha, B, max(1, n), A, max(1, k), beta, C, max(1, n))
    return C
