"""numpy front end of the C oracle (oracle/core.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark; never by the product path.

Conventions: ``A`` is op(A) as an (m, k) complex numpy array, ``B`` is op(B)
as a (k, n) complex array (any memory order; complex64 is promoted exactly to
complex128).  Exponents are integers with a per-row flag: 0 = the row carries
no scaling (all-zero row, or a vanishing accurate-mode bound), 1 = ok,
2 = the row holds a non-finite value.
"""
from __future__ import annotations

import bisect
import ctypes
import os
from functools import lru_cache

import numpy as np

from . import reference as ref

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_orc_core.so")
_lib = None

FLAG_ZERO, FLAG_OK, FLAG_NONFINITE = 0, 1, 2


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build
            build.build()
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


I64 = ctypes.c_int64


# ---------------------------------------------------------------- constants

@lru_cache(maxsize=None)
def constants(n_moduli: int):
    """Moduli, P, q, s (Python ints) plus word-split copies for the C code."""
    p, P, q, s = ref.crt_constants(n_moduli)
    words = lambda v: [(v >> (64 * j)) & ((1 << 64) - 1) for j in range(4)]
    s_words = np.array([words(v) for v in s], dtype=np.uint64)
    P_words = np.array(words(P), dtype=np.uint64)
    F = ref.SIGMA_FRAC_BITS
    tmax = ref.fast_t_max(P)
    # fast: sigma <= floor((P-1) 2^(2F) / (8 * 4^t)), t = tmax - d
    fast_thr = []
    for d in range(160):
        t = tmax - d
        e2 = 2 * F - 3 - 2 * t
        fast_thr.append(((P - 1) << e2) if e2 >= 0 else ((P - 1) >> (-e2)))
    thi = ref.accurate_t(1, P)
    accu_thr = []
    for d in range(160):
        t = thi - d
        e2 = -1 - 2 * t
        accu_thr.append(((P - 1) << e2) if e2 >= 0 else ((P - 1) >> (-e2)))
    return dict(p=p, P=P, q=q, s=s, s_words=s_words, P_words=P_words,
                p_arr=np.array(p, dtype=np.int32), fast_tmax=tmax, fast_thr=fast_thr,
                accu_thi=thi, accu_thr=accu_thr)


# ---------------------------------------------------------------- helpers

def rows_of_A(A):
    """(re, im) row-major float64 arrays of the rows of op(A)."""
    A = np.asarray(A).astype(np.complex128)
    return np.ascontiguousarray(A.real), np.ascontiguousarray(A.imag)


def rows_of_B(B):
    """(re, im) row-major float64 arrays of the columns of op(B)."""
    B = np.asarray(B).astype(np.complex128)
    return np.ascontiguousarray(B.real.T), np.ascontiguousarray(B.imag.T)


def row_exponents(re, im):
    lib = _load()
    rows, ln = re.shape
    e = np.zeros(rows, np.int32)
    raw = np.zeros(rows, np.uint8)
    lib.orc_row_exponents(_p(re), _p(im), I64(rows), I64(ln), _p(e), _p(raw))
    # C flags: 0 ok, 1 zero, 2 non-finite  ->  python flags
    flags = np.where(raw == 0, FLAG_OK, np.where(raw == 1, FLAG_ZERO, FLAG_NONFINITE)).astype(np.uint8)
    return e, flags


def _cflags(flags):
    """python flags -> C flags (0 ok, 1 zero, 2 non-finite)."""
    return np.where(flags == FLAG_OK, 0, np.where(flags == FLAG_ZERO, 1, 2)).astype(np.uint8)


# ---------------------------------------------------------------- exponents

def fast_exponents(re, im, n_moduli):
    """Fast-mode exponents mu (Section III-B): returns (mu, flags, e, sigma)."""
    lib = _load()
    c = constants(n_moduli)
    rows, ln = re.shape
    e, flags = row_exponents(re, im)
    sigma = np.zeros(rows, np.uint64)
    lib.orc_fast_sigma(_p(re), _p(im), I64(rows), I64(ln), ctypes.c_int(ref.SIGMA_FRAC_BITS),
                       _p(e), _p(_cflags(flags)), _p(sigma))
    mu = np.zeros(rows, np.int32)
    for r in range(rows):
        if flags[r] == FLAG_OK:
            d = bisect.bisect_left(c["fast_thr"], int(sigma[r]))
            mu[r] = (c["fast_tmax"] - d) - int(e[r])
    return mu, flags, e, sigma


def ceil7(re, im, e, flags):
    lib = _load()
    rows, ln = re.shape
    bR = np.zeros((rows, ln), np.int8)
    bI = np.zeros((rows, ln), np.int8)
    lib.orc_ceil7(_p(re), _p(im), I64(rows), I64(ln), _p(e), _p(_cflags(flags)), _p(bR), _p(bI))
    return bR, bI


def accurate_exponents(Are, Aim, Bre, Bim, n_moduli):
    """Accurate-mode exponents (Section III-B): returns (mu, nu, fa, fb, X, Y)."""
    lib = _load()
    c = constants(n_moduli)
    m, ln = Are.shape
    n = Bre.shape[0]
    eA, fa = row_exponents(Are, Aim)
    eB, fb = row_exponents(Bre, Bim)
    aR, aI = ceil7(Are, Aim, eA, fa)
    bR, bI = ceil7(Bre, Bim, eB, fb)
    X = np.zeros(m, np.int64)
    Y = np.zeros(n, np.int64)
    lib.orc_bound_max(_p(aR), _p(aI), I64(m), _p(bR), _p(bI), I64(n), I64(ln), _p(X), _p(Y))
    base = ref.ACCU_INT_BITS - 1

    def fin(e, f, V):
        mu = np.zeros(len(e), np.int32)
        f = f.copy()
        for r in range(len(e)):
            if f[r] != FLAG_OK:
                continue
            if V[r] == 0:
                f[r] = FLAG_ZERO
                continue
            d = bisect.bisect_left(c["accu_thr"], int(V[r]))
            mu[r] = base - int(e[r]) + (c["accu_thi"] - d)
        return mu, f

    mu, fa = fin(eA, fa, X)
    nu, fb = fin(eB, fb, Y)
    return mu, nu, fa, fb, X, Y


# ---------------------------------------------------------------- pipeline

def residues(re, im, mu, flags, n_moduli):
    """Residue planes [l][R,I,S][rows][k] of trunc(x 2^mu) (Step IV, V-i/ii)."""
    lib = _load()
    c = constants(n_moduli)
    rows, ln = re.shape
    out = np.zeros((n_moduli, 3, rows, ln), np.int8)
    valid = (flags == FLAG_OK).astype(np.uint8)
    of = lib.orc_residues(_p(re), _p(im), I64(rows), I64(ln), _p(mu.astype(np.int32)), _p(valid),
                          ctypes.c_int(n_moduli), _p(c["p_arr"]), _p(out))
    if of:
        raise OverflowError("truncated integer exceeds 126 bits")
    return out


def products(resA, resB, n_moduli, algo="karatsuba", want_raw=False):
    """E' planes [l][R,I][m][n] (and optionally the raw integer products)."""
    lib = _load()
    c = constants(n_moduli)
    _, _, m, ln = resA.shape
    n = resB.shape[2]
    a = 0 if algo == "karatsuba" else 1
    Ep = np.zeros((n_moduli, 2, m, n), np.int8)
    raw = np.zeros((n_moduli, 3 if a == 0 else 4, m, n), np.int64) if want_raw else None
    lib.orc_products(_p(np.ascontiguousarray(resA)), I64(m), _p(np.ascontiguousarray(resB)),
                     I64(n), I64(ln), ctypes.c_int(n_moduli), _p(c["p_arr"]), ctypes.c_int(a),
                     _p(Ep), _p(raw) if raw is not None else None)
    return Ep, raw


def crt_output(Ep, mu, fa, nu, fb, n_moduli, alpha=1.0, beta=0.0, Cin=None, want_cp=False,
               want_lo=False):
    """Steps V-v, V-vi, VI.  Returns (out, RNE(C') or None, low parts or None): the low part
    of an entry is ldexp(RNE(C' - RNE(C')), -(mu_i + nu_j)), the second word of the
    double-double value of the scaled C'."""
    lib = _load()
    c = constants(n_moduli)
    m, n = Ep.shape[2], Ep.shape[3]
    out = np.zeros((m, n), np.complex128)
    cp = np.zeros((m, n), np.complex128) if want_cp else None
    lo = np.zeros((m, n), np.complex128) if want_lo else None
    al = np.array([complex(alpha).real, complex(alpha).imag], np.float64)
    be = np.array([complex(beta).real, complex(beta).imag], np.float64)
    cin = np.ascontiguousarray(np.asarray(Cin, dtype=np.complex128)) if Cin is not None else None
    if cin is None and (be != 0).any():
        raise ValueError("beta != 0 needs C")
    lib.orc_crt_output(_p(np.ascontiguousarray(Ep)), I64(m), I64(n), ctypes.c_int(n_moduli),
                       _p(c["s_words"]), _p(c["P_words"]), _p(mu.astype(np.int32)),
                       _p(fa.astype(np.uint8)), _p(nu.astype(np.int32)), _p(fb.astype(np.uint8)),
                       _p(al), _p(be), _p(cin) if cin is not None else None, _p(out),
                       _p(cp) if cp is not None else None, _p(lo) if lo is not None else None)
    return out, cp, lo


def emulate(A, B, n_moduli, mode="fast", algo="karatsuba", alpha=1.0, beta=0.0, C=None,
            single=False, want_raw=False, want_cp=False, exponents=None, fault=0, want_lo=False):
    """alpha * A @ B + beta * C by the complex Ozaki-II scheme, computed exactly.

    A: (m, k) op(A); B: (k, n) op(B).  ``single`` rounds the result to
    complex64 (CGEMM: inputs promoted exactly, output rounded once more).
    ``exponents`` may carry precomputed (mu, fa, nu, fb) (e.g. for sampled
    entries of a large accurate-mode problem).
    ``want_lo`` adds the low parts of the double-double value of the scaled C'
    (``lo``; with alpha = 1, beta = 0, out + lo is that value).
    ``fault`` = 1 plants a mistake for tests of the verification step: the
    real part of E'_1 at entry (0, 0) has its bits 0x5a flipped before the
    reconstruction.
    Returns a dict of the intermediates and ``out``.
    """
    Are, Aim = rows_of_A(A)
    Bre, Bim = rows_of_B(B)
    if exponents is not None:
        mu, fa, nu, fb = exponents
    elif mode == "fast":
        mu, fa, _, _ = fast_exponents(Are, Aim, n_moduli)
        nu, fb, _, _ = fast_exponents(Bre, Bim, n_moduli)
    elif mode == "accurate":
        mu, nu, fa, fb, _, _ = accurate_exponents(Are, Aim, Bre, Bim, n_moduli)
    else:
        raise ValueError(mode)
    resA = residues(Are, Aim, mu, fa, n_moduli)
    resB = residues(Bre, Bim, nu, fb, n_moduli)
    Ep, raw = products(resA, resB, n_moduli, algo, want_raw)
    if fault == 1 and Ep.size:
        Ep[0, 0, 0, 0] = np.int8(Ep[0, 0, 0, 0] ^ np.int8(0x5A))
    elif fault:
        raise ValueError(fault)
    Cin = None if C is None else np.asarray(C, dtype=np.complex128)
    al, be = complex(alpha), complex(beta)
    if single:
        al, be = complex(np.complex64(al)), complex(np.complex64(be))
    out, cp, lo = crt_output(Ep, mu, fa, nu, fb, n_moduli, al, be, Cin, want_cp, want_lo)
    if single:
        out = out.astype(np.complex64)
    return dict(mu=mu, nu=nu, fa=fa, fb=fb, resA=resA, resB=resB, Ep=Ep, raw=raw, Cp=cp, out=out,
                lo=lo)


def emulate_real(A, B, n_moduli, mode="fast", alpha=1.0, beta=0.0, C=None, single=False,
                 want_raw=False, exponents=None):
    """alpha * A @ B + beta * C for real A (m, k), B (k, n) by Algorithm 1, computed exactly.

    Scaling (Step III): a real row is scaled by the rule of Section III-B for a
    row of k reals (the complex rule reads a row as its 2k reals; with no
    imaginary parts both coincide), so the exponent routines run on the rows
    with zero imaginary parts.  Steps IV-VI: a' = trunc(a 2^mu), one residue
    plane per modulus, D'_l = A'_l B'_l, E'_l = mod(D'_l, p_l), C' = mod(sum_l
    s_l E'_l, P) exactly, ldexp(RNE(C'), -(mu_i + nu_j)), then x = alpha c
    (one rounding) and out = x (beta = 0) or fma(beta, C_in, x).  ``single``:
    float32 inputs promoted exactly, the float64 result rounded once to float32.
    """
    lib = _load()
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    Are = np.ascontiguousarray(A)
    Bre = np.ascontiguousarray(B.T)
    Aim = np.zeros_like(Are)
    Bim = np.zeros_like(Bre)
    if exponents is not None:
        mu, fa, nu, fb = exponents
    elif mode == "fast":
        mu, fa, _, _ = fast_exponents(Are, Aim, n_moduli)
        nu, fb, _, _ = fast_exponents(Bre, Bim, n_moduli)
    elif mode == "accurate":
        mu, nu, fa, fb, _, _ = accurate_exponents(Are, Aim, Bre, Bim, n_moduli)
    else:
        raise ValueError(mode)
    c = constants(n_moduli)
    resA = np.ascontiguousarray(residues(Are, Aim, mu, fa, n_moduli)[:, 0])   # the real plane
    resB = np.ascontiguousarray(residues(Bre, Bim, nu, fb, n_moduli)[:, 0])
    m, ln = Are.shape
    n = Bre.shape[0]
    Ep = np.zeros((n_moduli, m, n), np.int8)
    raw = np.zeros((n_moduli, m, n), np.int64) if want_raw else None
    lib.orc_real_products(_p(resA), I64(m), _p(resB), I64(n), I64(ln), ctypes.c_int(n_moduli),
                          _p(c["p_arr"]), _p(Ep), _p(raw) if raw is not None else None)
    al, be = float(alpha), float(beta)
    if single:
        al, be = float(np.float32(al)), float(np.float32(be))
    cin = None
    if be != 0.0:
        if C is None:
            raise ValueError("beta != 0 needs C")
        cin = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    out = np.zeros((m, n), np.float64)
    lib.orc_real_crt_output(_p(Ep), I64(m), I64(n), ctypes.c_int(n_moduli), _p(c["s_words"]),
                            _p(c["P_words"]), _p(mu.astype(np.int32)), _p(fa.astype(np.uint8)),
                            _p(nu.astype(np.int32)), _p(fb.astype(np.uint8)), ctypes.c_double(al),
                            ctypes.c_double(be), _p(cin) if cin is not None else None, _p(out),
                            None)
    if single:
        out = out.astype(np.float32)
    return dict(mu=mu, nu=nu, fa=fa, fb=fb, resA=resA, resB=resB, Ep=Ep, raw=raw, out=out)


def set_threads(n: int) -> int:
    """Run the C loops on n OpenMP threads; returns the previous count."""
    lib = _load()
    old = lib.orc_max_threads()
    lib.orc_set_threads(ctypes.c_int(int(n)))
    return old


def max_threads() -> int:
    return _load().orc_max_threads()


# ---------------------------------------------------------------- yardsticks

def dd_gemm(A, B):
    """Double-double complex product: returns (hi, lo) complex arrays, hi + lo ~ A @ B."""
    lib = _load()
    Are, Aim = rows_of_A(A)
    Bre, Bim = rows_of_B(B)
    m, ln = Are.shape
    n = Bre.shape[0]
    hi = np.zeros((m, n), np.complex128)
    lo = np.zeros((m, n), np.complex128)
    lib.orc_dd_gemm(_p(Are), _p(Aim), I64(m), _p(Bre), _p(Bim), I64(n), I64(ln), _p(hi), _p(lo))
    return hi, lo


def abs_product(A, B):
    """(|A||B|)_ij with complex moduli."""
    lib = _load()
    Are, Aim = rows_of_A(A)
    Bre, Bim = rows_of_B(B)
    m, ln = Are.shape
    n = Bre.shape[0]
    out = np.zeros((m, n), np.float64)
    lib.orc_abs_product(_p(Are), _p(Aim), I64(m), _p(Bre), _p(Bim), I64(n), I64(ln), _p(out))
    return out


def err_nc(out, ref_hi, ref_lo, absAB):
    """max_ij |out - C_ref| / (|A||B|)_ij (complex modulus; entries with a zero bound skipped)."""
    d = (np.asarray(out, np.complex128) - ref_hi) - ref_lo
    mask = absAB > 0
    if not mask.any():
        return 0.0
    return float(np.max(np.abs(d[mask]) / absAB[mask]))


def err_cw(out, ref_hi, ref_lo):
    """The paper's componentwise relative error (Section IV-A)."""
    out = np.asarray(out, np.complex128)
    r = ref_hi + ref_lo
    er = np.abs((out.real - ref_hi.real) - ref_lo.real)
    ei = np.abs((out.imag - ref_hi.imag) - ref_lo.imag)
    with np.errstate(divide="ignore", invalid="ignore"):
        a = np.where(r.real != 0, er / np.abs(r.real), np.where(er == 0, 0.0, np.inf))
        b = np.where(r.imag != 0, ei / np.abs(r.imag), np.where(ei == 0, 0.0, np.inf))
    return float(max(a.max(initial=0.0), b.max(initial=0.0)))
