"""Freivalds check of an emulated complex product (CPU reference).

TEST INFRASTRUCTURE ONLY: used by the tests to check the library's own
verification step; nothing in the product path imports it.

The check is not part of the paper.  It guards the output of the Ozaki-II
pipeline (Section II, Algorithm 1; Section III) against a violated uniqueness
condition (equation (4)) or a corrupted residue product: with a random sign
vector x,

    w = C_out x,   z = op(A) (op(B) x),   v = C_in x,

the result is accepted when for every row i

    |w_i - alpha z_i - beta v_i|
        <= rel (|alpha| (|op(A)| (|op(B)| |x|))_i + |beta| (|C_in| |x|)_i)
           + gam (|C_out| |x| + |alpha| |op(A)| |op(B)| |x| + |beta| |C_in| |x|)_i,

where the second term is the evaluation slack of the library's double-double
accumulation (gam = 4 (n + k + 4) 2^-104).  Here the three matrix-vector
products and the residual are computed exactly (rational arithmetic on the
double inputs), so the slack only has to match the library's tolerance.  The
default relative tolerance is 4 k u with u = 2^-53 (ZGEMM) or 2^-24 (CGEMM),
the classical bound of a k-term dot product in the target precision.  |z| for
complex z is its modulus.

x_j = -1 if bit 0 of SplitMix64(seed, j) is set, else +1.  SplitMix64 is the
generator of Steele, Lea and Flood (OOPSLA 2014): the j-th output (counting
from 0) of the stream with initial state ``seed``.

A wrong entry c_ij shifts w_i by exactly |c_ij - c*_ij| because |x_j| = 1, so
a single wrong entry larger than the row's tolerance is always caught.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, j: int) -> int:
    """Output j (0-based) of SplitMix64 started from state ``seed``."""
    z = (seed + (j + 1) * _GAMMA) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def sign_vector(seed: int, n: int) -> np.ndarray:
    """x_j = +1 or -1 from bit 0 of SplitMix64(seed, j)."""
    return np.array([-1.0 if splitmix64(seed, j) & 1 else 1.0 for j in range(n)])


def default_rel(k: int, single: bool) -> float:
    return 4.0 * k * (2.0 ** -24 if single else 2.0 ** -53)


def _exact_matvec(M, x):
    """Exact complex M @ x with M of doubles and x of (re, im) Fraction pairs."""
    out = []
    for row in M:
        re = im = Fraction(0)
        for mij, (xr, xi) in zip(row, x):
            mr, mi = Fraction(float(mij.real)), Fraction(float(mij.imag))
            re += mr * xr - mi * xi
            im += mr * xi + mi * xr
        out.append((re, im))
    return out


def check(opA, opB, C_out, alpha=1.0, beta=0.0, C_in=None, seed=0x5EED, rel=0.0, single=False):
    """Row-wise Freivalds test.

    opA: m x k, opB: k x n, C_out and C_in: m x n complex arrays (op already
    applied).  Returns (ratio, failed): ratio_i = |residual_i| / tol_i (0 where
    both are 0, inf where only the residual is nonzero or it is NaN), and the
    number of rows with ratio_i > 1.
    """
    opA = np.asarray(opA, dtype=np.complex128)
    opB = np.asarray(opB, dtype=np.complex128)
    C_out = np.asarray(C_out, dtype=np.complex128)
    m, k = opA.shape
    n = opB.shape[1]
    alpha = complex(alpha)
    beta = complex(beta)
    if rel <= 0.0:
        rel = default_rel(k, single)
    gam = 4.0 * (n + k + 4) * 2.0 ** -104
    x = sign_vector(seed, n)
    xs = [(Fraction(float(v)), Fraction(0)) for v in x]
    ya = np.abs(opB) @ np.abs(x)
    za = np.abs(opA) @ ya
    wa = np.abs(C_out) @ np.abs(x)
    bound = rel * abs(alpha) * za
    evals = wa + abs(alpha) * za
    finite = np.all(np.isfinite(C_out.real)) and np.all(np.isfinite(C_out.imag))
    use_beta = beta != 0 and C_in is not None
    if use_beta:
        C_in = np.asarray(C_in, dtype=np.complex128)
        va = np.abs(C_in) @ np.abs(x)
        bound = bound + rel * abs(beta) * va
        evals = evals + abs(beta) * va
    tol = bound + gam * evals
    r = np.full(m, np.nan)
    if finite:
        z = _exact_matvec(opA, _exact_matvec(opB, xs))
        w = _exact_matvec(C_out, xs)
        ar, ai = Fraction(alpha.real), Fraction(alpha.imag)
        v = _exact_matvec(C_in, xs) if use_beta else None
        br, bi = Fraction(beta.real), Fraction(beta.imag)
        for i in range(m):
            er = w[i][0] - (ar * z[i][0] - ai * z[i][1])
            ei = w[i][1] - (ar * z[i][1] + ai * z[i][0])
            if use_beta:
                er -= br * v[i][0] - bi * v[i][1]
                ei -= br * v[i][1] + bi * v[i][0]
            r[i] = float(np.hypot(float(er), float(ei)))
    else:  # rows with a non-finite output entry fail; the others are checked exactly
        bad = ~(np.isfinite(C_out.real) & np.isfinite(C_out.imag)).all(axis=1)
        good = np.where(~bad)[0]
        if good.size:
            sub_r, _ = check(opA[good], opB, C_out[good], alpha, beta,
                             None if C_in is None else np.asarray(C_in)[good], seed, rel, single)
            r[good] = sub_r * tol[good]
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(tol > 0, r / np.where(tol > 0, tol, 1.0), np.where(r > 0, np.inf, 0.0))
    ratio = np.where(np.isnan(ratio) | np.isnan(r) | np.isnan(tol), np.inf, ratio)
    return ratio, int(np.count_nonzero(ratio > 1.0))
