"""Pins of the accuracy yardstick (Section IV-A): (|A||B|)_ij, err_nc and err_cw.

The yardstick decides whether an emulated result "meets the FP64 bound", so each
function is pinned against values that do not come from the oracle itself: sums
evaluated in 60-digit arithmetic (mpmath), exact rationals, hand-built cases whose
answers are closed forms, and special cases (zero components).  The last test plants
mistakes in copies of the functions (a doubled denominator, a dropped low part, swapped
real and imaginary parts) and checks that the pins reject every one of them.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import workloads

mpmath.mp.dps = 60


def _mp_modulus(z) -> mpmath.mpf:
    return mpmath.sqrt(mpmath.mpf(float(z.real)) ** 2 + mpmath.mpf(float(z.imag)) ** 2)


def _abs_product_mp(A, B):
    m, k = A.shape
    n = B.shape[1]
    out = [[mpmath.mpf(0)] * n for _ in range(m)]
    for i in range(m):
        for j in range(n):
            out[i][j] = mpmath.fsum(_mp_modulus(A[i, h]) * _mp_modulus(B[h, j]) for h in range(k))
    return out


def _check_abs_product(fn):
    """(|A||B|)_ij with complex moduli, within k 2^-50 relative of a 60-digit evaluation."""
    A = workloads.complex_matrix(4, 29, 2.0, 901)
    B = workloads.complex_matrix(29, 3, 2.0, 902)
    A[1, 3] = 0
    A[2, :] = A[2, :].real          # a purely real row
    B[:, 1] = 1j * B[:, 1].imag     # a purely imaginary column
    got = fn(A, B)
    ref = _abs_product_mp(A, B)
    tol = 29 * 2.0 ** -50
    for i in range(4):
        for j in range(3):
            if abs(mpmath.mpf(float(got[i, j])) - ref[i][j]) > tol * ref[i][j]:
                return False
    # Pythagorean triples: |3+4i| |5+12i| = 65 exactly, k times
    a = np.full((2, 7), 3 + 4j)
    b = np.full((7, 2), 5 - 12j)
    return bool(np.array_equal(fn(a, b), np.full((2, 2), 65.0 * 7)))


def _check_err_nc(fn):
    """max_ij |out - (hi + lo)| / (|A||B|)_ij, complex modulus, zero bounds skipped."""
    u = 2.0 ** -60
    hi = np.array([[1 + 1j, 2 - 1j], [0.5j, -4 + 0j]])
    lo = np.array([[(3 + 4j) * u, 0j], [0j, 2j * u]])
    out = hi.copy()
    out[1, 0] += 2.0 ** -53          # a plain error in the high part
    absab = np.array([[2.0, 8.0], [1.0, 0.0]])  # (1, 1) has a zero bound: skipped
    # entries: (0,0) |lo| = 5u over 2; (1,0) 2^-53 over 1; (1,1) skipped
    exp = max(Fraction(5) * Fraction(u) / 2, Fraction(2.0 ** -53))
    if fn(out, hi, lo, absab) != float(exp):
        return False
    # the low part decides: with the high part exact, the error is |lo| / bound
    out2 = hi.copy()
    got = fn(out2, hi, lo, np.array([[1.0, 1.0], [1.0, 1.0]]))
    if got != 5 * u:
        return False
    # exact-rational check on random data whose low parts matter
    rng = np.random.default_rng(903)
    hi = workloads.complex_matrix(6, 5, 1.0, 904)
    lo = (rng.standard_normal((6, 5)) + 1j * rng.standard_normal((6, 5))) * 2.0 ** -58
    out = hi + (rng.standard_normal((6, 5)) + 1j * rng.standard_normal((6, 5))) * 2.0 ** -57
    absab = np.abs(hi) + 1.0
    best = mpmath.mpf(0)
    for i in range(6):
        for j in range(5):
            dr = Fraction(out[i, j].real) - Fraction(hi[i, j].real) - Fraction(lo[i, j].real)
            di = Fraction(out[i, j].imag) - Fraction(hi[i, j].imag) - Fraction(lo[i, j].imag)
            mod = mpmath.sqrt(mpmath.mpf(dr.numerator) / dr.denominator * (mpmath.mpf(dr.numerator) / dr.denominator)
                              + mpmath.mpf(di.numerator) / di.denominator * (mpmath.mpf(di.numerator) / di.denominator))
            best = max(best, mod / mpmath.mpf(float(absab[i, j])))
    got = fn(out, hi, lo, absab)
    return abs(mpmath.mpf(got) - best) <= 2.0 ** -48 * best


def _check_err_cw(fn):
    """max over entries and components of |out_c - ref_c| / |ref_c| (Section IV-A);
    a zero reference component gives 0 if matched exactly and inf otherwise."""
    u = 2.0 ** -40
    hi = np.array([[1e-3 + 1j, 2 + 0j]])
    lo = np.zeros_like(hi)
    out = hi.copy()
    out[0, 0] += u + 1j * u            # Re error u on |ref| 1e-3, Im error u on |ref| 1
    if fn(out, hi, lo) != u / 1e-3:
        return False
    # swapping the magnitudes of Re and Im changes the answer
    out = hi.copy()
    out[0, 0] += 1j * u
    if fn(out, hi, lo) != u:
        return False
    # the zero imaginary part of entry (0, 1): exact -> 0, any error -> inf
    out = hi.copy()
    if fn(out, hi, lo) != 0.0:
        return False
    out[0, 1] += 1j * u
    if fn(out, hi, lo) != np.inf:
        return False
    # the low part of the reference counts: Im of entry (0, 1) is 2^-70, the output's 0
    lo = np.array([[0j, 1j * 2.0 ** -70]])
    out = hi.copy()
    return fn(out, hi, lo) == 1.0


def test_abs_product_pinned(orc):
    assert _check_abs_product(orc.abs_product)


def test_err_nc_pinned(orc):
    assert _check_err_nc(orc.err_nc)


def test_err_cw_pinned(orc):
    assert _check_err_cw(orc.err_cw)


def test_err_nc_of_exact_and_one_ulp_results(orc):
    """Integer inputs: the double-double product is exact, so the exact result has error 0
    and one ulp added to one entry gives ulp / (|A||B|) for that entry."""
    A = workloads.integer_matrix(7, 40, 10, 905)
    B = workloads.integer_matrix(40, 6, 10, 906)
    hi, lo = orc.dd_gemm(A, B)
    exact = A @ B
    assert np.array_equal(hi, exact) and not lo.any()
    absab = orc.abs_product(A, B)
    assert orc.err_nc(exact, hi, lo, absab) == 0.0
    out = exact.copy()
    out[3, 2] = complex(np.nextafter(out[3, 2].real, np.inf), out[3, 2].imag)
    ulp = out[3, 2].real - exact[3, 2].real
    assert orc.err_nc(out, hi, lo, absab) == ulp / absab[3, 2]
    assert orc.err_cw(out, hi, lo) == ulp / abs(exact[3, 2].real)


def test_planted_yardstick_mistakes_are_caught(orc):
    """Mutated copies of the three functions must fail their pins."""
    doubled = lambda A, B: 2.0 * orc.abs_product(A, B)
    l1_moduli = lambda A, B: (np.abs(np.asarray(A).real) + np.abs(np.asarray(A).imag)) @ \
        (np.abs(np.asarray(B).real) + np.abs(np.asarray(B).imag))
    no_lo = lambda out, hi, lo, ab: orc.err_nc(out, hi, np.zeros_like(lo), ab)
    re_only = lambda out, hi, lo, ab: float(np.max(np.abs(((out - hi) - lo).real)[ab > 0] / ab[ab > 0]))
    no_mask = lambda out, hi, lo, ab: float(np.max(np.abs((out - hi) - lo) / np.where(ab > 0, ab, 1e-300)))

    def swapped(out, hi, lo):
        sw = lambda z: np.asarray(z).imag + 1j * np.asarray(z).real
        r = hi + lo
        er = np.abs((out.real - hi.real) - lo.real)
        ei = np.abs((out.imag - hi.imag) - lo.imag)
        with np.errstate(divide="ignore", invalid="ignore"):
            a = np.where(r.imag != 0, er / np.abs(r.imag), np.where(er == 0, 0.0, np.inf))
            b = np.where(r.real != 0, ei / np.abs(r.real), np.where(ei == 0, 0.0, np.inf))
        return float(max(a.max(initial=0.0), b.max(initial=0.0)))

    cw_no_lo = lambda out, hi, lo: orc.err_cw(out, hi, np.zeros_like(lo))
    assert not _check_abs_product(doubled)
    assert not _check_abs_product(l1_moduli)
    assert not _check_err_nc(no_lo)
    assert not _check_err_nc(re_only)
    assert not _check_err_nc(no_mask)
    assert not _check_err_cw(swapped)
    assert not _check_err_cw(cw_no_lo)
