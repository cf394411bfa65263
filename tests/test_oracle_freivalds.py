"""Pins of the CPU Freivalds check (oracle/freivalds.py).

The generator is pinned to published SplitMix64 test vectors; the test itself
to exact products (zero residual), correctly rounded products (accepted:
no false rejection) and planted errors (a single wrong entry beyond the row
tolerance is always rejected, in exactly that row).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import core
from oracle import freivalds as fv
from oracle import reference as ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def test_splitmix64_published_vectors():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 2
    for r in rows:
        seed, outs = int(r[0]), [int(v) for v in r[1:]]
        assert [fv.splitmix64(seed, j) for j in range(len(outs))] == outs


def test_sign_vector_is_pm1_and_mixed():
    x = fv.sign_vector(7, 4096)
    assert set(np.unique(x)) == {-1.0, 1.0}
    assert abs(x.sum()) < 4 * np.sqrt(4096)


def _int_complex(rng, r, c, lim=50):
    return rng.integers(-lim, lim + 1, (r, c)) + 1j * rng.integers(-lim, lim + 1, (r, c))


def test_exact_integer_product_has_zero_residual():
    rng = np.random.default_rng(3)
    A, B, Cin = _int_complex(rng, 9, 13), _int_complex(rng, 13, 7), _int_complex(rng, 9, 7)
    alpha, beta = 3 - 2j, -1 + 4j
    C = alpha * (A @ B) + beta * Cin          # small integers: exact in float64
    ratio, failed = fv.check(A, B, C, alpha, beta, Cin)
    assert failed == 0 and np.all(ratio == 0.0)


def _rounded_exact(A, B):
    ex = ref.exact_product(A.tolist(), B.tolist())
    return np.array([[complex(float(re), float(im)) for re, im in row] for row in ex])


@pytest.mark.parametrize("single", [False, True])
def test_correctly_rounded_product_is_accepted(single):
    A = workloads.complex_matrix(12, 40, phi=1.0, seed=11).astype(np.complex128)
    B = workloads.complex_matrix(40, 10, phi=1.0, seed=12).astype(np.complex128)
    C = _rounded_exact(A, B)
    if single:
        C = C.astype(np.complex64).astype(np.complex128)
    ratio, failed = fv.check(A, B, C, single=single)
    assert failed == 0 and ratio.max() < 1.0


@pytest.mark.parametrize("row,col", [(0, 0), (5, 3), (11, 9)])
def test_planted_error_is_caught_in_its_row(row, col):
    A = workloads.complex_matrix(12, 40, phi=1.0, seed=21).astype(np.complex128)
    B = workloads.complex_matrix(40, 10, phi=1.0, seed=22).astype(np.complex128)
    C = _rounded_exact(A, B)
    bad = C.copy()
    bad[row, col] += 1e-6 * (1 + 1j) * np.abs(C[row]).max()
    ratio, failed = fv.check(A, B, bad)
    assert failed == 1 and ratio[row] > 1.0
    assert np.all(np.delete(ratio, row) < 1.0)
    small = C.copy()
    small[row, col] += 1e-20 * np.abs(C[row]).max()
    assert fv.check(A, B, small)[1] == 0


def test_conjugate_transpose_operands():
    """op(A) = A^H, op(B) = B^T passed explicitly: an exact product passes."""
    rng = np.random.default_rng(5)
    A, B = _int_complex(rng, 11, 6), _int_complex(rng, 8, 11)   # A: k x m, B: n x k
    C = A.conj().T @ B.T
    ratio, failed = fv.check(A.conj().T, B.T, C)
    assert failed == 0 and np.all(ratio == 0.0)
    C[2, 1] += 1
    assert fv.check(A.conj().T, B.T, C)[1] == 1


def test_nan_output_is_rejected():
    rng = np.random.default_rng(6)
    A, B = _int_complex(rng, 4, 5), _int_complex(rng, 5, 3)
    C = A @ B
    C[1, 2] = complex(np.nan, 0)
    ratio, failed = fv.check(A, B, C)
    assert failed == 1 and np.isinf(ratio[1])


def test_emulation_accepted_at_full_n_rejected_when_too_coarse():
    """The Ozaki-II output (Algorithm 1) at N = 14 passes the FP64 test, at N = 4
    (P < 2^32: a few significant bits) it does not."""
    A = workloads.complex_matrix(24, 64, phi=0.5, seed=31)
    B = workloads.complex_matrix(64, 16, phi=0.5, seed=32)
    good = core.emulate(A, B, 14, mode="fast", algo="karatsuba")["out"]
    assert fv.check(A, B, good)[1] == 0
    coarse = core.emulate(A, B, 4, mode="fast", algo="karatsuba")["out"]
    assert fv.check(A, B, coarse)[1] > 0
