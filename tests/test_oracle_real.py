"""Pins of the oracle's real-matrix path (Algorithm 1 as stated for real A, B).

Each pin checks a property fixed by the mathematics, not the oracle against a
retyped copy of itself: the reconstructed integers equal the exact integer
product of the truncated inputs and satisfy the uniqueness condition (4);
integer-valued inputs come back exactly; the truncation error obeys its closed
form; the error meets the double-precision level at 14 moduli; the C oracle
equals the pure-Python statement on every intermediate; a real product equals
the complex scheme's result on the same matrices with zero imaginary parts.
Planted mistakes (a dropped modulus, a non-symmetric remainder) fail the
brute-force pin.
"""
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import reference as ref


def _mat(rows, cols, phi, seed):
    rng = np.random.default_rng(seed)
    return (rng.random((rows, cols)) - 0.5) * np.exp(phi * rng.standard_normal((rows, cols)))


def _cases():
    rnd = random.Random(11)
    for t in range(16):
        m, n, k = rnd.randint(1, 4), rnd.randint(1, 4), rnd.randint(1, 7)
        yield (m, n, k, rnd.choice([2, 3, 5, 8, 13, 14, 17, 20]), rnd.choice([0.0, 0.5, 2.0, 4.0]),
               rnd.choice(["fast", "accurate"]), 500 + t)


def _brute_force_ok(r, k):
    """C' is the exact integer product A'B' and 2 sum |a'||b'| < P (condition (4))."""
    P = r["P"]
    Ai, Bi, Cp = r["Ai"], r["Bi"], r["Cp"]
    for i in range(len(Ai)):
        for j in range(len(Bi[0]) if Bi else 0):
            exact = sum(Ai[i][h] * Bi[h][j] for h in range(k))
            if Cp[i][j] != exact:
                return False
            if 2 * sum(abs(Ai[i][h]) * abs(Bi[h][j]) for h in range(k)) >= P:
                return False
    return True


@pytest.mark.parametrize("m,n,k,N,phi,mode,seed", list(_cases()))
def test_real_reconstruction_is_the_exact_integer_product(m, n, k, N, phi, mode, seed):
    A = _mat(m, k, phi, seed)
    B = _mat(k, n, phi, seed + 1)
    r = ref.emulate_real(A.tolist(), B.tolist(), N, mode)
    assert _brute_force_ok(r, k)
    # each E'_l is the symmetric residue of the integer product (Step V-iv)
    for l, pl in enumerate(r["p"]):
        for i in range(m):
            for j in range(n):
                e = r["Ep"][l][i][j]
                assert -(pl // 2) <= e <= (pl + 1) // 2 - 1
                assert (r["Cp"][i][j] - e) % pl == 0


def test_planted_mistakes_fail_the_brute_force_pin(monkeypatch):
    A = _mat(3, 5, 1.0, 71)
    B = _mat(5, 2, 1.0, 72)
    good = ref.emulate_real(A.tolist(), B.tolist(), 8)
    assert _brute_force_ok(good, 5)
    # a non-symmetric remainder in [0, p) breaks the reconstruction of negative products
    monkeypatch.setattr(ref, "smod", lambda x, p: x % p)
    bad = ref.emulate_real(A.tolist(), B.tolist(), 8)
    assert not _brute_force_ok(bad, 5)
    monkeypatch.undo()
    # the CRT constants of a smaller set (a dropped modulus) break it as well
    real_crt = ref.crt_constants
    monkeypatch.setattr(ref, "crt_constants",
                        lambda n: (lambda p, P, q, s: (p, P, q, [x if i else 0 for i, x in enumerate(s)]))(*real_crt(n)))
    bad = ref.emulate_real(A.tolist(), B.tolist(), 8)
    assert not _brute_force_ok(bad, 5)


@pytest.mark.parametrize("mode", ["fast", "accurate"])
def test_integer_inputs_are_exact(mode):
    rng = np.random.default_rng(5)
    A = rng.integers(-1000, 1001, size=(4, 6)).astype(np.float64)
    B = rng.integers(-1000, 1001, size=(6, 3)).astype(np.float64)
    r = ref.emulate_real(A.tolist(), B.tolist(), 8, mode)
    exact = [[sum(int(A[i, h]) * int(B[h, j]) for h in range(6)) for j in range(3)] for i in range(4)]
    assert r["out"] == [[float(v) for v in row] for row in exact]


@pytest.mark.parametrize("N", [6, 10, 14])
def test_truncation_bound_closed_form(N):
    """|out - AB| <= 2^-mu ||b_j||_1 + 2^-nu ||a_i||_1 + ulp(out): a' and b' differ from
    a 2^mu and b 2^nu by less than 1 each (trunc), so the product differs by at most the
    sum of those terms, and the final conversion adds one rounding."""
    A = _mat(5, 9, 2.0, 81)
    B = _mat(9, 4, 2.0, 82)
    r = ref.emulate_real(A.tolist(), B.tolist(), N)
    for i in range(5):
        for j in range(4):
            exact = sum(Fraction(A[i, h]) * Fraction(B[h, j]) for h in range(9))
            out = r["out"][i][j]
            na = sum(abs(Fraction(A[i, h])) for h in range(9))
            nb = sum(abs(Fraction(B[h, j])) for h in range(9))
            bound = (nb * Fraction(2) ** -r["mu"][i] + na * Fraction(2) ** -r["nu"][j]
                     + Fraction(abs(out)) * Fraction(2) ** -52)
            assert abs(Fraction(out) - exact) <= bound


def test_error_meets_double_precision_at_14_moduli():
    """Section IV-A / Section II: at 14 moduli the emulated product is at the level of
    double precision, max |out - AB| / (|A||B|) <= 4 k 2^-53."""
    k = 16
    A = _mat(6, k, 0.5, 91)
    B = _mat(k, 5, 0.5, 92)
    for mode in ["fast", "accurate"]:
        r = ref.emulate_real(A.tolist(), B.tolist(), 14, mode)
        worst = Fraction(0)
        for i in range(6):
            for j in range(5):
                exact = sum(Fraction(A[i, h]) * Fraction(B[h, j]) for h in range(k))
                ab = sum(abs(Fraction(A[i, h]) * Fraction(B[h, j])) for h in range(k))
                worst = max(worst, abs(Fraction(r["out"][i][j]) - exact) / ab)
        assert worst <= Fraction(4 * k, 2 ** 53)


def test_alpha_beta_order():
    A = _mat(3, 4, 1.0, 101)
    B = _mat(4, 2, 1.0, 102)
    C = _mat(3, 2, 1.0, 103)
    plain = ref.emulate_real(A.tolist(), B.tolist(), 11)["out"]
    r = ref.emulate_real(A.tolist(), B.tolist(), 11, alpha=-0.75, beta=1.5, C=C.tolist())
    for i in range(3):
        for j in range(2):
            x = float(Fraction(-0.75) * Fraction(plain[i][j]))
            assert r["out"][i][j] == ref.fma(1.5, float(C[i, j]), x)


def _core():
    from oracle import core

    core._load()
    return core


@pytest.mark.parametrize("mode", ["fast", "accurate"])
@pytest.mark.parametrize("N", [2, 7, 14, 20])
def test_c_oracle_equals_reference(mode, N):
    core = _core()
    A = _mat(6, 11, 1.5, 200 + N)
    B = _mat(11, 5, 1.5, 300 + N)
    A[2, :] = 0.0           # a zero row: no scaling, zero output row
    C = _mat(6, 5, 1.0, 400 + N)
    r = ref.emulate_real(A.tolist(), B.tolist(), N, mode, alpha=1.25, beta=-0.5, C=C.tolist())
    c = core.emulate_real(A, B, N, mode, alpha=1.25, beta=-0.5, C=C, want_raw=True)
    assert np.array_equal(c["out"], np.array(r["out"]))
    assert np.array_equal(c["Ep"], np.array(r["Ep"], dtype=np.int8))
    assert np.array_equal(c["raw"], np.array(r["prods"], dtype=np.int64))
    mu_ref = [v if v is not None else 0 for v in r["mu"]]
    ok = c["fa"] == 1
    assert np.array_equal(c["mu"][ok], np.array(mu_ref)[ok])
    assert not ok[2]


@pytest.mark.parametrize("mode", ["fast", "accurate"])
def test_real_equals_complex_with_zero_imaginary_parts(mode):
    """The complex scheme (Section III) on real matrices reduces to the real one: the
    same exponents, E'_I = 0, and the real part of the result bit for bit."""
    core = _core()
    A = _mat(9, 40, 2.0, 501)
    B = _mat(40, 7, 2.0, 502)
    r = core.emulate_real(A, B, 13, mode)
    z = core.emulate(A.astype(np.complex128), B.astype(np.complex128), 13, mode=mode)
    assert np.array_equal(r["mu"], z["mu"]) and np.array_equal(r["nu"], z["nu"])
    assert not z["Ep"][:, 1].any()
    assert np.array_equal(z["out"].real, r["out"]) and not z["out"].imag.any()


def test_single_precision_rounds_once():
    core = _core()
    A = _mat(5, 8, 1.0, 601).astype(np.float32)
    B = _mat(8, 3, 1.0, 602).astype(np.float32)
    r64 = core.emulate_real(A.astype(np.float64), B.astype(np.float64), 9)["out"]
    r32 = core.emulate_real(A, B, 9, single=True)["out"]
    assert r32.dtype == np.float32 and np.array_equal(r32, r64.astype(np.float32))
