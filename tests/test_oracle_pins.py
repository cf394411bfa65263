"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a property that
holds independently of how the oracle is written (a congruence, the CRT basis
identity, an exact product computed by brute force, a closed-form error
bound, an invariance, a value computed from the paper's printed formula).
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import reference as ref


# ------------------------------------------------------------ moduli / CRT (Alg. 1 Steps I-II)

def test_moduli_pairwise_coprime_greedy():
    p = ref.moduli(24)
    assert p[0] == 256 and all(x <= 256 for x in p)
    assert all(a > b for a, b in zip(p, p[1:]))
    for i in range(len(p)):
        for j in range(i):
            assert math.gcd(p[i], p[j]) == 1
    # greedy: every integer skipped between two chosen moduli shares a factor with an earlier one
    for c in range(p[-1] + 1, 257):
        if c not in p:
            assert any(math.gcd(c, x) > 1 for x in p if x > c)


def test_smod_range_and_congruence():
    """smod(x, p) is the unique r = x (mod p) in [-floor(p/2), ceil(p/2) - 1] (Section II)."""
    rnd = random.Random(1)
    xs = list(range(-3000, 3001)) + [rnd.randrange(-(1 << 100), 1 << 100) for _ in range(2000)]
    for p in ref.moduli(24):
        lo, hi = -(p // 2), (p + 1) // 2 - 1
        for x in xs:
            r = ref.smod(x, p)
            assert lo <= r <= hi and (x - r) % p == 0
    # the residue range fits INT8 (Section II: symmetric residues are INT8)
    assert ref.smod(128, 256) == -128 and ref.smod(-128, 256) == -128


@pytest.mark.parametrize("n", [2, 6, 13, 14, 20, 24])
def test_crt_basis_identity(n):
    """s_l = (P/p_l) q_l is 1 mod p_l and 0 mod every other modulus (Step II)."""
    p, P, q, s = ref.crt_constants(n)
    assert P == math.prod(p)
    for l in range(n):
        assert 1 <= q[l] < p[l]
        assert 0 < s[l] < P
        for j in range(n):
            assert s[l] % p[j] == (1 if j == l else 0)


def test_crt_reconstructs_any_integer_in_range():
    """Sum_l s_l mod(x, p_l) reduced mod P gives back x for |x| < P/2 (Section II)."""
    rnd = random.Random(7)
    p, P, q, s = ref.crt_constants(14)
    for _ in range(500):
        x = rnd.randrange(-(P // 2), P // 2)
        S = sum(sl * ref.smod(x, pl) for sl, pl in zip(s, p))
        assert ref.smod(S, P) == x


# ------------------------------------------------------------ the exact integer product

def _rand_cases():
    rnd = random.Random(3)
    for trial in range(14):
        m, n, k = rnd.randint(1, 4), rnd.randint(1, 4), rnd.randint(1, 6)
        N = rnd.choice([2, 3, 5, 8, 12, 14, 16, 20])
        phi = rnd.choice([0.0, 0.5, 2.0, 4.0])
        mode = rnd.choice(["fast", "accurate"])
        algo = rnd.choice(["karatsuba", "4m"])
        yield m, n, k, N, phi, mode, algo, 100 + trial


@pytest.mark.parametrize("m,n,k,N,phi,mode,algo,seed", list(_rand_cases()))
def test_reconstruction_equals_integer_product(m, n, k, N, phi, mode, algo, seed):
    """C' equals A'B' computed directly from the truncated integers, and the
    uniqueness condition (4) holds for every entry (Section II; eqs. (7), (10))."""
    A = workloads.complex_matrix(m, k, phi, seed).tolist()
    B = workloads.complex_matrix(k, n, phi, seed + 1).tolist()
    r = ref.emulate(A, B, N, mode, algo)
    CpR, CpI = r["Cp"]
    Ai, Bi = r["Ai"], r["Bi"]
    P = r["P"]
    for i in range(m):
        for j in range(n):
            re = sum(Ai[i][h][0] * Bi[h][j][0] - Ai[i][h][1] * Bi[h][j][1] for h in range(k))
            im = sum(Ai[i][h][0] * Bi[h][j][1] + Ai[i][h][1] * Bi[h][j][0] for h in range(k))
            bound = sum(abs(Ai[i][h][0]) * abs(Bi[h][j][0]) + abs(Ai[i][h][1]) * abs(Bi[h][j][1])
                        for h in range(k))
            bound_i = sum(abs(Ai[i][h][0]) * abs(Bi[h][j][1]) + abs(Ai[i][h][1]) * abs(Bi[h][j][0])
                          for h in range(k))
            assert 2 * bound < P and 2 * bound_i < P
            assert CpR[i][j] == re and CpI[i][j] == im


def test_karatsuba_and_expanded_give_identical_residues():
    """Equations (7) and (10) are integer identities: E' agrees bit for bit."""
    A = workloads.complex_matrix(5, 9, 1.0, 11).tolist()
    B = workloads.complex_matrix(9, 4, 1.0, 12).tolist()
    for N in (3, 14):
        a = ref.emulate(A, B, N, "fast", "karatsuba")
        b = ref.emulate(A, B, N, "fast", "4m")
        assert a["Ep"] == b["Ep"] and a["out"] == b["out"]


def test_integer_inputs_give_exact_product():
    """Integer-valued inputs are scaled up without truncation, so the result is AB exactly."""
    A = workloads.integer_matrix(6, 24, 10, 21)
    B = workloads.integer_matrix(24, 5, 10, 22)
    exact = A @ B  # all partial sums < 2^26: exact in double
    for mode in ("fast", "accurate"):
        r = ref.emulate(A.tolist(), B.tolist(), 12, mode)
        assert all(mu >= 0 for mu in r["mu"])
        assert np.array_equal(np.array(r["out"]), exact)


@pytest.mark.parametrize("seed,phi,N,mode", [(31, 0.5, 6, "fast"), (32, 4.0, 10, "fast"),
                                             (33, 2.0, 8, "accurate"), (34, 0.5, 3, "accurate")])
def test_truncation_error_closed_form(seed, phi, N, mode):
    """|C - out| <= 2^-mu_i ||b_j||_1 + 2^-nu_j ||a_i||_1 + ulp (1-norms over the 2k reals),
    from |a 2^mu - trunc(a 2^mu)| < 1 (Step IV)."""
    m, n, k = 3, 3, 7
    A = workloads.complex_matrix(m, k, phi, seed).tolist()
    B = workloads.complex_matrix(k, n, phi, seed + 50).tolist()
    r = ref.emulate(A, B, N, mode)
    ex = ref.exact_product(A, B)
    for i in range(m):
        a1 = sum(Fraction(abs(z.real)) + Fraction(abs(z.imag)) for z in A[i])
        for j in range(n):
            b1 = sum(Fraction(abs(B[h][j].real)) + Fraction(abs(B[h][j].imag)) for h in range(k))
            bound = b1 * Fraction(2) ** (-r["mu"][i]) + a1 * Fraction(2) ** (-r["nu"][j])
            for comp, val in ((0, r["out"][i][j].real), (1, r["out"][i][j].imag)):
                e = ex[i][j][comp]
                ulp = Fraction(math.ulp(float(e))) if e != 0 else Fraction(0)
                assert abs(Fraction(val) - e) <= bound + ulp


def test_row_power_of_two_scaling_is_exact():
    """Scaling row i of A by 2^s shifts mu_i by -s and scales the output row by 2^s exactly."""
    A = workloads.complex_matrix(4, 6, 2.0, 41)
    B = workloads.complex_matrix(6, 3, 2.0, 42)
    shifts = np.array([0, 7, -13, 300])
    A2 = workloads.skewed(A, row_exp=shifts)
    for mode in ("fast", "accurate"):
        r1 = ref.emulate(A.tolist(), B.tolist(), 12, mode)
        r2 = ref.emulate(A2.tolist(), B.tolist(), 12, mode)
        assert r1["Ai"] == r2["Ai"]
        for i in range(4):
            assert r2["mu"][i] == r1["mu"][i] - shifts[i]
            for j in range(3):
                o1, o2 = r1["out"][i][j], r2["out"][i][j]
                assert o2.real == math.ldexp(o1.real, int(shifts[i]))
                assert o2.imag == math.ldexp(o1.imag, int(shifts[i]))


def test_transpose_and_conjugate_symmetry():
    """(AB)^T = B^T A^T and conj(A)conj(B) = conj(AB) hold bit for bit."""
    A = workloads.complex_matrix(3, 5, 1.0, 51)
    B = workloads.complex_matrix(5, 4, 1.0, 52)
    for mode in ("fast", "accurate"):
        for algo in ("karatsuba", "4m"):
            r = ref.emulate(A.tolist(), B.tolist(), 9, mode, algo)
            rt = ref.emulate(B.T.tolist(), A.T.tolist(), 9, mode, algo)
            rc = ref.emulate(A.conj().tolist(), B.conj().tolist(), 9, mode, algo)
            out = np.array(r["out"])
            assert np.array_equal(np.array(rt["out"]).T, out)
            assert np.array_equal(np.array(rc["out"]), out.conj())


# ------------------------------------------------------------ scaling rules vs the printed formulas

def _log2_exact(x) -> float:
    """log2 of a positive rational, accurate to ~1e-15 (enough to compare floors away from ties)."""
    x = Fraction(x)
    e = x.numerator.bit_length() - x.denominator.bit_length()
    return e + math.log2(float(x / Fraction(2) ** e))


def test_fast_exponent_matches_printed_rule():
    """Fast mode (Section III-B): mu_i = floor(P' - max(1, log2||a_i~||_2)) - floor(log2 max|a|)
    with P' = log2(P-1)/2 - 1.5 and a_i~ the row normalised by its top exponent.  The oracle's
    integer rule rounds the normalised magnitudes up (at most one exponent lower)."""
    rnd = random.Random(5)
    hits = 0
    for trial in range(300):
        N = rnd.choice([4, 8, 13, 14, 18, 20])
        k = rnd.randint(1, 40)
        row = list(np.asarray(workloads.complex_matrix(1, k, rnd.choice([0.5, 2, 8]), 500 + trial)).ravel())
        vals = [z.real for z in row] + [z.imag for z in row]
        _, P, _, _ = ref.crt_constants(N)
        mu, e, sigma = ref.fast_exponent(vals, P)
        norm2 = sum(Fraction(v) ** 2 for v in vals) / Fraction(4) ** e
        Pf = math.log2(P - 1) / 2 - 1.5
        printed = math.floor(Pf - max(1.0, 0.5 * _log2_exact(norm2))) - e
        assert printed - 1 <= mu <= printed
        hits += mu == printed
    assert hits >= 290


def test_accurate_exponent_matches_printed_rule():
    """Accurate mode (Section III-B): mu_i = mubar_i * 2^floor(P'_accu - log2(max_h max(Cbar))/2),
    P'_accu = log2(P-1)/2 - 0.5, mubar_i = 2^(5 - floor(log2 max|a_i|)); Cbar_R equals both
    Cbar_I + (AR-AI)(BR-BI) and AR BR + AI BI."""
    A = workloads.complex_matrix(5, 8, 3.0, 61).tolist()
    B = workloads.complex_matrix(8, 6, 3.0, 62).tolist()
    for N in (5, 13, 17):
        _, P, _, _ = ref.crt_constants(N)
        mu, nu, d = ref.accurate_exponents(A, B, P)
        for i in range(5):
            for j in range(6):
                direct = sum(d["AR"][i][h] * d["BR"][h][j] + d["AI"][i][h] * d["BI"][h][j]
                             for h in range(8))
                assert d["CR"][i][j] == direct
        Pa = math.log2(P - 1) / 2 - 0.5
        for i in range(5):
            printed = (5 - d["eA"][i]) + math.floor(Pa - 0.5 * math.log2(d["X"][i]))
            assert mu[i] == printed
            assert all(0 <= v <= 64 for v in d["AR"][i] + d["AI"][i])


# ------------------------------------------------------------ accuracy behaviour (Section IV-A)

def test_error_decreases_with_moduli_and_meets_fp64_bound(orc):
    """More moduli enlarge P and shrink the error until it meets the double-precision bound."""
    m = n = 48
    k = 256
    A = workloads.complex_matrix(m, k, 0.5, 71)
    B = workloads.complex_matrix(k, n, 0.5, 72)
    hi, lo = orc.dd_gemm(A, B)
    absab = orc.abs_product(A, B)
    errs = {}
    for N in (8, 10, 12, 14, 16):
        out = orc.emulate(A, B, N, "fast")["out"]
        errs[N] = orc.err_nc(out, hi, lo, absab)
    assert errs[8] > errs[10] > errs[12] > errs[14]
    assert errs[14] <= 4 * k * 2.0 ** -53 and errs[16] <= 4 * k * 2.0 ** -53
    # a native double GEMM for context: same order of magnitude as fast-14 or better
    native = orc.err_nc(A @ B, hi, lo, absab)
    assert native <= 4 * k * 2.0 ** -53


def test_dd_gemm_against_exact_rationals(orc):
    """Double-double product within 4k 2^-104 (|A||B|) of the exact rational product."""
    A = workloads.complex_matrix(3, 17, 4.0, 81)
    B = workloads.complex_matrix(17, 2, 4.0, 82)
    hi, lo = orc.dd_gemm(A, B)
    ex = ref.exact_product(A.tolist(), B.tolist())
    absab = np.abs(A.real) @ np.abs(B.real) + np.abs(A.imag) @ np.abs(B.imag) \
        + np.abs(A.real) @ np.abs(B.imag) + np.abs(A.imag) @ np.abs(B.real)
    for i in range(3):
        for j in range(2):
            got_r = Fraction(hi[i, j].real) + Fraction(lo[i, j].real)
            got_i = Fraction(hi[i, j].imag) + Fraction(lo[i, j].imag)
            tol = Fraction(4 * 17) * Fraction(2) ** -104 * Fraction(float(absab[i, j]) * 2)
            assert abs(got_r - ex[i][j][0]) <= tol and abs(got_i - ex[i][j][1]) <= tol


def test_alpha_beta_sequence():
    """out = alpha*c + beta*C with exactly representable data gives the exact value."""
    c = complex(3.0, -2.0)
    cin = complex(0.5, 4.0)
    out = ref.apply_alpha_beta(c, complex(2.0, 1.0), complex(-1.0, 0.5), cin)
    assert out == (2 + 1j) * c + (-1 + 0.5j) * cin
    assert ref.apply_alpha_beta(c, 1, 0, None) == c
