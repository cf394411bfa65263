"""The C oracle against the pure-Python reference and against properties at larger sizes,
plus planted mistakes showing that the pins catch them."""
import math

import numpy as np
import pytest

import workloads
from oracle import reference as ref


def _ref_arrays(r, m, n, N):
    mu = np.array([x if x is not None else 0 for x in r["mu"]])
    nu = np.array([x if x is not None else 0 for x in r["nu"]])
    Ep = np.array([[r["Ep"][l][c] for c in range(2)] for l in range(N)], dtype=np.int64)
    return mu, nu, Ep


CASES = [
    # m, n, k, N, phi, mode, algo, alpha, beta
    (3, 4, 5, 14, 0.5, "fast", "karatsuba", 1, 0),
    (4, 3, 6, 8, 2.0, "accurate", "karatsuba", 1, 0),
    (5, 5, 7, 20, 4.0, "fast", "4m", 1, 0),
    (2, 3, 4, 3, 1.0, "accurate", "4m", 1, 0),
    (4, 4, 9, 24, 8.0, "fast", "karatsuba", 0.5 - 2j, 1.5 + 0.25j),
    (3, 2, 3, 24, 8.0, "accurate", "karatsuba", -1, 0.75j),
    (1, 1, 1, 2, 0.0, "fast", "karatsuba", 1, 0),
    (6, 1, 11, 13, 0.5, "accurate", "4m", 2, -1),
]


@pytest.mark.parametrize("m,n,k,N,phi,mode,algo,alpha,beta", CASES)
def test_core_matches_reference_bit_for_bit(orc, m, n, k, N, phi, mode, algo, alpha, beta):
    A = workloads.complex_matrix(m, k, phi, 7 * m + k)
    B = workloads.complex_matrix(k, n, phi, 11 * n + k)
    C = workloads.complex_matrix(m, n, 1.0, 99)
    if m > 2:
        A[1, :] = 0  # an all-zero row
    r = ref.emulate(A.tolist(), B.tolist(), N, mode, algo, alpha, beta, C.tolist())
    c = orc.emulate(A, B, N, mode, algo, alpha, beta, C, want_raw=True)
    mu, nu, Ep = _ref_arrays(r, m, n, N)
    assert np.array_equal(c["mu"], mu) and np.array_equal(c["nu"], nu)
    assert np.array_equal(c["fa"] == orc.FLAG_OK, np.array([x is not None for x in r["mu"]]))
    for l in range(N):
        for pl, name in enumerate("RIS"):
            assert np.array_equal(c["resA"][l, pl], np.array(r["resA"][l][name]))
            assert np.array_equal(c["resB"][l, pl], np.array(r["resB"][l][name]).T)
        keys = ["D", "E", "F"] if algo == "karatsuba" else ["RR", "II", "RI", "IR"]
        for t, key in enumerate(keys):
            assert np.array_equal(c["raw"][l, t], np.array(r["prods"][l][key]))
    assert np.array_equal(c["Ep"], Ep)
    assert np.array_equal(c["out"], np.array(r["out"]))


def test_core_integer_inputs_exact_medium(orc):
    A = workloads.integer_matrix(64, 512, 12, 1)
    B = workloads.integer_matrix(512, 48, 12, 2)
    exact = A @ B  # |partial sums| < 2^35: exact in double
    for mode in ("fast", "accurate"):
        out = orc.emulate(A, B, 14, mode)["out"]
        assert np.array_equal(out, exact)


def test_core_algorithms_and_transpose_medium(orc):
    A = workloads.complex_matrix(40, 300, 2.0, 3)
    B = workloads.complex_matrix(300, 33, 2.0, 4)
    for mode in ("fast", "accurate"):
        k3 = orc.emulate(A, B, 13, mode, "karatsuba")
        k4 = orc.emulate(A, B, 13, mode, "4m")
        assert np.array_equal(k3["Ep"], k4["Ep"]) and np.array_equal(k3["out"], k4["out"])
        t = orc.emulate(B.T, A.T, 13, mode, "karatsuba")
        assert np.array_equal(t["out"].T, k3["out"])


def test_core_nonfinite_rows_and_columns(orc):
    A = workloads.complex_matrix(5, 6, 1.0, 5)
    B = workloads.complex_matrix(6, 4, 1.0, 6)
    A2 = A.copy()
    A2[2, 3] = complex(np.inf, 0.0)
    B2 = B.copy()
    B2[1, 0] = complex(0.0, np.nan)
    base = orc.emulate(A, B, 14)["out"]
    got = orc.emulate(A2, B2, 14)["out"]
    bad = np.zeros((5, 4), bool)
    bad[2, :] = True
    bad[:, 0] = True
    assert np.isnan(got[bad].real).all() and np.isnan(got[bad].imag).all()
    assert np.array_equal(got[~bad], base[~bad])


def test_core_single_precision_rounding(orc):
    """CGEMM: inputs promoted exactly, result = fl32 of the double-precision result."""
    A = workloads.complex_matrix(8, 20, 0.5, 8, dtype=np.complex64)
    B = workloads.complex_matrix(20, 8, 0.5, 9, dtype=np.complex64)
    c = orc.emulate(A, B, 7, single=True)["out"]
    d = orc.emulate(A.astype(np.complex128), B.astype(np.complex128), 7)["out"]
    assert c.dtype == np.complex64 and np.array_equal(c, d.astype(np.complex64))


# ------------------------------------------------------------ planted mistakes (on the CPU)

def _reconstruction_pin_holds(emulate_fn):
    A = workloads.complex_matrix(3, 5, 1.0, 123).tolist()
    B = workloads.complex_matrix(5, 3, 1.0, 124).tolist()
    r = emulate_fn(A, B, 10, "fast", "karatsuba")
    CpR, CpI = r["Cp"]
    Ai, Bi = r["Ai"], r["Bi"]
    for i in range(3):
        for j in range(3):
            re = sum(Ai[i][h][0] * Bi[h][j][0] - Ai[i][h][1] * Bi[h][j][1] for h in range(5))
            im = sum(Ai[i][h][0] * Bi[h][j][1] + Ai[i][h][1] * Bi[h][j][0] for h in range(5))
            if CpR[i][j] != re or CpI[i][j] != im:
                return False
    return True


def test_planted_mistakes_are_caught(monkeypatch):
    assert _reconstruction_pin_holds(ref.emulate)
    # 1) a non-symmetric remainder: negative results no longer come back
    with monkeypatch.context() as mp:
        mp.setattr(ref, "smod", lambda x, p: x % p)
        assert not _reconstruction_pin_holds(ref.emulate)
    # 2) a wrong CRT inverse
    orig = ref.crt_constants

    def bad_constants(n):
        p, P, q, s = orig(n)
        q = list(q)
        q[3] = (q[3] + 1) % p[3]
        return p, P, q, [(P // pl) * ql for pl, ql in zip(p, q)]

    with monkeypatch.context() as mp:
        mp.setattr(ref, "crt_constants", bad_constants)
        assert not _reconstruction_pin_holds(ref.emulate)
    # 3) an exponent two steps too large breaks the uniqueness condition (4)
    orig_fast = ref.fast_exponent

    def greedy(row, P):
        mu, e, sig = orig_fast(row, P)
        return (mu + 3 if mu is not None else None), e, sig

    with monkeypatch.context() as mp:
        mp.setattr(ref, "fast_exponent", greedy)
        assert not _reconstruction_pin_holds(ref.emulate)


@pytest.mark.parametrize("mode", ["fast", "accurate"])
@pytest.mark.parametrize("N", [8, 16, 24])
def test_double_double_low_parts(orc, mode, N):
    """The low part of the double-double value of the scaled C' (the reconstruction is
    exact): with hi = RNE(C') and lo = RNE(C' - hi), both scaled by 2^-(mu + nu), the C
    oracle agrees with Python integers (float() of an int rounds to nearest even), and
    hi + lo is C' exactly while |C' - hi| < 2^53."""
    from fractions import Fraction

    from oracle import reference as ref

    A = workloads.complex_matrix(4, 9, 3.0, 700 + N)
    B = workloads.complex_matrix(9, 3, 3.0, 800 + N)
    r = ref.emulate(A.tolist(), B.tolist(), N, mode)
    c = orc.emulate(A, B, N, mode, want_lo=True)
    CpR, CpI = r["Cp"]
    for i in range(4):
        for j in range(3):
            sh = -(r["mu"][i] + r["nu"][j])
            for part, cp in ((0, CpR[i][j]), (1, CpI[i][j])):
                hi = float(cp)
                lo = float(cp - int(hi))
                got_hi = (c["out"][i, j].real, c["out"][i, j].imag)[part]
                got_lo = (c["lo"][i, j].real, c["lo"][i, j].imag)[part]
                assert got_hi == math.ldexp(hi, sh) and got_lo == math.ldexp(lo, sh)
                if abs(cp - int(hi)) < 2 ** 53:
                    assert Fraction(got_hi) + Fraction(got_lo) == Fraction(cp) * Fraction(2) ** sh
