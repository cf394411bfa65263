"""Exact-integer reference of the complex Ozaki-II scheme, written to be read.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
module; only the tests, the smoke check and the CPU baseline of the benchmark
use it.  It is deliberately slow (pure Python integers and fractions) and is
meant for tiny matrices; ``oracle.core`` is the same computation in C for
larger shapes and is pinned against this file.

The steps follow the paper (arXiv 2512.08321):

* Section II, Algorithm 1: moduli (Step I), CRT inverses (Step II), scaling
  vectors (Step III), truncation to integers (Step IV), residues, modular
  products, symmetric reduction, CRT accumulation and final reduction modulo P
  (Step V), inverse scaling (Step VI).
* Section III-A, equations (7), (8), (10): the complex product either as the
  expanded real product (4 real products) or by Karatsuba (3 products).
* Section III-B: fast-mode scaling (Cauchy-Schwarz bound) and accurate-mode
  scaling (an extra product of 7-bit ceiling matrices).

Readings of passages that the paper leaves open:

* The moduli are the greedy descending pairwise-coprime integers <= 256, in
  that order; the first N are used.
* The symmetric remainder maps into [-floor(p/2), ceil(p/2) - 1]; for p = 256
  the tie x = 128 (mod 256) goes to -128.
* q_l is taken in [1, p_l - 1], so s_l = (P/p_l) q_l lies in (0, P).
* Fast mode: the sum of squares of a row is taken after normalising the row by
  2^-e (e = exponent of the row's largest magnitude), each normalised
  magnitude rounded up to SIGMA_FRAC_BITS fractional bits; the paper's
  logarithm bound is replaced by the exact integer test it approximates.
* Accurate mode: one exponent per row shared by the real and imaginary parts;
  the 7-bit matrices are ceil(|x| * 2^(5-e)).
* A row (column) for which the method's bound is zero (an all-zero row, or in
  accurate mode a row whose bound product vanishes) contributes nothing: its
  integers are all zero and its exponent is reported as ``None``.
* Output: out = ldexp(RNE(C'), -(mu_i + nu_j)); alpha/beta are applied with
  the fused multiply-add sequence documented in ``apply_alpha_beta``.
"""
from __future__ import annotations

import math
from fractions import Fraction

MAX_MODULI = 24
SIGMA_FRAC_BITS = 20     # fixed-point fraction bits of the fast-mode sum of squares
ACCU_INT_BITS = 6        # accurate mode: magnitudes scaled below 2^6 before the ceiling


# ---------------------------------------------------------------- Step I / II

def moduli(n: int) -> list[int]:
    """First n of the greedy descending pairwise-coprime integers <= 256 (Step I)."""
    if not 1 <= n <= MAX_MODULI:
        raise ValueError("number of moduli out of range")
    chosen: list[int] = []
    cand = 256
    while len(chosen) < n:
        if all(math.gcd(cand, p) == 1 for p in chosen):
            chosen.append(cand)
        cand -= 1
    return chosen


def crt_constants(n: int):
    """P, q_l = (P/p_l)^-1 mod p_l and s_l = (P/p_l) q_l (Step II; Section II)."""
    p = moduli(n)
    P = math.prod(p)
    q = [pow(P // pl, -1, pl) for pl in p]
    s = [(P // pl) * ql for pl, ql in zip(p, q)]
    return p, P, q, s


def smod(x: int, p: int) -> int:
    """Symmetric remainder x - p*round(x/p) (Section II), ties toward -p/2."""
    return x - p * ((2 * x + p) // (2 * p))


# ---------------------------------------------------------------- Step III

def ufp_exponent(x: float) -> int:
    """floor(log2 |x|) for x != 0 (the exponent returned by ilogb)."""
    return math.frexp(abs(x))[1] - 1


def _pow2(e: int) -> Fraction:
    return Fraction(2) ** e


def fast_t_max(P: int) -> int:
    """Largest integer t with t <= P'_fast - 1, i.e. 2^(2t+5) <= P - 1.

    P'_fast = log2(P-1)/2 - 1.5 (Section III-B); the max(1, .) clamp of the
    fast-mode rule contributes the bound t <= P'_fast - 1.
    """
    t = (P - 1).bit_length()  # safely above
    while Fraction(2) ** (2 * t + 5) > P - 1:
        t -= 1
    return t


def fast_exponent(row: list[float], P: int):
    """Fast-mode scaling exponent of one row of A-hat (Section III-B, fast mode).

    ``row`` holds the 2k real numbers of the row (real and imaginary parts).
    Returns (mu, e, sigma) where mu is the exponent of mu_i = 2^mu, or
    (None, None, 0) for an all-zero row.

    The bound mu_i * ||a_i||_2 <= 2^(P'_fast) is what makes the Cauchy-Schwarz
    estimate satisfy the uniqueness condition (4); with the row normalised by
    2^-e, ||a_i||^2 <= 2^(2e) * sigma / 2^(2F), so t = mu + e must satisfy
    t <= P'_fast - 1 and 8 * sigma * 4^t <= (P - 1) * 2^(2F).
    """
    nz = [v for v in row if v != 0.0]
    if not nz:
        return None, None, 0
    e = max(ufp_exponent(v) for v in nz)
    F = SIGMA_FRAC_BITS
    sigma = sum(math.ceil(Fraction(abs(v)) * _pow2(F - e)) ** 2 for v in row)
    t = fast_t_max(P)
    while 8 * sigma * _pow2(2 * t) > (P - 1) * _pow2(2 * F):
        t -= 1
    return t - e, e, sigma


def accurate_t(X: int, P: int) -> int:
    """Largest t with 2 * X * 4^t <= P - 1 (accurate mode, Section III-B)."""
    t = (P - 1).bit_length()
    while 2 * X * _pow2(2 * t) > P - 1:
        t -= 1
    return t


def ceil7(x: float, e: int) -> int:
    """ceil(|x| * 2^(5-e)), an integer in [0, 64] when |x| < 2^(e+1)."""
    return math.ceil(Fraction(abs(x)) * _pow2(ACCU_INT_BITS - 1 - e))


def accurate_exponents(A, B, P: int):
    """Accurate-mode exponents for op(A) (m x k) and op(B) (k x n) (Section III-B).

    Builds the 7-bit matrices Abar_R, Abar_I, Bbar_R, Bbar_I, the bound product
    Cbar_I = Abar_I Bbar_R + Abar_R Bbar_I and
    Cbar_R = Cbar_I + (Abar_R - Abar_I)(Bbar_R - Bbar_I), and then per row the
    largest t with 2 * max_j max(Cbar_R, Cbar_I)_ij * 4^t <= P - 1.
    Returns (mu, nu, details).
    """
    m, k, n = len(A), len(B), len(B[0]) if B else 0

    def row_exp(vals):
        nz = [v for v in vals if v != 0.0]
        return max(ufp_exponent(v) for v in nz) if nz else None

    eA = [row_exp([z.real for z in A[i]] + [z.imag for z in A[i]]) for i in range(m)]
    eB = [row_exp([B[h][j].real for h in range(k)] + [B[h][j].imag for h in range(k)])
          for j in range(n)]
    AR = [[ceil7(A[i][h].real, eA[i]) if eA[i] is not None else 0 for h in range(k)] for i in range(m)]
    AI = [[ceil7(A[i][h].imag, eA[i]) if eA[i] is not None else 0 for h in range(k)] for i in range(m)]
    BR = [[ceil7(B[h][j].real, eB[j]) if eB[j] is not None else 0 for j in range(n)] for h in range(k)]
    BI = [[ceil7(B[h][j].imag, eB[j]) if eB[j] is not None else 0 for j in range(n)] for h in range(k)]
    CI = [[sum(AI[i][h] * BR[h][j] + AR[i][h] * BI[h][j] for h in range(k)) for j in range(n)]
          for i in range(m)]
    CR = [[CI[i][j] + sum((AR[i][h] - AI[i][h]) * (BR[h][j] - BI[h][j]) for h in range(k))
           for j in range(n)] for i in range(m)]
    X = [max([max(CR[i][j], CI[i][j]) for j in range(n)], default=0) for i in range(m)]
    Y = [max([max(CR[i][j], CI[i][j]) for i in range(m)], default=0) for j in range(n)]
    base = ACCU_INT_BITS - 1
    mu = [None if (eA[i] is None or X[i] == 0) else base - eA[i] + accurate_t(X[i], P)
          for i in range(m)]
    nu = [None if (eB[j] is None or Y[j] == 0) else base - eB[j] + accurate_t(Y[j], P)
          for j in range(n)]
    details = dict(eA=eA, eB=eB, AR=AR, AI=AI, BR=BR, BI=BI, CR=CR, CI=CI, X=X, Y=Y)
    return mu, nu, details


# ---------------------------------------------------------------- Step IV

def trunc_scaled(x: float, mu) -> int:
    """trunc(x * 2^mu), exactly (Step IV); zero for a row without exponent."""
    if mu is None:
        return 0
    return int(Fraction(x) * _pow2(mu))  # int() of a Fraction truncates toward zero


# ---------------------------------------------------------------- output

def fma(a: float, b: float, c: float) -> float:
    """Correctly rounded a*b + c (finite operands)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def apply_alpha_beta(c: complex, alpha: complex, beta: complex, cin) -> complex:
    """out = alpha*c + beta*cin with the fixed operation order of the library.

    x_r = fma(alpha_r, c_r, -(alpha_i * c_i)),  x_i = fma(alpha_r, c_i, alpha_i * c_r)
    beta == 0: out = x (cin is not read)
    else: out_r = fma(beta_r, cin_r, fma(-beta_i, cin_i, x_r))
          out_i = fma(beta_r, cin_i, fma(beta_i, cin_r, x_i))
    """
    ar, ai = float(alpha.real), float(alpha.imag)
    xr = fma(ar, c.real, -(ai * c.imag))
    xi = fma(ar, c.imag, ai * c.real)
    if beta == 0:
        return complex(xr, xi)
    br, bi = float(beta.real), float(beta.imag)
    return complex(fma(br, cin.real, fma(-bi, cin.imag, xr)),
                   fma(br, cin.imag, fma(bi, cin.real, xi)))


# ---------------------------------------------------------------- pipeline

def emulate(A, B, n_moduli: int, mode: str = "fast", algo: str = "karatsuba",
            alpha: complex = 1, beta: complex = 0, C=None):
    """C = alpha * A @ B + beta * C by the complex Ozaki-II scheme, exactly.

    A: m lists of k complex numbers (op(A)); B: k lists of n complex numbers.
    Returns a dict with every intermediate:
      mu, nu            scaling exponents (None for a zero row/column)
      Ai, Bi            truncated integers (pairs (re, im))
      resA, resB        per modulus: dict of residue matrices 'R', 'I', 'S'
      prods             per modulus: the integer products of the chosen algorithm
      Ep                per modulus: (E'_R, E'_I) symmetric residues of C' mod p_l
      Cp                (C'_R, C'_I) reconstructed integers
      out               output as complex floats
    """
    m, k = len(A), len(B)
    n = len(B[0]) if B else 0
    p, P, q, s = crt_constants(n_moduli)

    # Step III
    if mode == "fast":
        mu = [fast_exponent([z.real for z in A[i]] + [z.imag for z in A[i]], P)[0]
              for i in range(m)]
        nu = [fast_exponent([B[h][j].real for h in range(k)] + [B[h][j].imag for h in range(k)], P)[0]
              for j in range(n)]
    elif mode == "accurate":
        mu, nu, _ = accurate_exponents(A, B, P)
    else:
        raise ValueError(mode)

    # Step IV
    Ai = [[(trunc_scaled(A[i][h].real, mu[i]), trunc_scaled(A[i][h].imag, mu[i]))
           for h in range(k)] for i in range(m)]
    Bi = [[(trunc_scaled(B[h][j].real, nu[j]), trunc_scaled(B[h][j].imag, nu[j]))
           for j in range(n)] for h in range(k)]

    resA, resB, prods, Ep = [], [], [], []
    for pl in p:
        # Step V-i, V-ii; the Karatsuba sums are reduced before the product (Sec. III-A)
        ra = {"R": [[smod(Ai[i][h][0], pl) for h in range(k)] for i in range(m)],
              "I": [[smod(Ai[i][h][1], pl) for h in range(k)] for i in range(m)]}
        ra["S"] = [[smod(ra["R"][i][h] + ra["I"][i][h], pl) for h in range(k)] for i in range(m)]
        rb = {"R": [[smod(Bi[h][j][0], pl) for j in range(n)] for h in range(k)],
              "I": [[smod(Bi[h][j][1], pl) for j in range(n)] for h in range(k)]}
        rb["S"] = [[smod(rb["R"][h][j] + rb["I"][h][j], pl) for j in range(n)] for h in range(k)]
        resA.append(ra)
        resB.append(rb)

        def mm(X, Y):
            return [[sum(X[i][h] * Y[h][j] for h in range(k)) for j in range(n)] for i in range(m)]

        # Step V-iii / V-iv
        if algo == "karatsuba":          # equation (10)
            D, E, Fm = mm(ra["R"], rb["R"]), mm(ra["I"], rb["I"]), mm(ra["S"], rb["S"])
            prods.append({"D": D, "E": E, "F": Fm})
            ER = [[smod(D[i][j] - E[i][j], pl) for j in range(n)] for i in range(m)]
            EI = [[smod(Fm[i][j] - D[i][j] - E[i][j], pl) for j in range(n)] for i in range(m)]
        elif algo == "4m":               # equation (7)
            RR, II = mm(ra["R"], rb["R"]), mm(ra["I"], rb["I"])
            RI, IR = mm(ra["R"], rb["I"]), mm(ra["I"], rb["R"])
            prods.append({"RR": RR, "II": II, "RI": RI, "IR": IR})
            ER = [[smod(RR[i][j] - II[i][j], pl) for j in range(n)] for i in range(m)]
            EI = [[smod(RI[i][j] + IR[i][j], pl) for j in range(n)] for i in range(m)]
        else:
            raise ValueError(algo)
        Ep.append((ER, EI))

    # Step V-v / V-vi: S = sum_l s_l E'_l, C' = mod(S, P)
    CpR = [[smod(sum(s[l] * Ep[l][0][i][j] for l in range(n_moduli)), P) for j in range(n)]
           for i in range(m)]
    CpI = [[smod(sum(s[l] * Ep[l][1][i][j] for l in range(n_moduli)), P) for j in range(n)]
           for i in range(m)]

    # Step VI: inverse scaling, then alpha/beta
    out = []
    for i in range(m):
        row = []
        for j in range(n):
            if mu[i] is None or nu[j] is None:
                c = complex(0.0, 0.0)
            else:
                sh = -(mu[i] + nu[j])
                c = complex(math.ldexp(float(CpR[i][j]), sh), math.ldexp(float(CpI[i][j]), sh))
            cin = C[i][j] if (C is not None and beta != 0) else 0j
            row.append(apply_alpha_beta(c, complex(alpha), complex(beta), cin))
        out.append(row)
    return dict(p=p, P=P, q=q, s=s, mu=mu, nu=nu, Ai=Ai, Bi=Bi, resA=resA, resB=resB,
                prods=prods, Ep=Ep, Cp=(CpR, CpI), out=out)


def emulate_real(A, B, n_moduli: int, mode: str = "fast", alpha: float = 1.0, beta: float = 0.0,
                 C=None):
    """C = alpha * A @ B + beta * C for real matrices by Algorithm 1, exactly.

    A: m lists of k floats; B: k lists of n floats.  Step I/II: moduli and CRT
    constants; Step III: fast mode by the Cauchy-Schwarz rule on the k reals of a
    row (Section II; Section III-B states the same rule for the 2k reals of a
    complex row), accurate mode with the bound Abar Bbar of the 7-bit ceilings;
    Step IV: a' = trunc(a 2^mu); Step V: residues, D'_l = A'_l B'_l,
    E'_l = mod(D'_l, p_l), S = sum_l s_l E'_l, C' = mod(S, P); Step VI:
    ldexp(C', -(mu_i + nu_j)) rounded to nearest, x = alpha c, and
    out = x (beta = 0) or fma(beta, C_in, x).
    """
    m, k = len(A), len(B)
    n = len(B[0]) if B else 0
    p, P, q, s = crt_constants(n_moduli)
    if mode == "fast":
        mu = [fast_exponent(list(A[i]), P)[0] for i in range(m)]
        nu = [fast_exponent([B[h][j] for h in range(k)], P)[0] for j in range(n)]
    elif mode == "accurate":
        def row_exp(vals):
            nz = [v for v in vals if v != 0.0]
            return max(ufp_exponent(v) for v in nz) if nz else None
        eA = [row_exp(list(A[i])) for i in range(m)]
        eB = [row_exp([B[h][j] for h in range(k)]) for j in range(n)]
        Ab = [[ceil7(A[i][h], eA[i]) if eA[i] is not None else 0 for h in range(k)] for i in range(m)]
        Bb = [[ceil7(B[h][j], eB[j]) if eB[j] is not None else 0 for j in range(n)] for h in range(k)]
        Cb = [[sum(Ab[i][h] * Bb[h][j] for h in range(k)) for j in range(n)] for i in range(m)]
        X = [max(Cb[i], default=0) for i in range(m)]
        Y = [max([Cb[i][j] for i in range(m)], default=0) for j in range(n)]
        base = ACCU_INT_BITS - 1
        mu = [None if (eA[i] is None or X[i] == 0) else base - eA[i] + accurate_t(X[i], P)
              for i in range(m)]
        nu = [None if (eB[j] is None or Y[j] == 0) else base - eB[j] + accurate_t(Y[j], P)
              for j in range(n)]
    else:
        raise ValueError(mode)
    Ai = [[trunc_scaled(A[i][h], mu[i]) for h in range(k)] for i in range(m)]
    Bi = [[trunc_scaled(B[h][j], nu[j]) for j in range(n)] for h in range(k)]
    Ep, prods = [], []
    for pl in p:
        Al = [[smod(Ai[i][h], pl) for h in range(k)] for i in range(m)]
        Bl = [[smod(Bi[h][j], pl) for j in range(n)] for h in range(k)]
        D = [[sum(Al[i][h] * Bl[h][j] for h in range(k)) for j in range(n)] for i in range(m)]
        prods.append(D)
        Ep.append([[smod(D[i][j], pl) for j in range(n)] for i in range(m)])
    Cp = [[smod(sum(s[l] * Ep[l][i][j] for l in range(n_moduli)), P) for j in range(n)]
          for i in range(m)]
    out = []
    for i in range(m):
        row = []
        for j in range(n):
            c = 0.0
            if mu[i] is not None and nu[j] is not None:
                c = math.ldexp(float(Cp[i][j]), -(mu[i] + nu[j]))
            x = float(alpha) * c
            row.append(x if beta == 0 else fma(float(beta), float(C[i][j]), x))
        out.append(row)
    return dict(p=p, P=P, mu=mu, nu=nu, Ai=Ai, Bi=Bi, prods=prods, Ep=Ep, Cp=Cp, out=out)


def exact_product(A, B):
    """Exact rational complex product A @ B (brute force, for tiny matrices)."""
    m, k = len(A), len(B)
    n = len(B[0]) if B else 0
    out = []
    for i in range(m):
        row = []
        for j in range(n):
            re = sum(Fraction(A[i][h].real) * Fraction(B[h][j].real)
                     - Fraction(A[i][h].imag) * Fraction(B[h][j].imag) for h in range(k))
            im = sum(Fraction(A[i][h].real) * Fraction(B[h][j].imag)
                     + Fraction(A[i][h].imag) * Fraction(B[h][j].real) for h in range(k))
            row.append((re, im))
        out.append(row)
    return out
