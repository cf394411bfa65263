/*
 * CPU oracle of the complex Ozaki-II scheme (arXiv 2512.08321), in exact
 * integer arithmetic.  TEST INFRASTRUCTURE ONLY: it is called by the tests,
 * the smoke check and the CPU baseline of the benchmark, never by the
 * product path, and it shares no code with the GPU library.
 *
 * Every matrix handled here is a set of "rows" of k complex numbers, stored
 * as separate real and imaginary row-major arrays: the rows of op(A) and the
 * columns of op(B) (the rows of A-hat and the columns of B-hat of equation
 * (6) share one scaling exponent each, Section III-B).
 *
 * Steps (Algorithm 1; Section III):
 *   orc_row_exponents   e = floor(log2 max|x|) per row, zero / non-finite flags
 *   orc_fast_sigma      fast mode: sum of ceil(|x| 2^(F-e))^2 (Section III-B)
 *   orc_ceil7           accurate mode: ceil(|x| 2^(5-e)) in [0, 64]
 *   orc_bound_max       accurate mode: Cbar_I, Cbar_R = Cbar_I + (AR-AI)(BR-BI),
 *                       row and column maxima
 *   orc_residues        a' = trunc(x 2^mu) (Step IV), symmetric residues of
 *                       a'_R, a'_I and of a'_R + a'_I (Step V-i/ii, Sec. III-A)
 *   orc_products        per-modulus products, eq. (10) Karatsuba or eq. (7),
 *                       and the reduced E'_R, E'_I (Step V-iii/iv)
 *   orc_crt_output      S = sum_l s_l E'_l, C' = mod(S, P) exactly (Step V-v/vi),
 *                       C = ldexp(RNE(C'), -(mu+nu)) (Step VI), alpha/beta
 *   orc_real_products,  the same two steps for real matrices (Algorithm 1 as
 *   orc_real_crt_output stated): one product per modulus, one E' plane
 *   orc_dd_gemm         double-double complex product (the accuracy yardstick
 *                       of Section IV-A)
 * Thresholds for the exponent rules are evaluated by the Python layer with
 * exact big integers.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_FLAG_OK 0
#define ORC_FLAG_ZERO 1
#define ORC_FLAG_NONFINITE 2

/* ------------------------------------------------------------ exponents */

/* Exact decomposition |x| = M * 2^E with integer M < 2^53 (x finite, != 0). */
static void decompose(double x, uint64_t *M, int *E) {
    int ex;
    double f = frexp(fabs(x), &ex);          /* |x| = f 2^ex, f in [0.5, 1) */
    *M = (uint64_t)ldexp(f, 53);             /* exact: f has <= 53 significant bits */
    *E = ex - 53;
}

int orc_row_exponents(const double *re, const double *im, int64_t rows, int64_t len,
                      int32_t *e, uint8_t *flags) {
    int any_nonfinite = 0;
#pragma omp parallel for reduction(| : any_nonfinite)
    for (int64_t r = 0; r < rows; ++r) {
        int best = INT32_MIN, nonfinite = 0;
        for (int64_t h = 0; h < len; ++h) {
            double v[2] = {re[r * len + h], im[r * len + h]};
            for (int c = 0; c < 2; ++c) {
                if (!isfinite(v[c])) { nonfinite = 1; continue; }
                if (v[c] != 0.0) {
                    int ex = ilogb(v[c]);
                    if (ex > best) best = ex;
                }
            }
        }
        if (nonfinite) { flags[r] = ORC_FLAG_NONFINITE; e[r] = 0; any_nonfinite = 1; }
        else if (best == INT32_MIN) { flags[r] = ORC_FLAG_ZERO; e[r] = 0; }
        else { flags[r] = ORC_FLAG_OK; e[r] = best; }
    }
    return any_nonfinite;
}

/* ceil(|x| * 2^sh) for finite x, as an exact integer (must fit in 64 bits). */
static uint64_t ceil_scaled(double x, int sh) {
    if (x == 0.0) return 0;
    uint64_t M; int E;
    decompose(x, &M, &E);
    int s = E + sh;
    if (s >= 0) return M << s;
    if (-s >= 64) return 1;
    uint64_t q = M >> (-s);
    return (q << (-s)) == M ? q : q + 1;
}

void orc_fast_sigma(const double *re, const double *im, int64_t rows, int64_t len, int F,
                    const int32_t *e, const uint8_t *flags, uint64_t *sigma) {
#pragma omp parallel for
    for (int64_t r = 0; r < rows; ++r) {
        uint64_t acc = 0;
        if (flags[r] == ORC_FLAG_OK) {
            for (int64_t h = 0; h < len; ++h) {
                uint64_t a = ceil_scaled(re[r * len + h], F - e[r]);
                uint64_t b = ceil_scaled(im[r * len + h], F - e[r]);
                acc += a * a + b * b;
            }
        }
        sigma[r] = acc;
    }
}

void orc_ceil7(const double *re, const double *im, int64_t rows, int64_t len,
               const int32_t *e, const uint8_t *flags, int8_t *barR, int8_t *barI) {
#pragma omp parallel for
    for (int64_t r = 0; r < rows; ++r) {
        for (int64_t h = 0; h < len; ++h) {
            int ok = flags[r] == ORC_FLAG_OK;
            barR[r * len + h] = ok ? (int8_t)ceil_scaled(re[r * len + h], 5 - e[r]) : 0;
            barI[r * len + h] = ok ? (int8_t)ceil_scaled(im[r * len + h], 5 - e[r]) : 0;
        }
    }
}

/* Accurate-mode bound product: Cbar_I = AI BR + AR BI, Cbar_R = Cbar_I + (AR-AI)(BR-BI).
 * X[i] = max_j max(Cbar_R, Cbar_I)_ij, Y[j] = max_i (...).  B is given as n rows of len. */
void orc_bound_max(const int8_t *AR, const int8_t *AI, int64_t m, const int8_t *BR,
                   const int8_t *BI, int64_t n, int64_t len, int64_t *X, int64_t *Y) {
    for (int64_t j = 0; j < n; ++j) Y[j] = 0;
#pragma omp parallel
    {
        int64_t *Yl = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
#pragma omp for
        for (int64_t i = 0; i < m; ++i) {
            int64_t xi = 0;
            const int8_t *ar = AR + i * len, *ai = AI + i * len;
            for (int64_t j = 0; j < n; ++j) {
                const int8_t *br = BR + j * len, *bi = BI + j * len;
                int64_t ci = 0, cd = 0;
                for (int64_t h = 0; h < len; ++h) {
                    ci += (int64_t)ai[h] * br[h] + (int64_t)ar[h] * bi[h];
                    cd += (int64_t)(ar[h] - ai[h]) * (br[h] - bi[h]);
                }
                int64_t cr = ci + cd;
                int64_t v = cr > ci ? cr : ci;
                if (v > xi) xi = v;
                if (v > Yl[j]) Yl[j] = v;
            }
            X[i] = xi;
        }
#pragma omp critical
        for (int64_t j = 0; j < n; ++j)
            if (Yl[j] > Y[j]) Y[j] = Yl[j];
        free(Yl);
    }
}

/* ------------------------------------------------------------ residues */

/* smod(x, p) in [-floor(p/2), ceil(p/2)-1] for a 128-bit signed x. */
static int smod128(__int128 x, int p) {
    __int128 r = x % p;          /* sign follows x */
    if (r < 0) r += p;           /* [0, p) */
    if (2 * r >= p) r -= p;      /* ties (p even) go to -p/2 */
    return (int)r;
}

static int smod64(int64_t x, int p) {
    int64_t r = x % p;
    if (r < 0) r += p;
    if (2 * r >= p) r -= p;
    return (int)r;
}

/* trunc(x * 2^mu) as a 128-bit integer; *overflow set if |result| >= 2^126. */
static __int128 trunc_scaled(double x, int mu, int *overflow) {
    if (x == 0.0) return 0;
    uint64_t M; int E;
    decompose(x, &M, &E);
    int s = E + mu;
    unsigned __int128 mag;
    if (s >= 0) {
        if (s > 126 - 53) { *overflow = 1; return 0; }
        mag = (unsigned __int128)M << s;
    } else {
        mag = (-s >= 64) ? 0 : (M >> (-s));
    }
    return x < 0 ? -(__int128)mag : (__int128)mag;
}

/* out layout: [l][plane][rows][len], planes R, I, S (S = smod(R + I)). */
int orc_residues(const double *re, const double *im, int64_t rows, int64_t len,
                 const int32_t *mu, const uint8_t *valid, int nmod, const int32_t *p,
                 int8_t *out) {
    int overflow = 0;
    const int64_t plane = rows * len;
#pragma omp parallel for reduction(| : overflow)
    for (int64_t r = 0; r < rows; ++r) {
        for (int64_t h = 0; h < len; ++h) {
            __int128 aR = 0, aI = 0;
            int of = 0;
            if (valid[r]) {
                aR = trunc_scaled(re[r * len + h], mu[r], &of);
                aI = trunc_scaled(im[r * len + h], mu[r], &of);
            }
            overflow |= of;
            for (int l = 0; l < nmod; ++l) {
                int rR = smod128(aR, p[l]);
                int rI = smod128(aI, p[l]);
                int rS = smod64((int64_t)rR + rI, p[l]);
                out[((int64_t)l * 3 + 0) * plane + r * len + h] = (int8_t)rR;
                out[((int64_t)l * 3 + 1) * plane + r * len + h] = (int8_t)rI;
                out[((int64_t)l * 3 + 2) * plane + r * len + h] = (int8_t)rS;
            }
        }
    }
    return overflow;
}

/* ------------------------------------------------------------ products */

static int64_t dot8(const int8_t *a, const int8_t *b, int64_t len) {
    int64_t acc = 0;
    for (int64_t h = 0; h < len; ++h) acc += (int64_t)a[h] * b[h];
    return acc;
}

/* resA [l][3][m][len], resB [l][3][n][len] -> Ep [l][2][m][n] (int8).
 * algo 0: Karatsuba, eq. (10): D = R*R, E = I*I, F = S*S; E'_R = mod(D-E), E'_I = mod(F-D-E).
 * algo 1: expanded product, eq. (7): E'_R = mod(RR - II), E'_I = mod(RI + IR).
 * raw (optional) [l][nprod][m][n]: the integer products (D,E,F) or (RR,II,RI,IR). */
void orc_products(const int8_t *resA, int64_t m, const int8_t *resB, int64_t n, int64_t len,
                  int nmod, const int32_t *p, int algo, int8_t *Ep, int64_t *raw) {
    const int64_t pa = m * len, pb = n * len, pc = m * n;
    const int nprod = algo == 0 ? 3 : 4;
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int l = 0; l < nmod; ++l) {
        for (int64_t i = 0; i < m; ++i) {
            const int8_t *aR = resA + ((int64_t)l * 3 + 0) * pa + i * len;
            const int8_t *aI = resA + ((int64_t)l * 3 + 1) * pa + i * len;
            const int8_t *aS = resA + ((int64_t)l * 3 + 2) * pa + i * len;
            for (int64_t j = 0; j < n; ++j) {
                const int8_t *bR = resB + ((int64_t)l * 3 + 0) * pb + j * len;
                const int8_t *bI = resB + ((int64_t)l * 3 + 1) * pb + j * len;
                const int8_t *bS = resB + ((int64_t)l * 3 + 2) * pb + j * len;
                int64_t v[4];
                int eR, eI;
                if (algo == 0) {
                    v[0] = dot8(aR, bR, len);
                    v[1] = dot8(aI, bI, len);
                    v[2] = dot8(aS, bS, len);
                    eR = smod64(v[0] - v[1], p[l]);
                    eI = smod64(v[2] - v[0] - v[1], p[l]);
                } else {
                    v[0] = dot8(aR, bR, len);
                    v[1] = dot8(aI, bI, len);
                    v[2] = dot8(aR, bI, len);
                    v[3] = dot8(aI, bR, len);
                    eR = smod64(v[0] - v[1], p[l]);
                    eI = smod64(v[2] + v[3], p[l]);
                }
                Ep[((int64_t)l * 2 + 0) * pc + i * n + j] = (int8_t)eR;
                Ep[((int64_t)l * 2 + 1) * pc + i * n + j] = (int8_t)eI;
                if (raw)
                    for (int t = 0; t < nprod; ++t)
                        raw[((int64_t)l * nprod + t) * pc + i * n + j] = v[t];
            }
        }
    }
}

/* Real products (Algorithm 1 as stated for real A, B): resA [l][m][len] and resB [l][n][len]
 * (the residues of A'_l and of the columns of B'_l) -> Ep [l][m][n] = mod(A'_l B'_l, p_l)
 * (Step V-iii/iv); raw (optional) [l][m][n]: the integer products D'_l. */
void orc_real_products(const int8_t *resA, int64_t m, const int8_t *resB, int64_t n, int64_t len,
                       int nmod, const int32_t *p, int8_t *Ep, int64_t *raw) {
    const int64_t pa = m * len, pb = n * len, pc = m * n;
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int l = 0; l < nmod; ++l) {
        for (int64_t i = 0; i < m; ++i) {
            const int8_t *a = resA + (int64_t)l * pa + i * len;
            for (int64_t j = 0; j < n; ++j) {
                const int64_t d = dot8(a, resB + (int64_t)l * pb + j * len, len);
                Ep[(int64_t)l * pc + i * n + j] = (int8_t)smod64(d, p[l]);
                if (raw) raw[(int64_t)l * pc + i * n + j] = d;
            }
        }
    }
}

/* ------------------------------------------------------------ CRT (256-bit) */

typedef struct { uint64_t w[4]; } u256; /* two's complement when used as signed */

static void u256_add(u256 *a, const u256 *b) {
    unsigned __int128 c = 0;
    for (int j = 0; j < 4; ++j) { c += (unsigned __int128)a->w[j] + b->w[j]; a->w[j] = (uint64_t)c; c >>= 64; }
}
static void u256_neg(u256 *a) {
    for (int j = 0; j < 4; ++j) a->w[j] = ~a->w[j];
    u256 one = {{1, 0, 0, 0}};
    u256_add(a, &one);
}
static void u256_sub(u256 *a, const u256 *b) { u256 t = *b; u256_neg(&t); u256_add(a, &t); }
static int u256_isneg(const u256 *a) { return (int)(a->w[3] >> 63); }
static u256 u256_mul_small(const u256 *a, uint64_t s) {
    u256 r; unsigned __int128 c = 0;
    for (int j = 0; j < 4; ++j) { c += (unsigned __int128)a->w[j] * s; r.w[j] = (uint64_t)c; c >>= 64; }
    return r;
}
static int u256_cmp(const u256 *a, const u256 *b) { /* unsigned compare */
    for (int j = 3; j >= 0; --j) if (a->w[j] != b->w[j]) return a->w[j] < b->w[j] ? -1 : 1;
    return 0;
}
static long double u256_to_ld_signed(const u256 *a) {
    u256 t = *a; int neg = u256_isneg(&t);
    if (neg) u256_neg(&t);
    long double v = 0.0L;
    for (int j = 3; j >= 0; --j) v = v * 18446744073709551616.0L + (long double)t.w[j];
    return neg ? -v : v;
}
static int u256_bitlen(const u256 *a) {
    for (int j = 3; j >= 0; --j) if (a->w[j]) return 64 * j + 64 - __builtin_clzll(a->w[j]);
    return 0;
}
static int u256_bit(const u256 *a, int b) { return (int)((a->w[b >> 6] >> (b & 63)) & 1u); }

/* Round a signed 256-bit integer to the nearest double, ties to even. */
static double u256_to_double_rne(const u256 *a) {
    u256 t = *a; int neg = u256_isneg(&t);
    if (neg) u256_neg(&t);
    int b = u256_bitlen(&t);
    double v;
    if (b <= 53) {
        v = (double)t.w[0];
    } else {
        int sh = b - 53;
        uint64_t mant = 0;
        for (int q = 0; q < 53; ++q) mant |= (uint64_t)u256_bit(&t, sh + q) << q;
        int round_bit = u256_bit(&t, sh - 1);
        int sticky = 0;
        for (int q = 0; q < sh - 1; ++q) sticky |= u256_bit(&t, q);
        if (round_bit && (sticky || (mant & 1u))) mant += 1; /* mant may reach 2^53: exact */
        v = ldexp((double)mant, sh);
    }
    return neg ? -v : v;
}

/* The integer value of an integer-valued double (|d| < 2^255), as a signed 256-bit number. */
static u256 u256_from_double(double d) {
    u256 r = {{0, 0, 0, 0}};
    if (d == 0.0) return r;
    int e;
    double f = frexp(fabs(d), &e);            /* |d| = f 2^e, f in [0.5, 1) */
    uint64_t M = (uint64_t)ldexp(f, 53);      /* |d| = M 2^(e - 53) */
    int sh = e - 53;
    if (sh < 0) {
        r.w[0] = M >> (-sh);                  /* exact: d is an integer */
    } else {
        int q = sh / 64, o = sh % 64;
        if (q < 4) r.w[q] = M << o;
        if (o && q + 1 < 4) r.w[q + 1] = M >> (64 - o);
    }
    if (d < 0) u256_neg(&r);
    return r;
}

/* C' = mod(S, P) with S = sum_l s_l E'_l; s_l and P as 4 x 64-bit little-endian words. */
static u256 crt_reduce(const int8_t *const *ep, int nmod, const u256 *s, const u256 *P,
                       long double Pld) {
    u256 acc = {{0, 0, 0, 0}};
    for (int l = 0; l < nmod; ++l) {
        int e = *ep[l];
        if (e == 0) continue;
        u256 prod = u256_mul_small(&s[l], (uint64_t)(e < 0 ? -e : e));
        if (e > 0) u256_add(&acc, &prod); else u256_sub(&acc, &prod);
    }
    long double t = nearbyintl(u256_to_ld_signed(&acc) / Pld);
    int64_t ti = (int64_t)t;
    u256 tp = u256_mul_small(P, (uint64_t)(ti < 0 ? -ti : ti));
    if (ti > 0) u256_sub(&acc, &tp); else if (ti < 0) u256_add(&acc, &tp);
    /* symmetric range [-P/2, P/2): 2r < P and 2r >= -P */
    for (;;) {
        u256 twice = acc; u256_add(&twice, &acc);
        if (!u256_isneg(&twice) && u256_cmp(&twice, P) >= 0) { u256_sub(&acc, P); continue; }
        if (u256_isneg(&twice)) {
            u256 mag = twice; u256_neg(&mag);
            if (u256_cmp(&mag, P) > 0) { u256_add(&acc, P); continue; }
        }
        break;
    }
    return acc;
}

/* Ep [l][2][m][n]; mu/nu with valid flags (0 = zero row/col, 1 = ok, 2 = non-finite).
 * alpha, beta: 2 doubles each; Cin: m x n complex (interleaved re,im, row-major) or NULL.
 * out: m x n complex interleaved.  Cp_out (optional): m*n*2 doubles = RNE(C'). */
void orc_crt_output(const int8_t *Ep, int64_t m, int64_t n, int nmod, const uint64_t *s_words,
                    const uint64_t *P_words, const int32_t *mu, const uint8_t *rowflag,
                    const int32_t *nu, const uint8_t *colflag, const double *alpha,
                    const double *beta, const double *Cin, double *out, double *Cp_out,
                    double *lo_out) {
    u256 s[32], P;
    for (int l = 0; l < nmod; ++l) memcpy(s[l].w, s_words + 4 * l, 32);
    memcpy(P.w, P_words, 32);
    long double Pld = u256_to_ld_signed(&P);
    const int64_t pc = m * n;
    const int beta_zero = beta[0] == 0.0 && beta[1] == 0.0;
    const int alpha_zero = alpha[0] == 0.0 && alpha[1] == 0.0;
#pragma omp parallel for
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double cr = 0.0, ci = 0.0;
            if (lo_out) { lo_out[2 * (i * n + j)] = 0.0; lo_out[2 * (i * n + j) + 1] = 0.0; }
            if (rowflag[i] == 2 || colflag[j] == 2) {
                cr = NAN; ci = NAN;
                if (lo_out) { lo_out[2 * (i * n + j)] = NAN; lo_out[2 * (i * n + j) + 1] = NAN; }
            } else if (rowflag[i] == 1 && colflag[j] == 1) {
                const int8_t *pr[32], *pi[32];
                for (int l = 0; l < nmod; ++l) {
                    pr[l] = Ep + ((int64_t)l * 2 + 0) * pc + i * n + j;
                    pi[l] = Ep + ((int64_t)l * 2 + 1) * pc + i * n + j;
                }
                u256 R = crt_reduce(pr, nmod, s, &P, Pld);
                u256 I = crt_reduce(pi, nmod, s, &P, Pld);
                double dR = u256_to_double_rne(&R), dI = u256_to_double_rne(&I);
                if (Cp_out) { Cp_out[2 * (i * n + j)] = dR; Cp_out[2 * (i * n + j) + 1] = dI; }
                int sh = -(mu[i] + nu[j]);
                if (lo_out) { /* the rounding residual C' - RNE(C'), rounded, scaled */
                    u256 hR = u256_from_double(dR), hI = u256_from_double(dI);
                    u256 rR = R, rI = I;
                    u256_sub(&rR, &hR);
                    u256_sub(&rI, &hI);
                    lo_out[2 * (i * n + j)] = ldexp(u256_to_double_rne(&rR), sh);
                    lo_out[2 * (i * n + j) + 1] = ldexp(u256_to_double_rne(&rI), sh);
                }
                cr = ldexp(dR, sh);
                ci = ldexp(dI, sh);
            }
            double orr, oi;
            if (alpha_zero) { cr = 0.0; ci = 0.0; }
            double xr = fma(alpha[0], cr, -(alpha[1] * ci));
            double xi = fma(alpha[0], ci, alpha[1] * cr);
            if (beta_zero) {
                orr = xr; oi = xi;
            } else {
                double Cr = Cin[2 * (i * n + j)], Ci = Cin[2 * (i * n + j) + 1];
                orr = fma(beta[0], Cr, fma(-beta[1], Ci, xr));
                oi = fma(beta[0], Ci, fma(beta[1], Cr, xi));
            }
            out[2 * (i * n + j)] = orr;
            out[2 * (i * n + j) + 1] = oi;
        }
    }
}

/* Real output (Step V-v/vi, VI): Ep [l][m][n]; x = alpha * ldexp(RNE(C'), -(mu+nu)) (one
 * rounding), out = x if beta == 0, else fma(beta, Cin, x).  Cin: m x n row-major or NULL;
 * out: m x n row-major; Cp_out (optional): RNE(C'). */
void orc_real_crt_output(const int8_t *Ep, int64_t m, int64_t n, int nmod, const uint64_t *s_words,
                         const uint64_t *P_words, const int32_t *mu, const uint8_t *rowflag,
                         const int32_t *nu, const uint8_t *colflag, double alpha, double beta,
                         const double *Cin, double *out, double *Cp_out) {
    u256 s[32], P;
    for (int l = 0; l < nmod; ++l) memcpy(s[l].w, s_words + 4 * l, 32);
    memcpy(P.w, P_words, 32);
    long double Pld = u256_to_ld_signed(&P);
    const int64_t pc = m * n;
#pragma omp parallel for
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double c = 0.0;
            if (rowflag[i] == 2 || colflag[j] == 2) {
                c = NAN;
            } else if (rowflag[i] == 1 && colflag[j] == 1) {
                const int8_t *pl[32];
                for (int l = 0; l < nmod; ++l) pl[l] = Ep + (int64_t)l * pc + i * n + j;
                u256 R = crt_reduce(pl, nmod, s, &P, Pld);
                double d = u256_to_double_rne(&R);
                if (Cp_out) Cp_out[i * n + j] = d;
                c = ldexp(d, -(mu[i] + nu[j]));
            }
            if (alpha == 0.0) c = 0.0;
            double x = alpha * c;
            out[i * n + j] = beta == 0.0 ? x : fma(beta, Cin[i * n + j], x);
        }
    }
}

/* ------------------------------------------------------------ double-double GEMM */

typedef struct { double hi, lo; } dd;

static inline dd two_sum(double a, double b) {
    double s = a + b, bb = s - a;
    dd r = {s, (a - (s - bb)) + (b - bb)};
    return r;
}
static inline dd fast_two_sum(double a, double b) {
    double s = a + b;
    dd r = {s, b - (s - a)};
    return r;
}
static inline dd dd_add(dd x, dd y) { /* accurate double-word addition */
    dd s = two_sum(x.hi, y.hi), t = two_sum(x.lo, y.lo);
    double c = s.lo + t.hi;
    dd v = fast_two_sum(s.hi, c);
    double w = t.lo + v.lo;
    return fast_two_sum(v.hi, w);
}
static inline dd two_prod(double a, double b) {
    double p = a * b;
    dd r = {p, fma(a, b, -p)};
    return r;
}

/* A: m rows of len (re/im), B: n rows of len (columns of op(B)).
 * out_hi/out_lo: m x n complex interleaved (re, im). */
void orc_dd_gemm(const double *Are, const double *Aim, int64_t m, const double *Bre,
                 const double *Bim, int64_t n, int64_t len, double *out_hi, double *out_lo) {
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            dd sr = {0, 0}, si = {0, 0};
            const double *ar = Are + i * len, *ai = Aim + i * len;
            const double *br = Bre + j * len, *bi = Bim + j * len;
            for (int64_t h = 0; h < len; ++h) {
                dd p1 = two_prod(ar[h], br[h]), p2 = two_prod(-ai[h], bi[h]);
                dd p3 = two_prod(ar[h], bi[h]), p4 = two_prod(ai[h], br[h]);
                sr = dd_add(sr, p1); sr = dd_add(sr, p2);
                si = dd_add(si, p3); si = dd_add(si, p4);
            }
            out_hi[2 * (i * n + j)] = sr.hi; out_lo[2 * (i * n + j)] = sr.lo;
            out_hi[2 * (i * n + j) + 1] = si.hi; out_lo[2 * (i * n + j) + 1] = si.lo;
        }
    }
}

/* |A||B| with complex moduli: m x n real, in plain double (an upper-bound yardstick). */
void orc_abs_product(const double *Are, const double *Aim, int64_t m, const double *Bre,
                     const double *Bim, int64_t n, int64_t len, double *out) {
#pragma omp parallel for collapse(2)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t h = 0; h < len; ++h)
                acc += hypot(Are[i * len + h], Aim[i * len + h]) *
                       hypot(Bre[j * len + h], Bim[j * len + h]);
            out[i * n + j] = acc;
        }
}

/* Threads of the OpenMP loops above (for timing the oracle on a stated core count). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
