// CRT reconstruction, inverse scaling and alpha/beta (Algorithm 1 Steps
// V-v, V-vi and VI).
//
// For every output entry and each of the real and imaginary parts the kernel
// forms S = sum_l s_l E'_l with s_l = (P/p_l) q_l, reduces C' = mod(S, P)
// into [-P/2, P/2) and rounds C' to the nearest double (ties to even), then
// scales by 2^-(mu_i + nu_j).  The paper evaluates S as an unevaluated sum
// of two doubles and reduces it in double-double arithmetic (Section II,
// equation (5); Section IV-A); here S is accumulated exactly as 38-bit chunks
// in FP64 (s_l split into 38-bit chunks, every partial sum an integer below
// 24 * 2^38 * 2^7 < 2^53), and reduced mod P on the same chunks, which removes
// the reconstruction error altogether and makes the output bit-reproducible
// against an exact reference; the rounding works on the 256-bit integer |C'|.
#include "internal.h"

namespace ozc {
namespace {

using ConstTab = const OZC_AS_CONST NTable *;

// The reduction works on the 38-bit chunks of S held in FP64: every value it
// forms is an integer below 2^53, so every operation below is exact.
constexpr double kChunk = (double)(1ull << kChunkBits);   // 2^38
constexpr double kInvChunk = 1.0 / kChunk;                 // 2^-38, exact

// Chunks 0 .. C-2 into [0, 2^38), the carries into the top chunk (which keeps the sign).
template <int C>
__device__ __forceinline__ void normalize(double (&r)[C]) {
#pragma unroll
    for (int c = 0; c < C - 1; ++c) {
        const double f = floor(r[c] * kInvChunk);
        r[c] = fma(-f, kChunk, r[c]);
        r[c + 1] += f;
    }
}

// After normalize(): value >= 0  <=>  top chunk >= 0.  Brings R into [-P/2, P/2)
// when the quotient estimate was one off.
template <int C>
__device__ __forceinline__ void settle_range(double (&r)[C], ConstTab tab) {
    double t[C];
#pragma unroll
    for (int c = 0; c < C; ++c) t[c] = 2.0 * r[c] - tab->Pchunk[c];
    normalize<C>(t);
    if (t[C - 1] >= 0.0) {  // 2R >= P
#pragma unroll
        for (int c = 0; c < C; ++c) r[c] -= tab->Pchunk[c];
        normalize<C>(r);
        return;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) t[c] = 2.0 * r[c] + tab->Pchunk[c];
    normalize<C>(t);
    if (t[C - 1] < 0.0) {  // 2R < -P
#pragma unroll
        for (int c = 0; c < C; ++c) r[c] += tab->Pchunk[c];
        normalize<C>(r);
    }
}

// A 256-bit magnitude w (little-endian words) rounded to nearest-even as d * 2^sh.
__device__ __forceinline__ double round_w4(const uint64_t (&w)[4], int &sh) {
    if ((w[1] | w[2] | w[3]) == 0) {
        sh = 0;
        return (double)w[0];  // exact when < 2^53, otherwise one correct rounding
    }
    const int wi = w[3] ? 3 : (w[2] ? 2 : 1);
    const uint64_t top = wi == 3 ? w[3] : (wi == 2 ? w[2] : w[1]);
    const uint64_t below = wi == 3 ? w[2] : (wi == 2 ? w[1] : w[0]);
    uint64_t rest = wi == 3 ? (w[1] | w[0]) : (wi == 2 ? w[0] : 0);
    const int nb = 64 - __clzll((long long)top);  // 1..64
    uint64_t W;
    if (nb == 64) {
        W = top;
        rest |= below;
    } else {
        W = (top << (64 - nb)) | (below >> nb);
        rest |= below << (64 - nb);
    }
    W |= (rest != 0) ? 1ull : 0ull;  // sticky bit below the rounding position
    sh = 64 * (wi - 1) + nb;
    return (double)W;
}

// w - d 2^sh for the rounded value d 2^sh of w (|difference| <= half an ulp of d):
// the magnitude of the difference into r, its sign as the return value (true: negative).
__device__ __forceinline__ bool rounding_residual(const uint64_t (&w)[4], double d, int sh,
                                                  uint64_t (&r)[4]) {
    const uint64_t bits = (uint64_t)__double_as_longlong(d);
    const uint64_t M = (bits & ((1ull << 52) - 1)) | (1ull << 52);
    const int s = (int)(bits >> 52) - 1075 + sh;  // d 2^sh = M 2^s, s >= 0 when d is inexact
    uint64_t h[4] = {0, 0, 0, 0};
    const int q = s >> 6, o = s & 63;
    if (q < 4) h[q] = M << o;
    if (o && q + 1 < 4) h[q + 1] = M >> (64 - o);
    uint64_t borrow = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint64_t x = w[j], y = h[j];
        const uint64_t t = x - y;
        const uint64_t b2 = (x < y) ? 1ull : 0ull;
        r[j] = t - borrow;
        borrow = b2 | ((t < borrow) ? 1ull : 0ull);
    }
    if (!borrow) return false;
    uint64_t c = 1;  // negate the two's complement
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        r[j] = ~r[j] + c;
        c = (c && r[j] == 0) ? 1ull : 0ull;
    }
    return true;
}

// mod(S, P) rounded to nearest-even as d * 2^sh; S given as C unnormalised 38-bit
// chunks in FP64 (|r_c| < 2^50).  With low (and shl) non-null, also the rounding
// residual mod(S, P) - d 2^sh rounded to nearest-even as *low * 2^shl (0 when d is
// exact), for double-double outputs.
// The quotient q = rint(S / P) comes from the chunks' Horner sum times fl(1/P) (error
// far below 2^-20, since |S| < 2^7 N P); R = S - q P chunk by chunk (|q P_c| < 2^50,
// exact); a quotient within 2^-20 of a tie is checked exactly (settle_range).  |R| then
// goes to a 256-bit integer for the rounding.
template <int C>
__device__ __forceinline__ double reconstruct(double (&r)[C], ConstTab tab, int &sh,
                                              double *low = nullptr, int *shl = nullptr) {
    double sa = r[C - 1];
#pragma unroll
    for (int c = C - 2; c >= 0; --c) sa = fma(sa, kChunk, r[c]);
    const double x = sa * tab->inv_P;  // ~ S / P
    const double qd = rint(x);         // |q| <= 128 N + 1 < 2^12
#pragma unroll
    for (int c = 0; c < C; ++c) r[c] = fma(-qd, tab->Pchunk[c], r[c]);
    normalize<C>(r);
    if (fabs(x - qd) > 0.5 - 1.0 / 1048576.0) settle_range<C>(r, tab);

    const bool neg = r[C - 1] < 0.0;
    if (neg) {
#pragma unroll
        for (int c = 0; c < C; ++c) r[c] = -r[c];
        normalize<C>(r);
    }
    // chunk c (in [0, 2^38), the top one too since |R| < P / 2) at bit 38 c
    uint64_t w[4] = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double hi = floor(r[c] * 0x1p-32);
        const uint32_t lo32 = (uint32_t)fma(-hi, 0x1p32, r[c]);
        const uint64_t v = ((uint64_t)(uint32_t)hi << 32) | lo32;
        const int o = kChunkBits * c;
        w[o >> 6] |= v << (o & 63);
        if ((o & 63) + kChunkBits > 64) w[(o >> 6) + 1] |= v >> (64 - (o & 63));
    }
    const double d = round_w4(w, sh);
    if (low) {
        *low = 0.0;
        *shl = 0;
        const bool exact = (w[1] | w[2] | w[3]) == 0 && w[0] < (1ull << 53);
        if (!exact) {
            uint64_t rr[4];
            const bool rneg = rounding_residual(w, d, sh, rr);
            const double e = round_w4(rr, *shl);
            *low = e == 0.0 ? 0.0 : ((rneg != neg) ? -e : e);  // a zero residual is +0
        }
    }
    return neg ? -d : d;
}

__device__ __forceinline__ void alpha_beta(double cr, double ci, double ar, double ai, double br,
                                           double bi, bool beta_zero, double Cr, double Ci,
                                           double &orr, double &oi) {
    const double xr = fma(ar, cr, -(ai * ci));
    const double xi = fma(ar, ci, ai * cr);
    if (beta_zero) {
        orr = xr;
        oi = xi;
    } else {
        orr = fma(br, Cr, fma(-bi, Ci, xr));
        oi = fma(br, Ci, fma(bi, Cr, xi));
    }
}

// C elements of kind EK (ElemKind); real elements carry no imaginary part.
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));

template <int EK>
__device__ __forceinline__ void load_c(const void *C, int64_t idx, double &re, double &im) {
    if constexpr (EK == kElemC) {
        const fvec2 v = global_ptr(reinterpret_cast<const fvec2 *>(C))[idx];
        re = v.x;
        im = v.y;
    } else if constexpr (EK == kElemZ) {
        const dvec2 v = global_ptr(reinterpret_cast<const dvec2 *>(C))[idx];
        re = v.x;
        im = v.y;
    } else if constexpr (EK == kElemD) {
        re = global_ptr(reinterpret_cast<const double *>(C))[idx];
        im = 0.0;
    } else {
        re = global_ptr(reinterpret_cast<const float *>(C))[idx];
        im = 0.0;
    }
}

template <int EK>
__device__ __forceinline__ void store_c(void *C, int64_t idx, double re, double im) {
    if constexpr (EK == kElemC) global_ptr(reinterpret_cast<fvec2 *>(C))[idx] = fvec2{(float)re, (float)im};
    else if constexpr (EK == kElemZ) global_ptr(reinterpret_cast<dvec2 *>(C))[idx] = dvec2{re, im};
    else if constexpr (EK == kElemD) global_ptr(reinterpret_cast<double *>(C))[idx] = re;
    else global_ptr(reinterpret_cast<float *>(C))[idx] = (float)re;
}

// One thread: 4 consecutive rows i of one column j; block bx covers threads
// 256 bx ... 256 bx + 255 of the ceil(m / 4) x n grid (padding rows get no thread).
// Real outputs (EK real) reconstruct the one E' plane of each modulus; alpha and beta
// are real then (imaginary parts zero), so the fused multiply-add order below reduces
// to x = alpha c, out = fma(beta, C, x).
template <int C, int EK, bool DD = false>
__device__ __forceinline__ void crt_output_body(const CrtArgs &a, int64_t bx) {
    constexpr bool REAL = elem_real(EK);
    constexpr int EPL = REAL ? 1 : 2;  // E' planes per modulus
    const int64_t m4 = (a.m + 3) >> 2;
    const int64_t t = bx * 256 + threadIdx.x;
    const int64_t i4 = t % m4, j = t / m4;
    const int64_t ib = i4 * 4;
    if (j >= a.n || ib >= a.m) return;

    const int64_t planeC = a.n_pad * a.m_pad;
    // S = sum_l s_l E'_l in 38-bit chunks: |partial sums| < 24 2^38 2^7 < 2^50, every
    // fused multiply-add exact
    double accR[4][C], accI[4][C];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < C; ++c) accR[u][c] = accI[u][c] = 0.0;

    ConstTab tab = const_ptr(a.tab);
    const OZC_AS_GLOBAL int8_t *E = global_ptr(a.eprime) + j * a.m_pad + ib;
#pragma unroll 4
    for (int l = 0; l < a.nmod; ++l) {
        const uint32_t wr = *reinterpret_cast<const OZC_AS_GLOBAL uint32_t *>(E + (int64_t)(EPL * l) * planeC);
        const uint32_t wi =
            REAL ? 0u : *reinterpret_cast<const OZC_AS_GLOBAL uint32_t *>(E + (int64_t)(EPL * l + 1) * planeC);
        double er[4], ei[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            er[u] = (double)(int)(int8_t)(wr >> (8 * u));
            ei[u] = (double)(int)(int8_t)(wi >> (8 * u));
        }
        const OZC_AS_CONST double *sc = tab->mod[l].schunk;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const double s = sc[c];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                accR[u][c] = fma(s, er[u], accR[u][c]);
                if constexpr (!REAL) accI[u][c] = fma(s, ei[u], accI[u][c]);
            }
        }
    }

    const int nuj = global_ptr(a.nu)[j];
    const bool beta_zero = a.beta_r == 0.0 && a.beta_i == 0.0;
    // the row exponents before any store of C, so that no load waits behind one
    int mus[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) mus[u] = ib + u < a.m ? global_ptr(a.mu)[ib + u] : 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t i = ib + u;
        if (i >= a.m) continue;
        const int mui = mus[u];
        double cr, ci;
        double lr = 0.0, li = 0.0;  // double-double outputs: the low parts
        if (mui == kExpNonfinite || nuj == kExpNonfinite) {
            cr = ci = __builtin_nan("");
            lr = li = cr;
        } else if (mui == kExpZero || nuj == kExpZero) {
            cr = ci = 0.0;
        } else if constexpr (DD) {
            int shr, shi, slr, sli;
            double er, ei;
            const double dr = reconstruct<C>(accR[u], tab, shr, &er, &slr);
            const double di = reconstruct<C>(accI[u], tab, shi, &ei, &sli);
            cr = ldexp(dr, shr - (mui + nuj));
            ci = ldexp(di, shi - (mui + nuj));
            lr = ldexp(er, slr - (mui + nuj));
            li = ldexp(ei, sli - (mui + nuj));
        } else {
            int shr, shi = 0;
            const double dr = reconstruct<C>(accR[u], tab, shr);
            const double di = REAL ? 0.0 : reconstruct<C>(accI[u], tab, shi);
            cr = ldexp(dr, shr - (mui + nuj));
            ci = REAL ? 0.0 : ldexp(di, shi - (mui + nuj));
        }
        const int64_t idx = j * a.ldc + i;
        if constexpr (DD) {  // alpha = 1, beta = 0: the two parts as they are
            global_ptr(reinterpret_cast<dvec2 *>(a.C))[idx] = dvec2{cr, ci};
            global_ptr(reinterpret_cast<dvec2 *>(a.C_lo))[idx] = dvec2{lr, li};
            continue;
        }
        double Cr = 0.0, Ci = 0.0;
        if (!beta_zero) load_c<EK>(a.C, idx, Cr, Ci);
        double orr, oi;
        alpha_beta(cr, ci, a.alpha_r, a.alpha_i, a.beta_r, a.beta_i, beta_zero, Cr, Ci, orr, oi);
        store_c<EK>(a.C, idx, orr, oi);
    }
}

template <int C, int EK>
__global__ __launch_bounds__(256) void crt_output_kernel(CrtArgs a) {
    crt_output_body<C, EK>(a, blockIdx.x);
}

template <int C>
__global__ __launch_bounds__(256) void crt_dd_kernel(CrtArgs a) {
    crt_output_body<C, kElemZ, true>(a, blockIdx.x);
}

template <int C, bool SINGLE>
__global__ __launch_bounds__(256) void batch_crt_kernel(const BatchCrt *probs, int nprob) {
    const int64_t b = blockIdx.x;
    int lo = 0, hi = nprob - 1;  // last problem whose first block is <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (probs[mid].blk0 <= b) lo = mid;
        else hi = mid - 1;
    }
    // The problem's arguments are copied out of the list first: read through a reference
    // into global memory, every field would be loaded again after each store of C (the
    // compiler cannot rule out that the stores overwrite the list).
    const CrtArgs a = probs[lo].a;
    crt_output_body<C, SINGLE>(a, b - probs[lo].blk0);
}

template <int C>
hipError_t launch_batch_C(const BatchCrt *probs, int nprob, int64_t blocks, bool single, hipStream_t s) {
    dim3 grid((unsigned)blocks);
    if (single) hipLaunchKernelGGL((batch_crt_kernel<C, true>), grid, dim3(256), 0, s, probs, nprob);
    else hipLaunchKernelGGL((batch_crt_kernel<C, false>), grid, dim3(256), 0, s, probs, nprob);
    return hipGetLastError();
}

// C := alpha * 0 + beta * C (alpha == 0 or k == 0), with the same operation order.
template <int EK>
__global__ void scale_c_kernel(void *C, int64_t m, int64_t n, int64_t ldc, double ar, double ai,
                               double br, double bi) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * n) return;
    const int64_t i = t % m, j = t / m;
    const bool beta_zero = br == 0.0 && bi == 0.0;
    double Cr = 0.0, Ci = 0.0;
    if (!beta_zero) load_c<EK>(C, j * ldc + i, Cr, Ci);
    double orr, oi;
    alpha_beta(0.0, 0.0, ar, ai, br, bi, beta_zero, Cr, Ci, orr, oi);
    store_c<EK>(C, j * ldc + i, orr, oi);
}

template <int C>
hipError_t launch_C(const CrtArgs &a, hipStream_t s) {
    const int64_t threads = ((a.m + 3) / 4) * a.n;
    dim3 grid((unsigned)((threads + 255) / 256));
    if (a.C_lo) {
        if (a.ek != kElemZ) return hipErrorInvalidValue;
        hipLaunchKernelGGL((crt_dd_kernel<C>), grid, dim3(256), 0, s, a);
        return hipGetLastError();
    }
    switch (a.ek) {
        case kElemZ: hipLaunchKernelGGL((crt_output_kernel<C, kElemZ>), grid, dim3(256), 0, s, a); break;
        case kElemC: hipLaunchKernelGGL((crt_output_kernel<C, kElemC>), grid, dim3(256), 0, s, a); break;
        case kElemD: hipLaunchKernelGGL((crt_output_kernel<C, kElemD>), grid, dim3(256), 0, s, a); break;
        case kElemS: hipLaunchKernelGGL((crt_output_kernel<C, kElemS>), grid, dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_crt_output(const CrtArgs &a, hipStream_t s) {
    if (a.m <= 0 || a.n <= 0) return hipSuccess;
    if (a.m_pad % 4) return hipErrorInvalidValue;
    switch (a.nchunks) {
        case 1: return launch_C<1>(a, s);
        case 2: return launch_C<2>(a, s);
        case 3: return launch_C<3>(a, s);
        case 4: return launch_C<4>(a, s);
        case 5: return launch_C<5>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_scale_c(void *C, int64_t m, int64_t n, int64_t ldc, int ek, double ar,
                          double ai, double br, double bi, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid((unsigned)((m * n + 255) / 256));
    switch (ek) {
        case kElemZ: hipLaunchKernelGGL(scale_c_kernel<kElemZ>, grid, dim3(256), 0, s, C, m, n, ldc, ar, ai, br, bi); break;
        case kElemC: hipLaunchKernelGGL(scale_c_kernel<kElemC>, grid, dim3(256), 0, s, C, m, n, ldc, ar, ai, br, bi); break;
        case kElemD: hipLaunchKernelGGL(scale_c_kernel<kElemD>, grid, dim3(256), 0, s, C, m, n, ldc, ar, ai, br, bi); break;
        case kElemS: hipLaunchKernelGGL(scale_c_kernel<kElemS>, grid, dim3(256), 0, s, C, m, n, ldc, ar, ai, br, bi); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int64_t batch_crt_blocks(int64_t m, int64_t n) { return (((m + 3) / 4) * n + 255) / 256; }

hipError_t launch_batch_crt(const BatchCrt *probs, int nprob, int64_t blocks, int nchunks,
                            bool single, hipStream_t s) {
    if (blocks <= 0 || nprob <= 0) return hipSuccess;
    switch (nchunks) {
        case 1: return launch_batch_C<1>(probs, nprob, blocks, single, s);
        case 2: return launch_batch_C<2>(probs, nprob, blocks, single, s);
        case 3: return launch_batch_C<3>(probs, nprob, blocks, single, s);
        case 4: return launch_batch_C<4>(probs, nprob, blocks, single, s);
        case 5: return launch_batch_C<5>(probs, nprob, blocks, single, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ozc
