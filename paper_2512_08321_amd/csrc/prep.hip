// Scaling and residue split: the two HBM-bound passes over A and B that
// precede the INT8 products (Section III-B; Algorithm 1 Steps III, IV, V-i/ii).
//
// Operands are handled as "rows": the rows of op(A) and the columns of op(B),
// each a vector of k complex numbers (rows i and i+m of A-hat share one
// exponent, Section III-B).  Two memory orders occur: rows whose k elements
// are contiguous (contig_h) and rows that are contiguous with each other
// (consecutive rows adjacent, stride_r == 1).  Every kernel has a variant for
// each so that global loads stay coalesced.
#include "internal.h"

namespace ozc {
namespace {

constexpr uint64_t kAbsMask = 0x7fffffffffffffffull;
constexpr uint64_t kInfBits = 0x7ff0000000000000ull;

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));

// One element of kind EK (ElemKind) at index idx; real elements have im = 0.
template <int EK>
__device__ __forceinline__ void load_elem(const void *base, int64_t idx, double &re, double &im) {
    if constexpr (EK == kElemC) {
        const fvec2 v = global_ptr(reinterpret_cast<const fvec2 *>(base))[idx];
        re = (double)v.x;
        im = (double)v.y;
    } else if constexpr (EK == kElemZ) {
        const dvec2 v = global_ptr(reinterpret_cast<const dvec2 *>(base))[idx];
        re = v.x;
        im = v.y;
    } else if constexpr (EK == kElemD) {
        re = global_ptr(reinterpret_cast<const double *>(base))[idx];
        im = 0.0;
    } else {
        re = (double)global_ptr(reinterpret_cast<const float *>(base))[idx];
        im = 0.0;
    }
}

__device__ __forceinline__ uint64_t abs_bits(double x) {
    return (uint64_t)__double_as_longlong(x) & kAbsMask;
}

// floor(log2 v) for the positive finite double whose bit pattern is `bits`.
__device__ __forceinline__ int ilogb_bits(uint64_t bits) {
    int ef = (int)(bits >> 52);
    if (ef == 0) return -1074 + 63 - __clzll((long long)bits);
    return ef - 1023;
}

// |x| = M * 2^E, M < 2^53 integer (x finite).
__device__ __forceinline__ void decompose(double x, uint64_t &M, int &E) {
    uint64_t b = abs_bits(x);
    int ef = (int)(b >> 52);
    uint64_t mant = b & ((1ull << 52) - 1);
    if (ef == 0) {
        M = mant;
        E = -1074;
    } else {
        M = mant | (1ull << 52);
        E = ef - 1075;
    }
}

// ceil(|x| * 2^sh) for finite x when the result is below 2^63.
__device__ __forceinline__ uint64_t ceil_scaled(double x, int sh) {
    uint64_t M;
    int E;
    decompose(x, M, E);
    if (M == 0) return 0;
    int s = E + sh;
    if (s >= 0) return M << s;
    if (s <= -64) return 1;
    int r = -s;
    return (M + ((1ull << r) - 1)) >> r;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        uint64_t o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

constexpr int kHChunk = 2048;  // k-elements per block along a row

__global__ void fill_u64_kernel(uint64_t *p, int64_t n, uint64_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- row max |x|

// Block (bx, by) of the scan grids: contig rows take 4 rows x kHChunk elements
// (a wave per row), strided rows 256 rows x kHChunk / 8 elements.
template <int EK>
__device__ __forceinline__ void maxabs_contig_body(const OperandView &v, uint64_t *maxbits,
                                                   int64_t bx, int64_t by) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r = bx * 4 + wave;
    if (r >= v.rows) return;
    const int64_t h0 = by * kHChunk;
    const int64_t h1 = min(v.k, h0 + kHChunk);
    uint64_t m = 0;
    for (int64_t h = h0 + lane; h < h1; h += 64) {
        double re, im;
        load_elem<EK>(v.base, r * v.stride_r + h, re, im);
        uint64_t a = abs_bits(re), b = abs_bits(im);
        m = max(m, max(a, b));
    }
    m = wave_max_u64(m);
    if (lane == 0 && m) atomicMax((unsigned long long *)&maxbits[r], (unsigned long long)m);
}

template <int EK>
__device__ __forceinline__ void maxabs_strided_body(const OperandView &v, uint64_t *maxbits,
                                                    int64_t bx, int64_t by, int hc) {
    const int64_t r = bx * 256 + threadIdx.x;
    if (r >= v.rows) return;
    const int64_t h0 = by * hc;
    const int64_t h1 = min(v.k, h0 + hc);
    uint64_t m = 0;
    for (int64_t h = h0; h < h1; ++h) {
        double re, im;
        load_elem<EK>(v.base, r + h * v.stride_h, re, im);
        m = max(m, max(abs_bits(re), abs_bits(im)));
    }
    if (m) atomicMax((unsigned long long *)&maxbits[r], (unsigned long long)m);
}

// ---------------------------------------------------------------- fast-mode sum of squares
// sigma_r = sum over the 2k reals of ceil(|x| 2^(F - e_r))^2, e_r = floor(log2 max|x|):
// an integer upper bound of 2^(2F) ||row / 2^e_r||_2^2, independent of summation order.
// With STATS (the moduli-count predictor's statistics, taken in the same pass):
// tau_r = sum ceil(|x| 2^(F - e_r)) (an upper bound of 2^F ||row / 2^e_r||_1) and the
// number of zero reals of the operand, added to *zeros (all rows, finite or not).
// Real operands have k reals per row (the imaginary parts do not exist).

template <int EK, bool STATS>
__device__ __forceinline__ void sigma_contig_body(const OperandView &v, const uint64_t *maxbits,
                                                  uint64_t *sigma, uint64_t *tau, uint64_t *zeros,
                                                  int64_t bx, int64_t by) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r = bx * 4 + wave;
    if (r >= v.rows) return;
    const uint64_t mb = maxbits[r];
    const bool live = mb != 0 && mb < kInfBits;
    if (!STATS && !live) return;
    const int sh = live ? kSigmaFracBits - ilogb_bits(mb) : 0;
    const int64_t h0 = by * kHChunk;
    const int64_t h1 = min(v.k, h0 + kHChunk);
    uint64_t s = 0, t = 0, z = 0;
    for (int64_t h = h0 + lane; h < h1; h += 64) {
        double re, im;
        load_elem<EK>(v.base, r * v.stride_r + h, re, im);
        if constexpr (STATS) z += (re == 0.0) + (!elem_real(EK) && im == 0.0);
        if (!live) continue;
        uint64_t a = ceil_scaled(re, sh), b = ceil_scaled(im, sh);
        s += a * a + b * b;
        if constexpr (STATS) t += a + b;
    }
    s = wave_sum_u64(s);
    if (lane == 0 && s) atomicAdd((unsigned long long *)&sigma[r], (unsigned long long)s);
    if constexpr (STATS) {
        t = wave_sum_u64(t);
        z = wave_sum_u64(z);
        if (lane == 0 && t) atomicAdd((unsigned long long *)&tau[r], (unsigned long long)t);
        if (lane == 0 && z) atomicAdd((unsigned long long *)zeros, (unsigned long long)z);
    }
}

template <int EK, bool STATS>
__device__ __forceinline__ void sigma_strided_body(const OperandView &v, const uint64_t *maxbits,
                                                   uint64_t *sigma, uint64_t *tau, uint64_t *zeros,
                                                   int64_t bx, int64_t by, int hc) {
    const int64_t r = bx * 256 + threadIdx.x;
    if (r >= v.rows) return;
    const uint64_t mb = maxbits[r];
    const bool live = mb != 0 && mb < kInfBits;
    if (!STATS && !live) return;
    const int sh = live ? kSigmaFracBits - ilogb_bits(mb) : 0;
    const int64_t h0 = by * hc;
    const int64_t h1 = min(v.k, h0 + hc);
    uint64_t s = 0, t = 0, z = 0;
    for (int64_t h = h0; h < h1; ++h) {
        double re, im;
        load_elem<EK>(v.base, r + h * v.stride_h, re, im);
        if constexpr (STATS) z += (re == 0.0) + (!elem_real(EK) && im == 0.0);
        if (!live) continue;
        uint64_t a = ceil_scaled(re, sh), b = ceil_scaled(im, sh);
        s += a * a + b * b;
        if constexpr (STATS) t += a + b;
    }
    if (s) atomicAdd((unsigned long long *)&sigma[r], (unsigned long long)s);
    if constexpr (STATS) {
        if (t) atomicAdd((unsigned long long *)&tau[r], (unsigned long long)t);
        if (z) atomicAdd((unsigned long long *)zeros, (unsigned long long)z);
    }
}

// ---------------------------------------------------------------- exponents
// Fast mode: mu_r = t - e_r with t the largest integer <= P'_fast - 1 such that
// 8 sigma 4^t <= (P - 1) 2^(2F)  (the Cauchy-Schwarz rule of Section III-B in
// exact integer form).  Accurate mode: mu_r = (5 - e_r) + t with t the largest
// integer such that 2 X_r 4^t <= P - 1, X_r the row maximum of the bound product.

__device__ __forceinline__ void fast_exponents_body(const uint64_t *maxbits, const uint64_t *sigma,
                                                    int64_t rows, int64_t rows_pad,
                                                    const NTable *tab, int16_t *mu,
                                                    uint32_t *status, int64_t bx) {
    const int64_t r = bx * 256 + threadIdx.x;
    if (r >= rows_pad) return;
    int16_t out = kExpZero;
    if (r < rows) {
        const uint64_t mb = maxbits[r];
        if (mb >= kInfBits) {
            out = kExpNonfinite;
            atomicOr(status, 1u);
        } else if (mb != 0) {
            const uint64_t s = sigma[r];
            int d = 0;
            const OZC_AS_CONST NTable *ct = const_ptr(tab);
            while (d < kThr - 1 && ct->fast_thr[d] < s) ++d;
            out = (int16_t)(ct->fast_tmax - d - ilogb_bits(mb));
        }
    }
    mu[r] = out;
}

__device__ __forceinline__ void accu_exponents_body(const uint64_t *maxbits, const int32_t *X,
                                                    int64_t rows, int64_t rows_pad,
                                                    const NTable *tab, int16_t *mu,
                                                    uint32_t *status, int64_t bx) {
    const int64_t r = bx * 256 + threadIdx.x;
    if (r >= rows_pad) return;
    int16_t out = kExpZero;
    if (r < rows) {
        const uint64_t mb = maxbits[r];
        if (mb >= kInfBits) {
            out = kExpNonfinite;
            atomicOr(status, 1u);
        } else if (mb != 0 && X[r] > 0) {
            const uint64_t x = (uint64_t)X[r];
            int d = 0;
            const OZC_AS_CONST NTable *ct = const_ptr(tab);
            while (d < kThr - 1 && ct->accu_thr[d] < x) ++d;
            out = (int16_t)((kAccuIntBits - 1) - ilogb_bits(mb) + ct->accu_thi - d);
        }
    }
    mu[r] = out;
}

__global__ __launch_bounds__(256) void accu_exponents_kernel(const uint64_t *maxbits,
                                                             const int32_t *X, int64_t rows,
                                                             int64_t rows_pad, const NTable *tab,
                                                             int16_t *mu, uint32_t *status) {
    accu_exponents_body(maxbits, X, rows, rows_pad, tab, mu, status, blockIdx.x);
}

// ---------------------------------------------------------------- accurate-mode magnitudes
// Tile of 32 rows x 64 k-elements per block.  Each thread takes 8 elements
// and writes the 7-bit magnitudes ceil(|x| 2^(5 - e)) of the real and
// imaginary parts and their difference (the three INT8 operands of the bound
// product, Section III-B), staged in LDS and stored zero-padded to
// rows_pad x k_pad in slab-major order: the 64-wide k-slab kb of a plane is a
// contiguous rows_pad x 64-byte block (row r at byte 64 r), so that the
// product kernels stream whole cache lines.

constexpr int kTileR = 32, kTileH = 64, kLdsPitch = 80;

template <int EK, bool CONTIG_H>
__device__ __forceinline__ void ceil7_body(const OperandView &v, const uint64_t *maxbits,
                                           int8_t *dst, int64_t rows_pad, int64_t k_pad,
                                           int64_t bx, int64_t by) {
    constexpr int NPLANES = elem_real(EK) ? 1 : 3;  // real: Abar only; complex: Abar_R, Abar_I, Abar_R - Abar_I
    __shared__ __align__(16) int8_t lds[NPLANES][kTileR][kLdsPitch];
    const int tid = threadIdx.x;
    const int64_t h0 = bx * kTileH;
    const int64_t r0 = by * kTileR;
    const int64_t plane_pitch = rows_pad * k_pad;

#pragma unroll
    for (int e = 0; e < 8; ++e) {
        // element coordinates: consecutive lanes follow the contiguous direction
        const int hl = CONTIG_H ? (tid & 63) : (tid >> 5) + 8 * e;
        const int rl = CONTIG_H ? (tid >> 6) + 4 * e : (tid & 31);
        const int64_t r = r0 + rl, h = h0 + hl;
        int a = 0, b = 0;
        if (r < v.rows && h < v.k) {
            const uint64_t mb = maxbits[r];
            if (mb != 0 && mb < kInfBits) {
                const int ex = ilogb_bits(mb);
                double re, im;
                load_elem<EK>(v.base, r * v.stride_r + h * v.stride_h, re, im);
                if (v.conj) im = -im;
                a = (int)ceil_scaled(re, (kAccuIntBits - 1) - ex);
                b = (int)ceil_scaled(im, (kAccuIntBits - 1) - ex);
            }
        }
        lds[0][rl][hl] = (int8_t)a;
        if constexpr (NPLANES == 3) {
            lds[1][rl][hl] = (int8_t)b;
            lds[2][rl][hl] = (int8_t)(a - b);
        }
    }
    __syncthreads();
    for (int t = tid; t < NPLANES * kTileR * 4; t += 256) {
        const int pl = t >> 7, row = (t >> 2) & 31, seg = t & 3;
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const u32x4 val = *reinterpret_cast<const u32x4 *>(&lds[pl][row][seg * 16]);
        int8_t *out = dst + (int64_t)pl * plane_pitch + (bx * rows_pad + r0 + row) * kTileH + seg * 16;
        *global_ptr(reinterpret_cast<u32x4 *>(out)) = val;
    }
}

// ---------------------------------------------------------------- residue split
// Truncation a' = trunc(x 2^mu) and symmetric residues modulo every p_l (and,
// for Karatsuba, the reduced sum of the real and imaginary residues), written
// with zero k-padding to k_pad in the slab-major order of the product kernels
// (rows up to rows_pad; the padding rows are left as they are).  No LDS staging: a block of 256 threads covers 16 rows and one
// 64-wide k-slab; each thread holds 4 consecutive k of one row and writes
// their residues as one 4-byte word per plane and modulus.  Sixteen
// consecutive lanes share a row, so each wave writes 4 whole 64-byte rows
// (256 contiguous bytes) per plane and modulus.  Loads: for rows contiguous
// with each other one load instruction reads 4 rows at 16 k (64-byte runs);
// for rows with contiguous k each lane reads its own 64-byte run.
//
// Residues through byte dot products: the signed a' is written as the W-word integer
// u = a' + 2^(32 W - 1) (0 <= u < 2^(32 W), W the smallest word count with
// |a'| < 2^(32 W - 1)), and per modulus x' = sum_j u_j w_j + 128 - (2^(32 W - 1) mod p),
// with u_j the bytes of u and w_j = 2^(8 j) mod p in [0, p - 1]: one unsigned 4-byte
// dot product per word (the offsets enter as the accumulator's start), so that
// x = x' - 128 is congruent to a' modulo p and |x| <= 16 * 255 * 255 + 255 < 2^20.
// Its symmetric residue s comes in FP32 as the byte s + 128 = x' - p q with
// q = floor(fl(x' fl(1/p) + (0.5 - 128 fl(1/p)))) = floor(fl(x fl(1/p) + 0.5)), one fma
// (the offset is exact): the computed value is within |x / p| 2^-24 + ulp / 2 < 1 / (2p)
// of x / p + 1/2, which for odd p lies at least 1 / (2p) from every integer, so q is
// x / p rounded to the nearest integer; for p = 256 everything is exact and a tie
// rounds up, giving s = -128.  So s + 128 is an exact integer in [0, 255]: one
// conversion-and-insert per byte, and flipping bit 7 of each byte gives the signed
// residue.  The reduced sum of the real and imaginary residues takes the same rule.
constexpr int kEPT = 4;                   // k-consecutive elements per thread
constexpr int kDirectRows = 4 * kEPT;     // 256 threads, 64 / kEPT threads per row

__device__ __forceinline__ uint32_t pack_bytes(int a, int b, int c, int d) {
    return (uint32_t)(a & 0xff) | ((uint32_t)(b & 0xff) << 8) | ((uint32_t)(c & 0xff) << 16) |
           ((uint32_t)(d & 0xff) << 24);
}

// Four residues (one byte each, k ascending) as one store.
__device__ __forceinline__ void store_word(int8_t *p, uint32_t w) {
    *global_ptr(reinterpret_cast<uint32_t *>(p)) = w;
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
// The residues r[0..kEPT-1] as one store.
static_assert(kEPT == 2 || kEPT == 4 || kEPT == 8, "2, 4 or 8 elements per thread");
template <int E>
__device__ __forceinline__ void store_res(int8_t *p, const int (&r)[E]) {
    if constexpr (E == 8) {
        const u32x2 w{pack_bytes(r[0], r[1], r[2], r[3]), pack_bytes(r[4], r[5], r[6], r[7])};
        *global_ptr(reinterpret_cast<u32x2 *>(p)) = w;
    } else if constexpr (E == 4) {
        *global_ptr(reinterpret_cast<uint32_t *>(p)) = pack_bytes(r[0], r[1], r[2], r[3]);
    } else {
        *global_ptr(reinterpret_cast<uint16_t *>(p)) = (uint16_t)((r[0] & 0xff) | ((r[1] & 0xff) << 8));
    }
}

// u = a' + 2^(32 W - 1) for a' = trunc(|x| 2^mu) signed like x (|a'| < 2^(32 W - 1)),
// as W little-endian 32-bit words, in FP64: a' is exact as a double (|x| 2^mu is a
// power-of-two scaling of x, and anything below 1 truncates to 0), and the words come
// off from the bottom, q_{i+1} = floor(q_i 2^-32), word_i = q_i - 2^32 q_{i+1} in
// [0, 2^32) (exact: an integer below 2^32); the top q is signed, and adding the bias
// 2^31 to it flips its sign bit.
template <int W>
__device__ __forceinline__ void biased_words(double x, int mu, uint32_t (&u)[W]) {
    double q = __builtin_trunc(__builtin_ldexp(x, mu));
#pragma unroll
    for (int i = 0; i < W - 1; ++i) {
        const double hi = __builtin_floor(q * 0x1p-32);
        u[i] = (uint32_t)__builtin_fma(hi, -0x1p32, q);
        q = hi;
    }
    u[W - 1] = (uint32_t)(int32_t)q ^ 0x80000000u;
}

// x' = sum_j u_j w_j + 128 - (2^(32 W - 1) mod p) as a float (an exact integer).
template <int W>
__device__ __forceinline__ float byte_dot(const uint32_t (&u)[W], const uint32_t (&wb)[W],
                                          uint32_t bias) {
    uint32_t acc = bias;
#pragma unroll
    for (int i = 0; i < W; ++i) acc = __builtin_amdgcn_udot4(u[i], wb[i], acc, false);
    return (float)(int32_t)acc;
}

// s + 128 for the symmetric residue s of x = x' - 128 (x' an exact integer, |x| < 2^20).
__device__ __forceinline__ float smod_u8(float xs, float p, float ip, float rbias) {
    return __builtin_fmaf(-__builtin_floorf(__builtin_fmaf(xs, ip, rbias)), p, xs);
}

template <int EK, bool CONTIG_H, int NPLANES, int W>
__device__ __forceinline__ void split_body(const OperandView &v, const int16_t *__restrict__ mu,
                                           const NTable *__restrict__ tab, int nmod,
                                           int8_t *__restrict__ dst, int64_t rows_pad,
                                           int64_t k_pad, int64_t bx, int64_t by) {
    const int tid = threadIdx.x;
    constexpr int TPR = kTileH / kEPT;  // threads per row
    const int rl = tid / TPR;
    const int oc = tid % TPR;
    const int64_t r = by * kDirectRows + rl;
    const int64_t h0 = bx * kTileH + kEPT * oc;
    const int64_t plane_pitch = rows_pad * k_pad;

    // Rows past the operand (row padding) are not written: they meet only output rows or
    // columns past the product, which nothing reads.  Padding along k must be zero.
    if (r >= v.rows) return;
    const int ex = global_ptr(mu)[r];
    const bool live = ex != kExpZero && ex != kExpNonfinite;
    int8_t *out = dst + (bx * rows_pad + r) * kTileH + kEPT * oc;
    if (!live || h0 >= v.k) {  // k padding, or a row without scaling: every residue is 0
        const int z[kEPT] = {};
        for (int q = 0; q < nmod * NPLANES; ++q) store_res(out + (int64_t)q * plane_pitch, z);
        return;
    }
    static_assert(NPLANES != 1 || elem_real(EK), "one residue plane for real operands only");
    static_assert(kEPT == 4, "one 4-byte word of residues per plane and modulus");
    // elements past k (the ragged last slab) enter as zeros, whose residues are 0
    uint32_t uR[kEPT][W], uI[kEPT][W];
#pragma unroll
    for (int j = 0; j < kEPT; ++j) {
        double re = 0.0, im = 0.0;
        const int64_t h = h0 + j;
        if (h < v.k) {
            load_elem<EK>(v.base, r * v.stride_r + h * v.stride_h, re, im);
            if (v.conj) im = -im;
        }
        biased_words<W>(re, ex, uR[j]);
        if constexpr (NPLANES > 1) biased_words<W>(im, ex, uI[j]);
    }

    for (int l = 0; l < nmod; ++l) {
        const OZC_AS_CONST ModConst &mc = const_ptr(tab)->mod[l];
        const float p = mc.pf, ip = mc.ipf, rb = mc.rbias;
        uint32_t wb[W];
#pragma unroll
        for (int i = 0; i < W; ++i) wb[i] = mc.wbyte[i];
        const uint32_t bias = mc.wbias[W - 1];
        uint32_t wa = 0, wbi = 0, wc = 0;  // residues + 128 as bytes, k ascending
#pragma unroll
        for (int j = 0; j < kEPT; ++j) {
            const float sa = smod_u8(byte_dot<W>(uR[j], wb, bias), p, ip, rb);
            wa = __builtin_amdgcn_cvt_pk_u8_f32(sa, j, wa);
            if constexpr (NPLANES > 1) {
                const float sb = smod_u8(byte_dot<W>(uI[j], wb, bias), p, ip, rb);
                wbi = __builtin_amdgcn_cvt_pk_u8_f32(sb, j, wbi);
                if constexpr (NPLANES == 3) {  // (s_a + s_b) + 128 = (sa - 128) + sb
                    const float sc = smod_u8((sa - 128.0f) + sb, p, ip, rb);
                    wc = __builtin_amdgcn_cvt_pk_u8_f32(sc, j, wc);
                }
            }
        }
        int8_t *o = out + (int64_t)l * NPLANES * plane_pitch;
        store_word(o, wa ^ 0x80808080u);
        if constexpr (NPLANES > 1) store_word(o + plane_pitch, wbi ^ 0x80808080u);
        if constexpr (NPLANES == 3) store_word(o + 2 * plane_pitch, wc ^ 0x80808080u);
    }
}

// ---------------------------------------------------------------- kernels (one problem)

template <int EK>
__global__ __launch_bounds__(256) void row_maxabs_contig(OperandView v, uint64_t *maxbits) {
    maxabs_contig_body<EK>(v, maxbits, blockIdx.x, blockIdx.y);
}
template <int EK>
__global__ __launch_bounds__(256) void row_maxabs_strided(OperandView v, uint64_t *maxbits, int hc) {
    maxabs_strided_body<EK>(v, maxbits, blockIdx.x, blockIdx.y, hc);
}
template <int EK, bool STATS>
__global__ __launch_bounds__(256) void row_sigma_contig(OperandView v, const uint64_t *maxbits,
                                                        uint64_t *sigma, uint64_t *tau,
                                                        uint64_t *zeros) {
    sigma_contig_body<EK, STATS>(v, maxbits, sigma, tau, zeros, blockIdx.x, blockIdx.y);
}
template <int EK, bool STATS>
__global__ __launch_bounds__(256) void row_sigma_strided(OperandView v, const uint64_t *maxbits,
                                                         uint64_t *sigma, uint64_t *tau,
                                                         uint64_t *zeros, int hc) {
    sigma_strided_body<EK, STATS>(v, maxbits, sigma, tau, zeros, blockIdx.x, blockIdx.y, hc);
}
// The scans of both operands of one call in one launch, blocks of A first, then those
// of B, each on the grid its own launch would have: one ramp-up and tail per pass
// instead of two, which shows where an operand takes tens of microseconds.  The
// maxima and the integer sums of squares are combined by atomics, so the result does
// not depend on the order of the blocks.
struct ScanSide {
    OperandView v;
    uint64_t *maxbits, *sigma;
    uint64_t *tau, *zeros;  // pass 2: the predictor's statistics
    int64_t gx, blocks;     // grid columns and blocks of this operand
    int hc;                 // strided layout: k-elements per thread
};
// PASS 0: row maxima; 1: sums of squares; 2: sums of squares and the statistics
template <int EK, int PASS>
__device__ __forceinline__ void scan_side(const ScanSide &sd, int64_t lb) {
    const int64_t bx = lb % sd.gx, by = lb / sd.gx;
    if (sd.v.contig_h) {
        if constexpr (PASS > 0) sigma_contig_body<EK, PASS == 2>(sd.v, sd.maxbits, sd.sigma, sd.tau, sd.zeros, bx, by);
        else maxabs_contig_body<EK>(sd.v, sd.maxbits, bx, by);
    } else {
        if constexpr (PASS > 0)
            sigma_strided_body<EK, PASS == 2>(sd.v, sd.maxbits, sd.sigma, sd.tau, sd.zeros, bx, by, sd.hc);
        else maxabs_strided_body<EK>(sd.v, sd.maxbits, bx, by, sd.hc);
    }
}
template <int EK, int PASS>
__global__ __launch_bounds__(256) void pair_scan_kernel(ScanSide a, ScanSide b) {
    const int64_t blk = blockIdx.x;
    if (blk < a.blocks) scan_side<EK, PASS>(a, blk);
    else scan_side<EK, PASS>(b, blk - a.blocks);
}
__global__ __launch_bounds__(256) void fast_exponents_kernel(const uint64_t *maxbits,
                                                             const uint64_t *sigma, int64_t rows,
                                                             int64_t rows_pad, const NTable *tab,
                                                             int16_t *mu, uint32_t *status) {
    fast_exponents_body(maxbits, sigma, rows, rows_pad, tab, mu, status, blockIdx.x);
}
// The exponents of both operands of one call in one launch (the blocks of A first).
struct ExpSide {
    const uint64_t *maxbits, *sigma;
    int64_t rows, rows_pad, blocks;
    int16_t *mu;
};
__global__ __launch_bounds__(256) void pair_fast_exponents_kernel(ExpSide a, ExpSide b,
                                                                  const NTable *tab, uint32_t *status) {
    const int64_t blk = blockIdx.x;
    if (blk < a.blocks) fast_exponents_body(a.maxbits, a.sigma, a.rows, a.rows_pad, tab, a.mu, status, blk);
    else fast_exponents_body(b.maxbits, b.sigma, b.rows, b.rows_pad, tab, b.mu, status, blk - a.blocks);
}
template <int EK, bool CONTIG_H, int NPLANES, int W>
__global__ __launch_bounds__(256) void split_kernel(OperandView v, const int16_t *__restrict__ mu,
                                                    const NTable *__restrict__ tab, int nmod,
                                                    int8_t *__restrict__ dst, int64_t rows_pad,
                                                    int64_t k_pad) {
    split_body<EK, CONTIG_H, NPLANES, W>(v, mu, tab, nmod, dst, rows_pad, k_pad, blockIdx.x,
                                             blockIdx.y);
}

template <int EK, bool CONTIG_H>
__global__ __launch_bounds__(256) void ceil7_kernel(OperandView v, const uint64_t *maxbits,
                                                    int8_t *dst, int64_t rows_pad, int64_t k_pad) {
    ceil7_body<EK, CONTIG_H>(v, maxbits, dst, rows_pad, k_pad, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------- kernels (batched)

// Last segment whose first block is <= b (first blocks ascending).
template <typename F>
__device__ __forceinline__ int find_seg(int n, int64_t b, F first) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first(mid) <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__host__ __device__ __forceinline__ int64_t scan_grid_x(const OperandView &v) {
    return v.contig_h ? (v.rows + 3) / 4 : (v.rows + 255) / 256;
}
__host__ __device__ __forceinline__ int64_t scan_grid_y(const OperandView &v) {
    const int64_t hc = v.contig_h ? kHChunk : kHChunk / 8;
    return (v.k + hc - 1) / hc;
}

// PASS 0: row maxima; 1: sums of squares; 2: sums of squares with the predictor's
// statistics (BatchOperand::tau, zeros)
template <int EK, int PASS>
__global__ __launch_bounds__(256) void batch_scan_kernel(const BatchOperand *ops, int nops) {
    const int64_t b = blockIdx.x;
    const int o = find_seg(nops, b, [&](int i) { return ops[i].blk_scan; });
    const OperandView v = ops[o].v;
    const int64_t lb = b - ops[o].blk_scan, gx = scan_grid_x(v);
    const int64_t bx = lb % gx, by = lb / gx;
    const BatchOperand &op = ops[o];
    if (v.contig_h) {
        if constexpr (PASS > 0) sigma_contig_body<EK, PASS == 2>(v, op.maxbits, op.sigma, op.tau, op.zeros, bx, by);
        else maxabs_contig_body<EK>(v, op.maxbits, bx, by);
    } else {
        if constexpr (PASS > 0)
            sigma_strided_body<EK, PASS == 2>(v, op.maxbits, op.sigma, op.tau, op.zeros, bx, by, kHChunk / 8);
        else maxabs_strided_body<EK>(v, op.maxbits, bx, by, kHChunk / 8);
    }
}

__global__ __launch_bounds__(256) void batch_fast_exponents_kernel(const BatchOperand *ops, int nops,
                                                                   uint32_t *status) {
    const int64_t b = blockIdx.x;
    const int o = find_seg(nops, b, [&](int i) { return ops[i].blk_exp; });
    const BatchOperand &op = ops[o];
    fast_exponents_body(op.maxbits, op.sigma, op.v.rows, op.rows_pad, op.tab, op.mu, status,
                        b - op.blk_exp);
}

__global__ __launch_bounds__(256) void batch_accu_exponents_kernel(const BatchOperand *ops, int nops,
                                                                   uint32_t *status) {
    const int64_t b = blockIdx.x;
    const int o = find_seg(nops, b, [&](int i) { return ops[i].blk_exp; });
    const BatchOperand &op = ops[o];
    accu_exponents_body(op.maxbits, op.X, op.v.rows, op.rows_pad, op.tab, op.mu, status,
                        b - op.blk_exp);
}

template <int EK>
__global__ __launch_bounds__(256) void batch_ceil7_kernel(const BatchOperand *ops, int nops) {
    const int64_t b = blockIdx.x;
    const int o = find_seg(nops, b, [&](int i) { return ops[i].blk_ceil7; });
    const BatchOperand &op = ops[o];
    const int64_t lb = b - op.blk_ceil7, gx = op.k_pad / kTileH;
    const int64_t bx = lb % gx, by = lb / gx;
    if (op.v.contig_h) ceil7_body<EK, true>(op.v, op.maxbits, op.bar, op.rows_pad, op.k_pad, bx, by);
    else ceil7_body<EK, false>(op.v, op.maxbits, op.bar, op.rows_pad, op.k_pad, bx, by);
}

// Operands of one launch may have different moduli counts; W covers the largest |a'|.
template <int EK, int NPLANES, int W>
__global__ __launch_bounds__(256) void batch_split_kernel(const BatchOperand *ops, int nops) {
    const int64_t b = blockIdx.x;
    const int o = find_seg(nops, b, [&](int i) { return ops[i].blk_split; });
    const BatchOperand &op = ops[o];
    const int64_t lb = b - op.blk_split, gx = op.k_pad / kTileH;
    const int64_t bx = lb % gx, by = lb / gx;
    if (op.v.contig_h)
        split_body<EK, true, NPLANES, W>(op.v, op.mu, op.tab, op.nmod, op.res, op.rows_pad,
                                             op.k_pad, bx, by);
    else
        split_body<EK, false, NPLANES, W>(op.v, op.mu, op.tab, op.nmod, op.res, op.rows_pad,
                                              op.k_pad, bx, by);
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

#define OZC_W_CASES(CASE) CASE(1) CASE(2) CASE(3) CASE(4)

template <int EK, int NPLANES>
hipError_t batch_split_w(const BatchOperand *ops, int nops, int64_t blocks, int nw, hipStream_t s) {
    dim3 grid((unsigned)blocks);
#define OZC_BSPLIT_CASE(W)                                                                   \
    case W:                                                                                  \
        hipLaunchKernelGGL((batch_split_kernel<EK, NPLANES, W>), grid, dim3(256), 0, s,  \
                           ops, nops);                                                       \
        break;
    switch (nw) {
        OZC_W_CASES(OZC_BSPLIT_CASE)
        default:
            return hipErrorInvalidValue;
    }
#undef OZC_BSPLIT_CASE
    return hipGetLastError();
}

template <int EK, bool CONTIG_H, int NPLANES>
hipError_t split_w(const OperandView &v, const int16_t *mu, const NTable *tab, int nmod, int nw,
                    int8_t *dst, int64_t rows_pad, int64_t k_pad, hipStream_t s) {
    dim3 grid((unsigned)(k_pad / kTileH), (unsigned)(rows_pad / kDirectRows));
#define OZC_SPLIT_CASE(W)                                                                    \
    case W:                                                                                  \
        hipLaunchKernelGGL((split_kernel<EK, CONTIG_H, NPLANES, W>), grid, dim3(256), 0,  \
                           s, v, mu, tab, nmod, dst, rows_pad, k_pad);                       \
        break;
    switch (nw) {
        OZC_W_CASES(OZC_SPLIT_CASE)
        default:
            return hipErrorInvalidValue;
    }
#undef OZC_SPLIT_CASE
    return hipGetLastError();
}
#undef OZC_W_CASES


}  // namespace

hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// k-elements per thread of the strided scans: 256, halved (down to 16) while the grid
// would have fewer than 1024 blocks, so that small operands still spread over the chip.
static int strided_chunk(const OperandView &v) {
    const int64_t bx = (v.rows + 255) / 256;
    int hc = kHChunk / 8;
    while (hc > 16 && bx * ((v.k + hc - 1) / hc) < 1024) hc /= 2;
    return hc;
}

template <int EK>
hipError_t row_maxabs_ek(const OperandView &v, uint64_t *maxbits, hipStream_t s) {
    if (v.contig_h) {
        dim3 grid((unsigned)((v.rows + 3) / 4), (unsigned)((v.k + kHChunk - 1) / kHChunk));
        hipLaunchKernelGGL(row_maxabs_contig<EK>, grid, dim3(256), 0, s, v, maxbits);
    } else {
        const int hc = strided_chunk(v);
        dim3 grid((unsigned)((v.rows + 255) / 256), (unsigned)((v.k + hc - 1) / hc));
        hipLaunchKernelGGL(row_maxabs_strided<EK>, grid, dim3(256), 0, s, v, maxbits, hc);
    }
    return hipGetLastError();
}

hipError_t launch_row_maxabs(const OperandView &v, int ek, uint64_t *maxbits, hipStream_t s) {
    if (v.rows <= 0 || v.k <= 0) return hipSuccess;
    switch (ek) {
        case kElemZ: return row_maxabs_ek<kElemZ>(v, maxbits, s);
        case kElemC: return row_maxabs_ek<kElemC>(v, maxbits, s);
        case kElemD: return row_maxabs_ek<kElemD>(v, maxbits, s);
        case kElemS: return row_maxabs_ek<kElemS>(v, maxbits, s);
        default: return hipErrorInvalidValue;
    }
}

template <int EK, bool STATS>
hipError_t row_sigma_ek(const OperandView &v, const uint64_t *maxbits, uint64_t *sigma,
                        uint64_t *tau, uint64_t *zeros, hipStream_t s) {
    if (v.contig_h) {
        dim3 grid((unsigned)((v.rows + 3) / 4), (unsigned)((v.k + kHChunk - 1) / kHChunk));
        hipLaunchKernelGGL((row_sigma_contig<EK, STATS>), grid, dim3(256), 0, s, v, maxbits, sigma,
                           tau, zeros);
    } else {
        const int hc = strided_chunk(v);
        dim3 grid((unsigned)((v.rows + 255) / 256), (unsigned)((v.k + hc - 1) / hc));
        hipLaunchKernelGGL((row_sigma_strided<EK, STATS>), grid, dim3(256), 0, s, v, maxbits, sigma,
                           tau, zeros, hc);
    }
    return hipGetLastError();
}

template <bool STATS>
hipError_t row_sigma_stats(const OperandView &v, int ek, const uint64_t *maxbits, uint64_t *sigma,
                           uint64_t *tau, uint64_t *zeros, hipStream_t s) {
    switch (ek) {
        case kElemZ: return row_sigma_ek<kElemZ, STATS>(v, maxbits, sigma, tau, zeros, s);
        case kElemC: return row_sigma_ek<kElemC, STATS>(v, maxbits, sigma, tau, zeros, s);
        case kElemD: return row_sigma_ek<kElemD, STATS>(v, maxbits, sigma, tau, zeros, s);
        case kElemS: return row_sigma_ek<kElemS, STATS>(v, maxbits, sigma, tau, zeros, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_row_sigma(const OperandView &v, int ek, const uint64_t *maxbits,
                            uint64_t *sigma, hipStream_t s, uint64_t *tau, uint64_t *zeros) {
    if (v.rows <= 0 || v.k <= 0) return hipSuccess;
    if ((tau == nullptr) != (zeros == nullptr)) return hipErrorInvalidValue;
    if (tau) return row_sigma_stats<true>(v, ek, maxbits, sigma, tau, zeros, s);
    return row_sigma_stats<false>(v, ek, maxbits, sigma, nullptr, nullptr, s);
}

static ScanSide scan_side_of(const OperandView &v, uint64_t *maxbits, uint64_t *sigma,
                             uint64_t *tau, uint64_t *zeros) {
    ScanSide sd{v, maxbits, sigma, tau, zeros, 0, 0, 0};
    if (v.rows <= 0 || v.k <= 0) return sd;  // no blocks
    if (v.contig_h) {
        sd.gx = (v.rows + 3) / 4;
        sd.blocks = sd.gx * ((v.k + kHChunk - 1) / kHChunk);
    } else {
        sd.hc = strided_chunk(v);
        sd.gx = (v.rows + 255) / 256;
        sd.blocks = sd.gx * ((v.k + sd.hc - 1) / sd.hc);
    }
    return sd;
}

template <int EK>
hipError_t pair_scans_ek(const ScanSide &a, const ScanSide &b, int pass, hipStream_t s) {
    const int64_t blocks = a.blocks + b.blocks;
    if (blocks == 0) return hipSuccess;
    if (blocks > INT32_MAX) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)blocks);
    if (pass == 2) hipLaunchKernelGGL((pair_scan_kernel<EK, 2>), grid, dim3(256), 0, s, a, b);
    else if (pass == 1) hipLaunchKernelGGL((pair_scan_kernel<EK, 1>), grid, dim3(256), 0, s, a, b);
    else hipLaunchKernelGGL((pair_scan_kernel<EK, 0>), grid, dim3(256), 0, s, a, b);
    return hipGetLastError();
}

hipError_t launch_pair_scans(const OperandView &va, const OperandView &vb, int ek, uint64_t *maxA,
                             uint64_t *maxB, uint64_t *sigA, uint64_t *sigB, bool sigma,
                             hipStream_t s, uint64_t *tauA, uint64_t *tauB, uint64_t *zeros) {
    const bool stats = tauA != nullptr;
    if (stats != (tauB != nullptr) || stats != (zeros != nullptr) || (stats && !sigma))
        return hipErrorInvalidValue;
    const ScanSide a = scan_side_of(va, maxA, sigA, tauA, zeros);
    const ScanSide b = scan_side_of(vb, maxB, sigB, tauB, zeros);
    const int pass = stats ? 2 : (sigma ? 1 : 0);
    switch (ek) {
        case kElemZ: return pair_scans_ek<kElemZ>(a, b, pass, s);
        case kElemC: return pair_scans_ek<kElemC>(a, b, pass, s);
        case kElemD: return pair_scans_ek<kElemD>(a, b, pass, s);
        case kElemS: return pair_scans_ek<kElemS>(a, b, pass, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pair_fast_exponents(const uint64_t *maxA, const uint64_t *sigA, int64_t m,
                                      int64_t m_pad, int16_t *mu, const uint64_t *maxB,
                                      const uint64_t *sigB, int64_t n, int64_t n_pad, int16_t *nu,
                                      const NTable *tab, uint32_t *status, hipStream_t s) {
    const ExpSide a{maxA, sigA, m, m_pad, m_pad > 0 ? (m_pad + 255) / 256 : 0, mu};
    const ExpSide b{maxB, sigB, n, n_pad, n_pad > 0 ? (n_pad + 255) / 256 : 0, nu};
    const int64_t blocks = a.blocks + b.blocks;
    if (blocks == 0) return hipSuccess;
    if (blocks > INT32_MAX) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(pair_fast_exponents_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, b, tab,
                       status);
    return hipGetLastError();
}

hipError_t launch_fast_exponents(const uint64_t *maxbits, const uint64_t *sigma, int64_t rows,
                                 int64_t rows_pad, const NTable *tab, int16_t *mu,
                                 uint32_t *status, hipStream_t s) {
    if (rows_pad <= 0) return hipSuccess;
    hipLaunchKernelGGL(fast_exponents_kernel, dim3((unsigned)((rows_pad + 255) / 256)), dim3(256),
                       0, s, maxbits, sigma, rows, rows_pad, tab, mu, status);
    return hipGetLastError();
}

hipError_t launch_accu_exponents(const uint64_t *maxbits, const int32_t *X, int64_t rows,
                                 int64_t rows_pad, const NTable *tab, int16_t *mu,
                                 uint32_t *status, hipStream_t s) {
    if (rows_pad <= 0) return hipSuccess;
    hipLaunchKernelGGL(accu_exponents_kernel, dim3((unsigned)((rows_pad + 255) / 256)), dim3(256),
                       0, s, maxbits, X, rows, rows_pad, tab, mu, status);
    return hipGetLastError();
}

hipError_t launch_split(const OperandView &v, int ek, const int16_t *mu, const NTable *tab,
                        int nmod, int nplanes, int abits, int8_t *dst, int64_t rows_pad,
                        int64_t k_pad, hipStream_t s) {
    if (abits > kMaxSplitBits) return hipErrorInvalidValue;
    const int nw = split_words(abits);
    if (rows_pad % kDirectRows || k_pad % kTileH) return hipErrorInvalidValue;
    if ((nplanes == 1) != elem_real(ek)) return hipErrorInvalidValue;
#define OZC_SPLIT_ARGS v, mu, tab, nmod, nw, dst, rows_pad, k_pad, s
#define OZC_SPLIT_EK(EKV)                                                                  \
    if (v.contig_h) return nplanes == 3 ? split_w<EKV, true, 3>(OZC_SPLIT_ARGS)            \
                                        : split_w<EKV, true, 2>(OZC_SPLIT_ARGS);           \
    return nplanes == 3 ? split_w<EKV, false, 3>(OZC_SPLIT_ARGS)                           \
                        : split_w<EKV, false, 2>(OZC_SPLIT_ARGS);
    switch (ek) {
        case kElemZ: OZC_SPLIT_EK(kElemZ)
        case kElemC: OZC_SPLIT_EK(kElemC)
        case kElemD:
            return v.contig_h ? split_w<kElemD, true, 1>(OZC_SPLIT_ARGS)
                              : split_w<kElemD, false, 1>(OZC_SPLIT_ARGS);
        case kElemS:
            return v.contig_h ? split_w<kElemS, true, 1>(OZC_SPLIT_ARGS)
                              : split_w<kElemS, false, 1>(OZC_SPLIT_ARGS);
        default: return hipErrorInvalidValue;
    }
#undef OZC_SPLIT_EK
#undef OZC_SPLIT_ARGS
}

template <int EK>
hipError_t ceil7_ek(const OperandView &v, const uint64_t *maxbits, int8_t *dst, int64_t rows_pad,
                    int64_t k_pad, hipStream_t s) {
    dim3 grid((unsigned)(k_pad / kTileH), (unsigned)(rows_pad / kTileR));
    if (v.contig_h) hipLaunchKernelGGL((ceil7_kernel<EK, true>), grid, dim3(256), 0, s, v, maxbits, dst, rows_pad, k_pad);
    else hipLaunchKernelGGL((ceil7_kernel<EK, false>), grid, dim3(256), 0, s, v, maxbits, dst, rows_pad, k_pad);
    return hipGetLastError();
}

hipError_t launch_ceil7(const OperandView &v, int ek, const uint64_t *maxbits, int8_t *dst,
                        int64_t rows_pad, int64_t k_pad, hipStream_t s) {
    if (rows_pad % kTileR || k_pad % kTileH) return hipErrorInvalidValue;
    switch (ek) {
        case kElemZ: return ceil7_ek<kElemZ>(v, maxbits, dst, rows_pad, k_pad, s);
        case kElemC: return ceil7_ek<kElemC>(v, maxbits, dst, rows_pad, k_pad, s);
        case kElemD: return ceil7_ek<kElemD>(v, maxbits, dst, rows_pad, k_pad, s);
        case kElemS: return ceil7_ek<kElemS>(v, maxbits, dst, rows_pad, k_pad, s);
        default: return hipErrorInvalidValue;
    }
}

int64_t batch_scan_blocks(const OperandView &v) {
    if (v.rows <= 0 || v.k <= 0) return 0;
    return scan_grid_x(v) * scan_grid_y(v);
}
int64_t batch_exp_blocks(int64_t rows_pad) { return (rows_pad + 255) / 256; }
int64_t batch_split_blocks(int64_t rows_pad, int64_t k_pad) {
    return (k_pad / kTileH) * (rows_pad / kDirectRows);
}

hipError_t launch_batch_scan(const BatchOperand *ops, int nops, int64_t blocks, bool single,
                             int pass, hipStream_t s) {
    if (blocks <= 0 || nops <= 0) return hipSuccess;
    dim3 grid((unsigned)blocks);
#define OZC_SCAN(EKV, PV) hipLaunchKernelGGL((batch_scan_kernel<EKV, PV>), grid, dim3(256), 0, s, ops, nops)
    switch ((single ? 3 : 0) + pass) {
        case 0: OZC_SCAN(kElemZ, 0); break;
        case 1: OZC_SCAN(kElemZ, 1); break;
        case 2: OZC_SCAN(kElemZ, 2); break;
        case 3: OZC_SCAN(kElemC, 0); break;
        case 4: OZC_SCAN(kElemC, 1); break;
        case 5: OZC_SCAN(kElemC, 2); break;
        default: return hipErrorInvalidValue;
    }
#undef OZC_SCAN
    return hipGetLastError();
}

hipError_t launch_batch_fast_exponents(const BatchOperand *ops, int nops, int64_t blocks,
                                       uint32_t *status, hipStream_t s) {
    if (blocks <= 0 || nops <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_fast_exponents_kernel, dim3((unsigned)blocks), dim3(256), 0, s, ops, nops,
                       status);
    return hipGetLastError();
}

hipError_t launch_batch_accu_exponents(const BatchOperand *ops, int nops, int64_t blocks,
                                       uint32_t *status, hipStream_t s) {
    if (blocks <= 0 || nops <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_accu_exponents_kernel, dim3((unsigned)blocks), dim3(256), 0, s, ops, nops,
                       status);
    return hipGetLastError();
}

int64_t batch_ceil7_blocks(int64_t rows_pad, int64_t k_pad) {
    return (k_pad / kTileH) * (rows_pad / kTileR);
}

hipError_t launch_batch_ceil7(const BatchOperand *ops, int nops, int64_t blocks, bool single,
                              hipStream_t s) {
    if (blocks <= 0 || nops <= 0) return hipSuccess;
    if (single) hipLaunchKernelGGL((batch_ceil7_kernel<true>), dim3((unsigned)blocks), dim3(256), 0, s, ops, nops);
    else hipLaunchKernelGGL((batch_ceil7_kernel<false>), dim3((unsigned)blocks), dim3(256), 0, s, ops, nops);
    return hipGetLastError();
}

hipError_t launch_batch_split(const BatchOperand *ops, int nops, int64_t blocks, bool single,
                              int nplanes, int abits, hipStream_t s) {
    if (blocks <= 0 || nops <= 0) return hipSuccess;
    if (abits > kMaxSplitBits) return hipErrorInvalidValue;
    const int nw = split_words(abits);
    if (single)
        return nplanes == 3 ? batch_split_w<true, 3>(ops, nops, blocks, nw, s)
                            : batch_split_w<true, 2>(ops, nops, blocks, nw, s);
    return nplanes == 3 ? batch_split_w<false, 3>(ops, nops, blocks, nw, s)
                        : batch_split_w<false, 2>(ops, nops, blocks, nw, s);
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace ozc
