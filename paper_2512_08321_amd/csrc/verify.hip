// Freivalds check of an emulated product: with a random sign vector x,
//   w = C_out x,  z = op(A) (op(B) x),  v = C_in x,
// the result is accepted when, for every row i,
//   |w_i - alpha z_i - beta v_i| <= tol_i,
//   tol_i = rel (|alpha| (|A| (|B| |x|))_i + |beta| (|C_in| |x|)_i) + eval_i,
// where eval_i bounds the double-precision rounding of the three products
// themselves (Higham's gamma_n applied to the same absolute sums).  A wrong
// entry c_ij moves w_i by |c_ij - c*_ij| (|x_j| = 1), so an error larger than
// the tolerance in any row is caught with probability >= 1/2 per vector.
//
// x_j = +1 or -1 from bit 0 of SplitMix64(seed, j) (Steele, Lea, Flood 2014).
// All reductions run in a fixed order, so the verdict is reproducible.
#include "internal.h"

namespace ozc {
namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double sign_of(uint64_t seed, int64_t j) {
    return (splitmix64(seed, (uint64_t)j) & 1ull) ? -1.0 : 1.0;
}

template <bool SINGLE>
__device__ __forceinline__ double2 load_c(const void *p, int64_t idx) {
    if constexpr (SINGLE) {
        const float2 v = reinterpret_cast<const float2 *>(p)[idx];
        return make_double2(v.x, v.y);
    } else {
        return reinterpret_cast<const double2 *>(p)[idx];
    }
}

// Vector source: either the sign vector (vec == nullptr) or a complex vector
// with its absolute companion.
struct VecIn {
    const double2 *v;   // nullptr: x_j = sign_of(seed, j), |x_j| = 1
    const double *va;
    uint64_t seed;
};

__device__ __forceinline__ void vec_at(const VecIn &x, int64_t j, double2 &v, double &va) {
    if (x.v) {
        v = x.v[j];
        va = x.va[j];
    } else {
        v = make_double2(sign_of(x.seed, j), 0.0);
        va = 1.0;
    }
}

constexpr int kChunk = 1024;  // columns per partial sum (N case)

// y = op(M) x for M stored column-major (rows x cols, ld) with op = N:
// y_r = sum_c M[r + c ld] x_c.  Thread per row, block column chunks write
// partials[chunk][r] (value and absolute sum), reduced in order afterwards.
template <bool SINGLE>
__global__ __launch_bounds__(256) void gemv_n_partial(const void *M, int64_t rows, int64_t cols,
                                                      int64_t ld, VecIn x, double2 *part,
                                                      double *part_abs) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    const int64_t c0 = (int64_t)blockIdx.y * kChunk, c1 = min(cols, c0 + kChunk);
    double sr = 0.0, si = 0.0, sa = 0.0;
    for (int64_t c = c0; c < c1; ++c) {
        const double2 m = load_c<SINGLE>(M, r + c * ld);
        double2 v;
        double va;
        vec_at(x, c, v, va);
        sr = fma(m.x, v.x, fma(-m.y, v.y, sr));
        si = fma(m.x, v.y, fma(m.y, v.x, si));
        sa = fma(hypot(m.x, m.y), va, sa);
    }
    part[blockIdx.y * rows + r] = make_double2(sr, si);
    part_abs[blockIdx.y * rows + r] = sa;
}

__global__ void reduce_partials(const double2 *part, const double *part_abs, int64_t rows,
                                int nchunk, double2 *y, double *ya) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    double sr = 0.0, si = 0.0, sa = 0.0;
    for (int c = 0; c < nchunk; ++c) {
        sr += part[c * rows + r].x;
        si += part[c * rows + r].y;
        sa += part_abs[c * rows + r];
    }
    y[r] = make_double2(sr, si);
    ya[r] = sa;
}

// y = op(M) x for op = T or C: y_c = sum_r op(M)[c][r] x_r = sum_r M[r + c ld]^(*) x_r.
// One wave per output entry c, lanes over r, fixed-order butterfly reduction.
template <bool SINGLE>
__global__ __launch_bounds__(256) void gemv_t(const void *M, int64_t rows, int64_t cols, int64_t ld,
                                              int conj, VecIn x, double2 *y, double *ya) {
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= cols) return;
    double sr = 0.0, si = 0.0, sa = 0.0;
    for (int64_t r = lane; r < rows; r += 64) {
        double2 m = load_c<SINGLE>(M, r + c * ld);
        if (conj) m.y = -m.y;
        double2 v;
        double va;
        vec_at(x, r, v, va);
        sr = fma(m.x, v.x, fma(-m.y, v.y, sr));
        si = fma(m.x, v.y, fma(m.y, v.x, si));
        sa = fma(hypot(m.x, m.y), va, sa);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sr += __shfl_xor(sr, off, 64);
        si += __shfl_xor(si, off, 64);
        sa += __shfl_xor(sa, off, 64);
    }
    if (lane == 0) {
        y[c] = make_double2(sr, si);
        ya[c] = sa;
    }
}

// Per-row residual test.  worst[0] receives max_i |res_i| / tol_i as the bit
// pattern of a non-negative double (order-preserving), worst[1] the number of
// failing rows.
__global__ void freivalds_rows(const double2 *w, const double *wa, const double2 *z,
                               const double *za, const double2 *v, const double *va, int64_t m,
                               double ar, double ai, double br, double bi, double rel,
                               double gam, unsigned long long *worst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double er = w[i].x - (ar * z[i].x - ai * z[i].y);
    double ei = w[i].y - (ar * z[i].y + ai * z[i].x);
    double bound = rel * hypot(ar, ai) * za[i];
    double evals = wa[i] + hypot(ar, ai) * za[i];
    if (v) {
        er -= br * v[i].x - bi * v[i].y;
        ei -= br * v[i].y + bi * v[i].x;
        bound += rel * hypot(br, bi) * va[i];
        evals += hypot(br, bi) * va[i];
    }
    const double tol = bound + gam * evals;
    const double res = hypot(er, ei);
    double ratio = tol > 0.0 ? res / tol : (res > 0.0 ? INFINITY : 0.0);
    if (!(ratio == ratio) || !(res == res) || !(tol == tol)) ratio = INFINITY;  // NaN fails
    atomicMax(&worst[0], (unsigned long long)__double_as_longlong(ratio));
    if (ratio > 1.0) atomicAdd(&worst[1], 1ull);
}

__global__ void fill_words(unsigned long long *p, int n) {
    if (threadIdx.x < n) p[threadIdx.x] = 0ull;
}

__global__ void debug_xor_byte(int8_t *p) { p[0] = (int8_t)(p[0] ^ 0x5a); }

__global__ void debug_add_exp(int16_t *mu, int delta) {
    if (mu[0] != kExpZero && mu[0] != kExpNonfinite) mu[0] = (int16_t)(mu[0] + delta);
}

}  // namespace

hipError_t launch_debug_xor_byte(int8_t *p, hipStream_t s) {
    hipLaunchKernelGGL(debug_xor_byte, dim3(1), dim3(1), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_debug_add_exp(int16_t *mu, int delta, hipStream_t s) {
    hipLaunchKernelGGL(debug_add_exp, dim3(1), dim3(1), 0, s, mu, delta);
    return hipGetLastError();
}

// y = op(M) x, ya = |op(M)| |x|.  M column-major rows x cols (ld); op: 0 N, 1 T, 2 C.
// scratch: (ceil(cols / 1024)) * rows * 24 bytes for op = N.
hipError_t launch_gemv(const void *M, bool single, int op, int64_t rows, int64_t cols, int64_t ld,
                       const double2 *xv, const double *xa, uint64_t seed, double2 *y, double *ya,
                       void *scratch, hipStream_t s) {
    VecIn x{xv, xa, seed};
    if (op == 0) {
        if (rows <= 0) return hipSuccess;
        const int nchunk = (int)((cols + kChunk - 1) / kChunk);
        double2 *part = (double2 *)scratch;
        double *part_abs = (double *)(part + (size_t)nchunk * rows);
        if (nchunk > 0) {
            dim3 grid((unsigned)((rows + 255) / 256), (unsigned)nchunk);
            if (single) hipLaunchKernelGGL(gemv_n_partial<true>, grid, dim3(256), 0, s, M, rows, cols, ld, x, part, part_abs);
            else hipLaunchKernelGGL(gemv_n_partial<false>, grid, dim3(256), 0, s, M, rows, cols, ld, x, part, part_abs);
        }
        hipLaunchKernelGGL(reduce_partials, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, part,
                           part_abs, rows, nchunk, y, ya);
    } else {
        if (cols <= 0) return hipSuccess;
        dim3 grid((unsigned)((cols + 3) / 4));
        if (single) hipLaunchKernelGGL(gemv_t<true>, grid, dim3(256), 0, s, M, rows, cols, ld, op == 2 ? 1 : 0, x, y, ya);
        else hipLaunchKernelGGL(gemv_t<false>, grid, dim3(256), 0, s, M, rows, cols, ld, op == 2 ? 1 : 0, x, y, ya);
    }
    return hipGetLastError();
}

size_t gemv_scratch_bytes(int64_t rows, int64_t cols) {
    const int64_t nchunk = (cols + kChunk - 1) / kChunk;
    return (size_t)(nchunk > 0 ? nchunk : 1) * (size_t)(rows > 0 ? rows : 1) * 24;
}

hipError_t launch_freivalds_rows(const double2 *w, const double *wa, const double2 *z,
                                 const double *za, const double2 *v, const double *va, int64_t m,
                                 const double alpha[2], const double beta[2], double rel,
                                 double gam, unsigned long long *worst, hipStream_t s) {
    hipLaunchKernelGGL(fill_words, dim3(1), dim3(64), 0, s, worst, 2);
    if (m <= 0) return hipGetLastError();
    hipLaunchKernelGGL(freivalds_rows, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, w, wa, z,
                       za, v, va, m, alpha[0], alpha[1], beta[0], beta[1], rel, gam, worst);
    return hipGetLastError();
}

}  // namespace ozc
