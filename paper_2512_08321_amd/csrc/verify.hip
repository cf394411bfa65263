// Freivalds check of an emulated product: with a random sign vector x,
//   w = C_out x,  z = op(A) (op(B) x),  v = C_in x,
// the result is accepted when, for every row i,
//   |w_i - alpha z_i - beta v_i| <= tol_i,
//   tol_i = rel (|alpha| (|A| (|B| |x|))_i + |beta| (|C_in| |x|)_i) + eval_i,
// where eval_i bounds the rounding of the check itself.  The three products
// are accumulated in double-double arithmetic (error-free sums and products,
// Dekker / Knuth; products via fused multiply-add), so eval_i is of order
// (n + k) 2^-104 of the same absolute sums and the check can resolve
// tolerances far below double precision.  A wrong entry c_ij moves w_i by
// |c_ij - c*_ij| (|x_j| = 1), so an error larger than the tolerance in any row
// is caught with probability >= 1/2 per vector.
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

// ---- double-double: value hi + lo with |lo| <= ulp(hi) / 2
struct dd {
    double hi, lo;
};
__device__ __forceinline__ dd two_sum(double a, double b) {
    const double s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd fast_two_sum(double a, double b) {  // |a| >= |b|
    const double s = a + b;
    return {s, b - (s - a)};
}
// acc += a * b
__device__ __forceinline__ void dd_fma(dd &acc, double a, double b) {
    const double p = a * b, pe = fma(a, b, -p);
    const dd s = two_sum(acc.hi, p);
    acc = fast_two_sum(s.hi, s.lo + (acc.lo + pe));
}
__device__ __forceinline__ void dd_add(dd &acc, dd x) {
    const dd s = two_sum(acc.hi, x.hi);
    acc = fast_two_sum(s.hi, s.lo + (acc.lo + x.lo));
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

// Vector source: the sign vector (v == nullptr) or a double-double complex
// vector (v: high parts, vlo: low parts) with its absolute companion va.
struct VecIn {
    const double2 *v, *vlo;
    const double *va;
    uint64_t seed;
};

// acc += m * x_j (complex), abs += |m| |x_j|
__device__ __forceinline__ void accum(const VecIn &x, int64_t j, double2 m, dd &re, dd &im,
                                      double &ab) {
    if (x.v) {
        const double2 h = x.v[j], l = x.vlo[j];
        dd_fma(re, m.x, h.x);
        dd_fma(re, -m.y, h.y);
        dd_fma(im, m.x, h.y);
        dd_fma(im, m.y, h.x);
        // low parts: contributions 2^-53 below the high ones, plain double is enough
        re.lo = fma(m.x, l.x, fma(-m.y, l.y, re.lo));
        im.lo = fma(m.x, l.y, fma(m.y, l.x, im.lo));
        ab = fma(hypot(m.x, m.y), x.va[j], ab);
    } else {
        const double s = sign_of(x.seed, j);
        dd_fma(re, m.x, s);
        dd_fma(im, m.y, s);
        ab += hypot(m.x, m.y);
    }
}

// y = op(M) x for M stored column-major (rows x cols, ld) with op = N:
// y_r = sum_c M[r + c ld] x_c.  Thread per row; block (bx, cy) sums the columns of
// chunk cy into partials[cy][r], reduced in order afterwards.
template <bool SINGLE>
__device__ __forceinline__ void gemv_n_partial_body(const void *M, int64_t rows, int64_t cols,
                                                    int64_t ld, int64_t chunk, const VecIn &x,
                                                    double2 *part_hi, double2 *part_lo,
                                                    double *part_abs, int64_t bx, int64_t cy) {
    const int64_t r = bx * 256 + threadIdx.x;
    if (r >= rows) return;
    const int64_t c0 = cy * chunk, c1 = min(cols, c0 + chunk);
    dd re{0.0, 0.0}, im{0.0, 0.0};
    double ab = 0.0;
    for (int64_t c = c0; c < c1; ++c) accum(x, c, load_c<SINGLE>(M, r + c * ld), re, im, ab);
    const int64_t o = cy * rows + r;
    part_hi[o] = make_double2(re.hi, im.hi);
    part_lo[o] = make_double2(re.lo, im.lo);
    part_abs[o] = ab;
}

template <bool SINGLE>
__global__ __launch_bounds__(256) void gemv_n_partial(const void *M, int64_t rows, int64_t cols,
                                                      int64_t ld, int64_t chunk, VecIn x,
                                                      double2 *part_hi, double2 *part_lo,
                                                      double *part_abs) {
    gemv_n_partial_body<SINGLE>(M, rows, cols, ld, chunk, x, part_hi, part_lo, part_abs,
                                blockIdx.x, blockIdx.y);
}

__device__ __forceinline__ void reduce_partials_body(const double2 *part_hi, const double2 *part_lo,
                                                     const double *part_abs, int64_t rows,
                                                     int nchunk, double2 *y, double2 *ylo,
                                                     double *ya, int64_t bx) {
    const int64_t r = bx * 256 + threadIdx.x;
    if (r >= rows) return;
    dd re{0.0, 0.0}, im{0.0, 0.0};
    double ab = 0.0;
    for (int c = 0; c < nchunk; ++c) {
        const double2 h = part_hi[c * rows + r], l = part_lo[c * rows + r];
        dd_add(re, {h.x, l.x});
        dd_add(im, {h.y, l.y});
        ab += part_abs[c * rows + r];
    }
    y[r] = make_double2(re.hi, im.hi);
    ylo[r] = make_double2(re.lo, im.lo);
    ya[r] = ab;
}

__global__ __launch_bounds__(256) void reduce_partials(const double2 *part_hi,
                                                       const double2 *part_lo,
                                                       const double *part_abs, int64_t rows,
                                                       int nchunk, double2 *y, double2 *ylo,
                                                       double *ya) {
    reduce_partials_body(part_hi, part_lo, part_abs, rows, nchunk, y, ylo, ya, blockIdx.x);
}

// y = op(M) x for op = T or C: y_c = sum_r M[r + c ld]^(*) x_r.  One wave per
// output entry (four per block), lanes over r, fixed-order butterfly reduction in
// double-double.
template <bool SINGLE>
__device__ __forceinline__ void gemv_t_body(const void *M, int64_t rows, int64_t cols, int64_t ld,
                                            int conj, const VecIn &x, double2 *y, double2 *ylo,
                                            double *ya, int64_t bx) {
    const int lane = threadIdx.x & 63;
    const int64_t c = bx * 4 + (threadIdx.x >> 6);
    if (c >= cols) return;
    dd re{0.0, 0.0}, im{0.0, 0.0};
    double ab = 0.0;
    for (int64_t r = lane; r < rows; r += 64) {
        double2 m = load_c<SINGLE>(M, r + c * ld);
        if (conj) m.y = -m.y;
        accum(x, r, m, re, im, ab);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        dd_add(re, {__shfl_xor(re.hi, off, 64), __shfl_xor(re.lo, off, 64)});
        dd_add(im, {__shfl_xor(im.hi, off, 64), __shfl_xor(im.lo, off, 64)});
        ab += __shfl_xor(ab, off, 64);
    }
    if (lane == 0) {
        y[c] = make_double2(re.hi, im.hi);
        ylo[c] = make_double2(re.lo, im.lo);
        ya[c] = ab;
    }
}

template <bool SINGLE>
__global__ __launch_bounds__(256) void gemv_t(const void *M, int64_t rows, int64_t cols, int64_t ld,
                                              int conj, VecIn x, double2 *y, double2 *ylo,
                                              double *ya) {
    gemv_t_body<SINGLE>(M, rows, cols, ld, conj, x, y, ylo, ya, blockIdx.x);
}

// (a_r + i a_i) * (z_hi + z_lo) for a double complex a and a double-double complex z
__device__ __forceinline__ void cmul_dd(double ar, double ai, double2 zh, double2 zl, dd &re, dd &im) {
    re = {0.0, 0.0};
    im = {0.0, 0.0};
    dd_fma(re, ar, zh.x);
    dd_fma(re, -ai, zh.y);
    dd_fma(im, ar, zh.y);
    dd_fma(im, ai, zh.x);
    re.lo = fma(ar, zl.x, fma(-ai, zl.y, re.lo));
    im.lo = fma(ar, zl.y, fma(ai, zl.x, im.lo));
}

// Per-row residual test.  worst[0] receives max_i |res_i| / tol_i as the bit
// pattern of a non-negative double (order-preserving), worst[1] the number of
// failing rows.
__device__ __forceinline__ void freivalds_rows_body(
    const double2 *w, const double2 *wl, const double *wa, const double2 *z, const double2 *zl,
    const double *za, const double2 *v, const double2 *vl, const double *va, int64_t m, double ar,
    double ai, double br, double bi, double rel, double gam, unsigned long long *worst, int64_t bx) {
    const int64_t i = bx * 256 + threadIdx.x;
    if (i >= m) return;
    dd er{w[i].x, wl[i].x}, ei{w[i].y, wl[i].y}, tr, ti;
    cmul_dd(-ar, -ai, z[i], zl[i], tr, ti);
    dd_add(er, tr);
    dd_add(ei, ti);
    double bound = rel * hypot(ar, ai) * za[i];
    double evals = wa[i] + hypot(ar, ai) * za[i];
    if (v) {
        cmul_dd(-br, -bi, v[i], vl[i], tr, ti);
        dd_add(er, tr);
        dd_add(ei, ti);
        bound += rel * hypot(br, bi) * va[i];
        evals += hypot(br, bi) * va[i];
    }
    const double tol = bound + gam * evals;
    const double res = hypot(er.hi + er.lo, ei.hi + ei.lo);
    double ratio = tol > 0.0 ? res / tol : (res > 0.0 ? INFINITY : 0.0);
    if (!(ratio == ratio) || !(res == res) || !(tol == tol)) ratio = INFINITY;  // NaN fails
    atomicMax(&worst[0], (unsigned long long)__double_as_longlong(ratio));
    if (ratio > 1.0) atomicAdd(&worst[1], 1ull);
}

__global__ __launch_bounds__(256) void freivalds_rows(
    const double2 *w, const double2 *wl, const double *wa, const double2 *z, const double2 *zl,
    const double *za, const double2 *v, const double2 *vl, const double *va, int64_t m, double ar,
    double ai, double br, double bi, double rel, double gam, unsigned long long *worst) {
    freivalds_rows_body(w, wl, wa, z, zl, za, v, vl, va, m, ar, ai, br, bi, rel, gam, worst,
                        blockIdx.x);
}

// ---- batched check: one launch per kernel over the blocks of many tasks; a block
// finds its task by binary search over the tasks' first blocks (tasks with no block
// in a kernel share their successor's first block and are never selected).
template <typename First>
__device__ __forceinline__ int find_task(int n, int64_t b, First first) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first(mid) <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <bool SINGLE>
__global__ __launch_bounds__(256) void batch_gemv_n_partial(const GemvTask *tasks, int n) {
    const int64_t b = blockIdx.x;
    const GemvTask &t = tasks[find_task(n, b, [&](int i) { return tasks[i].b0[0]; })];
    const int64_t nbx = (t.rows + 255) / 256, local = b - t.b0[0];
    const VecIn x{t.xv, t.xlo, t.xa, t.seed};
    gemv_n_partial_body<SINGLE>(t.M, t.rows, t.cols, t.ld, t.chunk, x, t.ph, t.pl, t.pa,
                                local % nbx, local / nbx);
}

__global__ __launch_bounds__(256) void batch_reduce_partials(const GemvTask *tasks, int n) {
    const int64_t b = blockIdx.x;
    const GemvTask &t = tasks[find_task(n, b, [&](int i) { return tasks[i].b0[1]; })];
    reduce_partials_body(t.ph, t.pl, t.pa, t.rows, t.nchunk, t.y, t.ylo, t.ya, b - t.b0[1]);
}

template <bool SINGLE>
__global__ __launch_bounds__(256) void batch_gemv_t(const GemvTask *tasks, int n) {
    const int64_t b = blockIdx.x;
    const GemvTask &t = tasks[find_task(n, b, [&](int i) { return tasks[i].b0[2]; })];
    const VecIn x{t.xv, t.xlo, t.xa, t.seed};
    gemv_t_body<SINGLE>(t.M, t.rows, t.cols, t.ld, t.op == 2 ? 1 : 0, x, t.y, t.ylo, t.ya,
                        b - t.b0[2]);
}

__global__ __launch_bounds__(256) void batch_freivalds_rows(const RowsTask *tasks, int n) {
    const int64_t b = blockIdx.x;
    const RowsTask &t = tasks[find_task(n, b, [&](int i) { return tasks[i].b0; })];
    freivalds_rows_body(t.w, t.wl, t.wa, t.z, t.zl, t.za, t.v, t.vl, t.va, t.m, t.ar, t.ai, t.br,
                        t.bi, t.rel, t.gam, t.worst, b - t.b0);
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

// Columns per partial sum (op = N): the smallest power of two in [32, 1024] whose
// square reaches cols, which balances the serial work of a partial-sum thread (chunk
// terms) against that of the reduction (cols / chunk terms) and gives small products
// enough blocks.  A function of the column count alone: a product is summed in the same
// order in single and batched checks, so their verdicts agree.
static int64_t gemv_chunk(int64_t cols) {
    int64_t ch = 32;
    while (ch < 1024 && ch * ch < cols) ch *= 2;
    return ch;
}

// y = op(M) x (double-double: y, ylo), ya = |op(M)| |x|.  M column-major rows x
// cols (ld); op: 0 N, 1 T, 2 C.  scratch: gemv_scratch_bytes(rows, cols) for op = N.
hipError_t launch_gemv(const void *M, bool single, int op, int64_t rows, int64_t cols, int64_t ld,
                       const double2 *xv, const double2 *xlo, const double *xa, uint64_t seed,
                       double2 *y, double2 *ylo, double *ya, void *scratch, hipStream_t s) {
    VecIn x{xv, xlo, xa, seed};
    if (op == 0) {
        if (rows <= 0) return hipSuccess;
        const int64_t chunk = gemv_chunk(cols);
        const int nchunk = (int)((cols + chunk - 1) / chunk);
        double2 *ph = (double2 *)scratch;
        double2 *pl = ph + (size_t)nchunk * rows;
        double *pa = (double *)(pl + (size_t)nchunk * rows);
        if (nchunk > 0) {
            dim3 grid((unsigned)((rows + 255) / 256), (unsigned)nchunk);
            if (single) hipLaunchKernelGGL(gemv_n_partial<true>, grid, dim3(256), 0, s, M, rows, cols, ld, chunk, x, ph, pl, pa);
            else hipLaunchKernelGGL(gemv_n_partial<false>, grid, dim3(256), 0, s, M, rows, cols, ld, chunk, x, ph, pl, pa);
        }
        hipLaunchKernelGGL(reduce_partials, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, ph, pl,
                           pa, rows, nchunk, y, ylo, ya);
    } else {
        if (cols <= 0) return hipSuccess;
        dim3 grid((unsigned)((cols + 3) / 4));
        if (single) hipLaunchKernelGGL(gemv_t<true>, grid, dim3(256), 0, s, M, rows, cols, ld, op == 2 ? 1 : 0, x, y, ylo, ya);
        else hipLaunchKernelGGL(gemv_t<false>, grid, dim3(256), 0, s, M, rows, cols, ld, op == 2 ? 1 : 0, x, y, ylo, ya);
    }
    return hipGetLastError();
}

GemvTask make_gemv_task(const void *M, int op, int64_t rows, int64_t cols, int64_t ld,
                        const double2 *xv, const double2 *xlo, const double *xa, uint64_t seed,
                        double2 *y, double2 *ylo, double *ya, void *scratch, int64_t nb[3]) {
    GemvTask t{};
    t.M = M;
    t.rows = rows;
    t.cols = cols;
    t.ld = ld;
    t.op = op;
    t.xv = xv;
    t.xlo = xlo;
    t.xa = xa;
    t.seed = seed;
    t.y = y;
    t.ylo = ylo;
    t.ya = ya;
    for (int i = 0; i < 3; ++i) t.b0[i] = nb[i];
    if (op == 0) {
        if (rows <= 0) return t;
        t.chunk = gemv_chunk(cols);
        t.nchunk = (int32_t)((cols + t.chunk - 1) / t.chunk);
        t.ph = (double2 *)scratch;
        t.pl = t.ph + (size_t)t.nchunk * rows;
        t.pa = (double *)(t.pl + (size_t)t.nchunk * rows);
        const int64_t nbx = (rows + 255) / 256;
        nb[0] += nbx * t.nchunk;
        nb[1] += nbx;
    } else {
        nb[2] += (cols + 3) / 4;
    }
    return t;
}

hipError_t launch_batch_gemv(const GemvTask *tasks, int n, const int64_t nb[3], bool single,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (nb[0] > 0) {
        if (single) hipLaunchKernelGGL(batch_gemv_n_partial<true>, dim3((unsigned)nb[0]), dim3(256), 0, s, tasks, n);
        else hipLaunchKernelGGL(batch_gemv_n_partial<false>, dim3((unsigned)nb[0]), dim3(256), 0, s, tasks, n);
    }
    if (nb[1] > 0)
        hipLaunchKernelGGL(batch_reduce_partials, dim3((unsigned)nb[1]), dim3(256), 0, s, tasks, n);
    if (nb[2] > 0) {
        if (single) hipLaunchKernelGGL(batch_gemv_t<true>, dim3((unsigned)nb[2]), dim3(256), 0, s, tasks, n);
        else hipLaunchKernelGGL(batch_gemv_t<false>, dim3((unsigned)nb[2]), dim3(256), 0, s, tasks, n);
    }
    return hipGetLastError();
}

hipError_t launch_batch_rows(const RowsTask *tasks, int n, int64_t nblocks, hipStream_t s) {
    if (n <= 0 || nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_freivalds_rows, dim3((unsigned)nblocks), dim3(256), 0, s, tasks, n);
    return hipGetLastError();
}

size_t gemv_scratch_bytes(int64_t rows, int64_t cols) {
    const int64_t chunk = gemv_chunk(cols);
    const int64_t nchunk = (cols + chunk - 1) / chunk;
    return (size_t)(nchunk > 0 ? nchunk : 1) * (size_t)(rows > 0 ? rows : 1) * 40;
}

hipError_t launch_freivalds_rows(const double2 *w, const double2 *wl, const double *wa,
                                 const double2 *z, const double2 *zl, const double *za,
                                 const double2 *v, const double2 *vl, const double *va, int64_t m,
                                 const double alpha[2], const double beta[2], double rel,
                                 double gam, unsigned long long *worst, hipStream_t s) {
    hipLaunchKernelGGL(fill_words, dim3(1), dim3(64), 0, s, worst, 2);
    if (m <= 0) return hipGetLastError();
    hipLaunchKernelGGL(freivalds_rows, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, w, wl, wa, z,
                       zl, za, v, vl, va, m, alpha[0], alpha[1], beta[0], beta[1], rel, gam, worst);
    return hipGetLastError();
}

}  // namespace ozc
