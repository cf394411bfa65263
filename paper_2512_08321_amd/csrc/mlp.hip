// Moduli-count predictor: input statistics and a small FP32 perceptron with its
// training step (forward, softmax cross-entropy, backward, Adam).  Not part of
// the paper; it chooses N before the emulation runs (each added modulus multiplies
// P by about 2^7.8, Section II, and the scaling shares those bits between the two
// operands, so the error falls by about 2^-4 per modulus).
//
// Statistics: per row of op(A) / column of op(B) (2k reals), with e = floor(log2
// max|x|) and the scaling pass's integer sums sigma = sum ceil(|x| 2^(20-e))^2 and
// tau = sum ceil(|x| 2^(20-e)) (taken in the same pass, prep.hip), l2 = 0.5 log2
// sigma - 20 and l1 = log2 tau - 20; the feature vector holds log2 m, log2 n,
// log2 k, min/max/mean/std of l2 and l1 over the nonzero rows of each operand, and
// the fraction of zero reals.
//
// Network (parameter layout shared with the C-ABI): xs = (x - mu) / sd,
// h1 = relu(W1 xs + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3; W row-major
// (out x in).  Every floating-point reduction runs in a fixed order and the row
// sums of the statistics are integers, so statistics, predictions and training are
// reproducible run to run.
#include <math.h>

#include "internal.h"

namespace ozc {
namespace {

// One block: statistics of l2 and l1 over the nonzero rows of both operands, from the
// scaling pass's integer sums sigma (2F fraction bits) and tau (F fraction bits):
// l2 = 0.5 (log2 sigma - 2F), l1 = log2 tau - F.
__device__ __forceinline__ void feat_reduce_body(const unsigned long long *s1a,
                                                 const unsigned long long *s2a, int64_t ra,
                                                 const unsigned long long *s1b,
                                                 const unsigned long long *s2b, int64_t rb,
                                                 const unsigned long long *zeros, double m,
                                                 double n, double k, float *out) {
    __shared__ double red[256][10];  // l2 statistics in 0..4, l1 statistics in 5..9
    const int t = threadIdx.x;
    constexpr int fb = kSigmaFracBits;
    float res[16];
    for (int op = 0; op < 2; ++op) {
        const unsigned long long *s1 = op ? s1b : s1a, *s2 = op ? s2b : s2a;
        const int64_t rows = op ? rb : ra;
        double mn[2] = {INFINITY, INFINITY}, mx[2] = {-INFINITY, -INFINITY};
        double sum[2] = {0.0, 0.0}, sq[2] = {0.0, 0.0}, cnt = 0.0;
        for (int64_t r = t; r < rows; r += 256) {
            if (s2[r] == 0) continue;  // zero row (or a row holding inf / NaN)
            const double x[2] = {0.5 * (log2((double)s2[r]) - 2 * fb), log2((double)s1[r]) - fb};
            for (int q = 0; q < 2; ++q) {  // q = 0: l2, 1: l1
                mn[q] = fmin(mn[q], x[q]);
                mx[q] = fmax(mx[q], x[q]);
                sum[q] += x[q];
                sq[q] += x[q] * x[q];
            }
            cnt += 1.0;
        }
        for (int q = 0; q < 2; ++q) {
            red[t][5 * q + 0] = mn[q];
            red[t][5 * q + 1] = mx[q];
            red[t][5 * q + 2] = sum[q];
            red[t][5 * q + 3] = sq[q];
            red[t][5 * q + 4] = cnt;
        }
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if (t < w) {
                for (int q = 0; q < 2; ++q) {
                    double *a = red[t] + 5 * q;
                    const double *b = red[t + w] + 5 * q;
                    a[0] = fmin(a[0], b[0]);
                    a[1] = fmax(a[1], b[1]);
                    a[2] += b[2];
                    a[3] += b[3];
                    a[4] += b[4];
                }
            }
            __syncthreads();
        }
        for (int q = 0; q < 2; ++q) {
            const double *a = red[0] + 5 * q;
            const double c = a[4];
            const double mean = c > 0 ? a[2] / c : 0.0;
            const double var = c > 0 ? fmax(0.0, a[3] / c - mean * mean) : 0.0;
            float *o = res + op * 8 + q * 4;
            o[0] = c > 0 ? (float)a[0] : 0.f;
            o[1] = c > 0 ? (float)a[1] : 0.f;
            o[2] = (float)mean;
            o[3] = (float)sqrt(var);
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = (float)log2(m);
        out[1] = (float)log2(n);
        out[2] = (float)log2(k);
        for (int i = 0; i < 16; ++i) out[3 + i] = res[i];
        out[19] = (float)((double)zeros[0] / (2.0 * (m + n) * k));
    }
}

__global__ __launch_bounds__(256) void feat_reduce_kernel(const unsigned long long *s1a,
                                                          const unsigned long long *s2a,
                                                          int64_t ra, const unsigned long long *s1b,
                                                          const unsigned long long *s2b, int64_t rb,
                                                          const unsigned long long *zeros,
                                                          double m, double n, double k,
                                                          float *out) {
    feat_reduce_body(s1a, s2a, ra, s1b, s2b, rb, zeros, m, n, k, out);
}

__global__ __launch_bounds__(256) void batch_feat_reduce_kernel(const FeatProblem *probs) {
    const FeatProblem &p = probs[blockIdx.x];
    feat_reduce_body(p.s1a, p.s2a, p.ra, p.s1b, p.s2b, p.rb, p.zeros, p.m, p.n, p.k, p.out);
}

// ---------------------------------------------------------------- network

// out[r][o] = act(sum_i W[o][i] in[idx(r)][i] + b[o]); pre keeps the pre-activation.
// With `standardize`, the input is (x - mu) / sd first.
__global__ void dense_fwd_kernel(const float *in, const int *idx, int rows, int din, int dout,
                                 const float *W, const float *b, const float *mu, const float *sd,
                                 int relu, float *pre, float *out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * dout) return;
    const int r = t / dout, o = t % dout;
    const int src = idx ? idx[r] : r;
    const float *x = in + (int64_t)src * din;
    float acc = b[o];
    for (int i = 0; i < din; ++i) {
        const float xi = mu ? (x[i] - mu[i]) / sd[i] : x[i];
        acc = fmaf(W[o * din + i], xi, acc);
    }
    if (pre) pre[(int64_t)r * dout + o] = acc;
    out[(int64_t)r * dout + o] = relu ? fmaxf(acc, 0.f) : acc;
}

// Inference: the three layers of the forward pass and the argmax for one row per
// block (H threads), with every output computed by the same operations in the same
// order as dense_fwd_kernel, so the class equals that of the layered forward pass.
constexpr int kInferMax = 256;  // widest layer the fused kernel holds in LDS
__global__ __launch_bounds__(kInferMax) void mlp_infer_kernel(MlpDims d, const float *params,
                                                              const float *X, int rows, int *cls) {
    const int r = blockIdx.x, t = threadIdx.x;
    if (r >= rows) return;
    __shared__ float h1[kInferMax], h2[kInferMax], z[kInferMax];
    const MlpOffsets o = mlp_offsets(d);
    const float *W1 = params + o.W1, *b1 = params + o.b1, *W2 = params + o.W2, *b2 = params + o.b2,
                *W3 = params + o.W3, *b3 = params + o.b3, *mu = params + o.mu, *sd = params + o.sd;
    const float *x = X + (int64_t)r * d.F;
    if (t < d.H) {
        float acc = b1[t];
        for (int i = 0; i < d.F; ++i) acc = fmaf(W1[t * d.F + i], (x[i] - mu[i]) / sd[i], acc);
        h1[t] = fmaxf(acc, 0.f);
    }
    __syncthreads();
    if (t < d.H) {
        float acc = b2[t];
        for (int i = 0; i < d.H; ++i) acc = fmaf(W2[t * d.H + i], h1[i], acc);
        h2[t] = fmaxf(acc, 0.f);
    }
    __syncthreads();
    if (t < d.C) {
        float acc = b3[t];
        for (int i = 0; i < d.H; ++i) acc = fmaf(W3[t * d.H + i], h2[i], acc);
        z[t] = acc;
    }
    __syncthreads();
    if (t == 0) {
        int best = 0;
        for (int c = 1; c < d.C; ++c)
            if (z[c] > z[best]) best = c;
        cls[r] = best;
    }
}

// standardised copy of the gathered batch (input of the first layer's weight gradient)
__global__ void standardize_kernel(const float *in, const int *idx, int rows, int din,
                                   const float *mu, const float *sd, float *out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * din) return;
    const int r = t / din, i = t % din;
    const int src = idx ? idx[r] : r;
    out[t] = (in[(int64_t)src * din + i] - mu[i]) / sd[i];
}

// dz = (softmax(z) - onehot(y)) / rows, loss_r = logsumexp(z) - z[y]
__global__ void softmax_ce_kernel(const float *z, const int *y, const int *idx, int rows, int C,
                                  float *dz, float *loss_r) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const float *zr = z + (int64_t)r * C;
    float mx = zr[0];
    for (int c = 1; c < C; ++c) mx = fmaxf(mx, zr[c]);
    float s = 0.f;
    for (int c = 0; c < C; ++c) s += expf(zr[c] - mx);
    const int yr = y[idx ? idx[r] : r];
    for (int c = 0; c < C; ++c) {
        const float p = expf(zr[c] - mx) / s;
        dz[(int64_t)r * C + c] = (p - (c == yr ? 1.f : 0.f)) / (float)rows;
    }
    loss_r[r] = (mx + logf(s)) - zr[yr];
}

// gW[o][i] = sum_r dout[r][o] in[r][i], gb[o] = sum_r dout[r][o] (rows in order)
__global__ void dense_bwd_w_kernel(const float *dout, const float *in, int rows, int din, int dimo,
                                   float *gW, float *gb) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < dimo * din) {
        const int o = t / din, i = t % din;
        float acc = 0.f;
        for (int r = 0; r < rows; ++r) acc = fmaf(dout[(int64_t)r * dimo + o], in[(int64_t)r * din + i], acc);
        gW[t] = acc;
    } else if (t < dimo * din + dimo) {
        const int o = t - dimo * din;
        float acc = 0.f;
        for (int r = 0; r < rows; ++r) acc += dout[(int64_t)r * dimo + o];
        gb[o] = acc;
    }
}

// din_grad[r][i] = (sum_o dout[r][o] W[o][i]) * [pre[r][i] > 0]
__global__ void dense_bwd_x_kernel(const float *dout, const float *W, const float *pre, int rows,
                                   int din, int dimo, float *dx) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * din) return;
    const int r = t / din, i = t % din;
    float acc = 0.f;
    for (int o = 0; o < dimo; ++o) acc = fmaf(dout[(int64_t)r * dimo + o], W[o * din + i], acc);
    dx[t] = pre[t] > 0.f ? acc : 0.f;
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int n, float lr, float b1,
                            float b2, float eps, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// one block: sum of the per-row losses in row order (thread 0), accumulated into *acc
__global__ void loss_sum_kernel(const float *loss_r, int rows, float *acc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += loss_r[r];
    *acc += s / (float)rows;
}

__global__ void fill_f32_kernel(float *p, int n, float v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void argmax_kernel(const float *z, int rows, int C, int *out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    int best = 0;
    for (int c = 1; c < C; ++c)
        if (z[(int64_t)r * C + c] > z[(int64_t)r * C + best]) best = c;
    out[r] = best;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_batch_feat_reduce(const FeatProblem *probs, int nprob, hipStream_t s) {
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_feat_reduce_kernel, dim3((unsigned)nprob), dim3(256), 0, s, probs);
    return hipGetLastError();
}

hipError_t launch_feat_reduce(const unsigned long long *s1a, const unsigned long long *s2a,
                              int64_t ra, const unsigned long long *s1b,
                              const unsigned long long *s2b, int64_t rb,
                              const unsigned long long *zeros,
                              int64_t m, int64_t n, int64_t k, float *out, hipStream_t s) {
    hipLaunchKernelGGL(feat_reduce_kernel, dim3(1), dim3(256), 0, s, s1a, s2a, ra, s1b, s2b, rb, zeros,
                       (double)m, (double)n, (double)k, out);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpDims &d, const float *params, const float *X, const int *idx,
                              int rows, MlpActs &a, hipStream_t s) {
    const MlpOffsets o = mlp_offsets(d);
    const float *W1 = params + o.W1, *b1 = params + o.b1, *W2 = params + o.W2, *b2 = params + o.b2,
                *W3 = params + o.W3, *b3 = params + o.b3, *mu = params + o.mu, *sd = params + o.sd;
    hipLaunchKernelGGL(dense_fwd_kernel, dim3(blocks_for((int64_t)rows * d.H)), dim3(256), 0, s, X, idx,
                       rows, d.F, d.H, W1, b1, mu, sd, 1, a.a1, a.h1);
    hipLaunchKernelGGL(dense_fwd_kernel, dim3(blocks_for((int64_t)rows * d.H)), dim3(256), 0, s, a.h1,
                       nullptr, rows, d.H, d.H, W2, b2, nullptr, nullptr, 1, a.a2, a.h2);
    hipLaunchKernelGGL(dense_fwd_kernel, dim3(blocks_for((int64_t)rows * d.C)), dim3(256), 0, s, a.h2,
                       nullptr, rows, d.H, d.C, W3, b3, nullptr, nullptr, 0, nullptr, a.z);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const MlpDims &d, const float *params, const float *X, int rows,
                            int *cls, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    if (d.H > kInferMax || d.C > kInferMax || d.F < 1) return hipErrorInvalidValue;
    const int threads = (d.H > d.C ? d.H : d.C) < 64 ? 64 : ((d.H > d.C ? d.H : d.C) + 63) / 64 * 64;
    hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)rows), dim3((unsigned)threads), 0, s, d, params, X,
                       rows, cls);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpDims &d, const float *params, const float *X, const int *y,
                           const int *idx, int rows, MlpActs &a, float *grad, float *loss_acc,
                           hipStream_t s) {
    hipError_t e = launch_mlp_forward(d, params, X, idx, rows, a, s);
    if (e != hipSuccess) return e;
    const MlpOffsets o = mlp_offsets(d);
    const float *W2 = params + o.W2, *W3 = params + o.W3, *mu = params + o.mu, *sd = params + o.sd;
    hipLaunchKernelGGL(softmax_ce_kernel, dim3(blocks_for(rows)), dim3(256), 0, s, a.z, y, idx, rows, d.C,
                       a.dz, a.loss_r);
    if (loss_acc) hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(64), 0, s, a.loss_r, rows, loss_acc);
    // layer 3
    hipLaunchKernelGGL(dense_bwd_w_kernel, dim3(blocks_for((int64_t)d.C * d.H + d.C)), dim3(256), 0, s,
                       a.dz, a.h2, rows, d.H, d.C, grad + o.W3, grad + o.b3);
    hipLaunchKernelGGL(dense_bwd_x_kernel, dim3(blocks_for((int64_t)rows * d.H)), dim3(256), 0, s, a.dz,
                       W3, a.a2, rows, d.H, d.C, a.d2);
    // layer 2
    hipLaunchKernelGGL(dense_bwd_w_kernel, dim3(blocks_for((int64_t)d.H * d.H + d.H)), dim3(256), 0, s,
                       a.d2, a.h1, rows, d.H, d.H, grad + o.W2, grad + o.b2);
    hipLaunchKernelGGL(dense_bwd_x_kernel, dim3(blocks_for((int64_t)rows * d.H)), dim3(256), 0, s, a.d2,
                       W2, a.a1, rows, d.H, d.H, a.d1);
    // layer 1 (input: the standardised features)
    hipLaunchKernelGGL(standardize_kernel, dim3(blocks_for((int64_t)rows * d.F)), dim3(256), 0, s, X, idx,
                       rows, d.F, mu, sd, a.xs);
    hipLaunchKernelGGL(dense_bwd_w_kernel, dim3(blocks_for((int64_t)d.H * d.F + d.H)), dim3(256), 0, s,
                       a.d1, a.xs, rows, d.F, d.H, grad + o.W1, grad + o.b1);
    hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks_for(2 * d.F)), dim3(256), 0, s, grad + o.mu, 2 * d.F,
                       0.f);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1,
                       float b2, float eps, int t, hipStream_t s) {
    const float bc1 = 1.f - powf(b1, (float)t), bc2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps,
                       bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_argmax(const float *z, int rows, int C, int *out, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(argmax_kernel, dim3(blocks_for(rows)), dim3(256), 0, s, z, rows, C, out);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, int n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace ozc
