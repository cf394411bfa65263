// Learned choice of the moduli count (include/ozc.h, "moduli-count predictor"):
// input statistics, the perceptron's buffers, its training loop, and the
// per-call prediction used when the handle is configured with N = 0.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "context.h"

namespace ozc {

constexpr MlpDims kDims{OZC_MLP_FEATURES, OZC_MLP_HIDDEN, OZC_MLP_CLASSES};

struct MlpState {
    float *params = nullptr;  // device, mlp_offsets(kDims).total floats
    float *m = nullptr, *v = nullptr, *grad = nullptr;
    float *loss_acc = nullptr;
    int *pred = nullptr;
    bool have_params = false;
    // activations, sized for `rows_cap` rows
    int rows_cap = 0;
    float *acts = nullptr;
    MlpActs a{};
    int *idx = nullptr;
    int idx_cap = 0;
    // statistics scratch for one operand pair
    int64_t stat_rows = 0;
    char *stat = nullptr;
    float *feat = nullptr;  // 1 x F
    int n_fix = 18;         // fallback moduli count
    int margin = 0;         // added to the predicted count
    char *many = nullptr;   // scratch of the many-product prediction
    size_t many_bytes = 0;
    // one product's predicted class, copied to pinned host memory and awaited through an
    // event, so that the stream keeps the work queued behind the copy
    int *cls_host = nullptr;
    hipEvent_t cls_ready = nullptr;

    void release() {
        for (void *p : {(void *)params, (void *)m, (void *)v, (void *)grad, (void *)loss_acc,
                        (void *)pred, (void *)acts, (void *)idx, (void *)stat, (void *)feat,
                        (void *)many})
            if (p) (void)hipFree(p);
        if (cls_host) (void)hipHostFree(cls_host);
        if (cls_ready) (void)hipEventDestroy(cls_ready);
    }
};

void mlp_release(ozc_context *h) {
    if (!h->mlp) return;
    h->mlp->release();
    delete h->mlp;
    h->mlp = nullptr;
}

namespace {

template <typename T>
hipError_t dev_alloc(T **p, size_t count) {
    *p = nullptr;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (count ? count : 1));
    if (e != hipSuccess) *p = nullptr;
    return e;
}

MlpState *mlp_state(ozc_context *h) {
    if (h->mlp) return h->mlp;
    MlpState *st = new (std::nothrow) MlpState();
    if (!st) return nullptr;
    const int P = mlp_offsets(kDims).total;
    if (dev_alloc(&st->params, P) != hipSuccess || dev_alloc(&st->m, P) != hipSuccess ||
        dev_alloc(&st->v, P) != hipSuccess || dev_alloc(&st->grad, P) != hipSuccess ||
        dev_alloc(&st->loss_acc, 1) != hipSuccess || dev_alloc(&st->pred, 1) != hipSuccess ||
        dev_alloc(&st->feat, kDims.F) != hipSuccess) {
        st->release();
        delete st;
        (void)hipGetLastError();
        return nullptr;
    }
    h->mlp = st;
    return st;
}

ozc_status_t ensure_acts(MlpState *st, int rows) {
    if (rows <= st->rows_cap) return OZC_STATUS_SUCCESS;
    if (st->acts) (void)hipFree(st->acts);
    st->acts = nullptr;
    st->rows_cap = 0;
    const size_t H = kDims.H, C = kDims.C, F = kDims.F, R = (size_t)rows;
    const size_t total = R * (6 * H + 2 * C + 1 + F);
    if (dev_alloc(&st->acts, total) != hipSuccess) {
        (void)hipGetLastError();
        return OZC_STATUS_ALLOC_FAILED;
    }
    float *p = st->acts;
    auto take = [&](size_t n) {
        float *q = p;
        p += n;
        return q;
    };
    st->a.a1 = take(R * H);
    st->a.h1 = take(R * H);
    st->a.a2 = take(R * H);
    st->a.h2 = take(R * H);
    st->a.d2 = take(R * H);
    st->a.d1 = take(R * H);
    st->a.z = take(R * C);
    st->a.dz = take(R * C);
    st->a.loss_r = take(R);
    st->a.xs = take(R * F);
    st->rows_cap = rows;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ensure_stats(MlpState *st, int64_t rows) {
    if (rows <= st->stat_rows) return OZC_STATUS_SUCCESS;
    if (st->stat) (void)hipFree(st->stat);
    st->stat = nullptr;
    st->stat_rows = 0;
    // per row: maxbits (8), sigma (8), tau (8); plus one zero counter
    if (dev_alloc(&st->stat, (size_t)rows * 24 + 256) != hipSuccess) {
        (void)hipGetLastError();
        return OZC_STATUS_ALLOC_FAILED;
    }
    st->stat_rows = rows;
    return OZC_STATUS_SUCCESS;
}

uint64_t splitmix64(uint64_t state, uint64_t i) {
    uint64_t z = state + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t seed, uint64_t i) { return (double)(splitmix64(seed, i) >> 11) * 0x1p-53; }

}  // namespace

// k of the statistics: a call above the INT32 limit runs in k-chunks (api.cpp), and
// its count is predicted from the first chunk (the relative error of the whole call is
// at most the largest of its chunks').
int64_t feature_k(int64_t k) {
    if (k <= OZC_MAX_K) return k;
    const int64_t nc = (k + OZC_MAX_K - 1) / OZC_MAX_K;
    return k / nc;
}

// Statistics of op(A) (m x k) and op(B) (k x n) into `out` (device, F floats): the
// scaling pass's row maxima and sums (sigma, with tau and the zero count), then the
// reduction.  The maxima and sigma stay in st->stat for the call that follows
// (PreStats: that call skips its own scaling statistics).
ozc_status_t compute_features(ozc_context *h, bool single, ozc_op_t ta, ozc_op_t tb, int64_t m,
                              int64_t n, int64_t k, const void *A, int64_t lda, const void *B,
                              int64_t ldb, float *out, PreStats *pre) {
    MlpState *st = mlp_state(h);
    if (!st) return OZC_STATUS_ALLOC_FAILED;
    ozc_status_t s = ensure_stats(st, m + n);
    if (s != OZC_STATUS_SUCCESS) return s;
    hipStream_t str = h->stream;
    const int64_t kf = feature_k(k);
    uint64_t *mb = (uint64_t *)st->stat;
    uint64_t *sig = (uint64_t *)(st->stat + 8 * (size_t)(m + n));
    uint64_t *tau = (uint64_t *)(st->stat + 16 * (size_t)(m + n));
    uint64_t *zeros = (uint64_t *)(st->stat + 24 * (size_t)(m + n));
    OZC_TRY(launch_fill_u64(mb, 3 * (m + n) + 1, 0, str));  // maxbits, sigma, tau, zeros
    const OperandView vA = view_A(A, ta, m, kf, lda), vB = view_B(B, tb, n, kf, ldb);
    OZC_TRY(launch_pair_scans(vA, vB, single, mb, mb + m, sig, sig + m, false, str));
    OZC_TRY(launch_pair_scans(vA, vB, single, mb, mb + m, sig, sig + m, true, str, tau, tau + m,
                              zeros));
    OZC_TRY(launch_feat_reduce((const unsigned long long *)tau, (const unsigned long long *)sig, m,
                               (const unsigned long long *)(tau + m),
                               (const unsigned long long *)(sig + m), n,
                               (const unsigned long long *)zeros, m, n, kf, out, str));
    if (pre) {
        *pre = PreStats{};
        if (kf == k) *pre = PreStats{mb, mb + m, sig, sig + m};
    }
    return OZC_STATUS_SUCCESS;
}

// Enqueues the prediction of N for one product.  *pending tells whether the count is
// still on its way (then predict_moduli_wait delivers it); otherwise *N is final (the
// fixed fallback count without parameters or for an empty product).  pre (may be
// null) receives the scaling statistics the prediction computes, for the call that
// follows.  Work the caller enqueues before the wait runs while the host waits.
ozc_status_t predict_moduli_begin(ozc_context *h, bool single, ozc_op_t ta, ozc_op_t tb,
                                  int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                                  const void *B, int64_t ldb, int *N, PreStats *pre, bool *pending) {
    *pending = false;
    if (pre) *pre = PreStats{};
    MlpState *st = mlp_state(h);
    if (!st) return OZC_STATUS_ALLOC_FAILED;
    if (!st->have_params || m == 0 || n == 0 || k == 0) {
        *N = st->n_fix;
        return OZC_STATUS_SUCCESS;
    }
    if (!st->cls_host) {
        if (hipHostMalloc((void **)&st->cls_host, sizeof(int) * 4, hipHostMallocDefault) != hipSuccess) {
            st->cls_host = nullptr;
            (void)hipGetLastError();
            return OZC_STATUS_ALLOC_FAILED;
        }
    }
    if (!st->cls_ready) OZC_TRY(hipEventCreateWithFlags(&st->cls_ready, hipEventDisableTiming));
    ozc_status_t s = compute_features(h, single, ta, tb, m, n, k, A, lda, B, ldb, st->feat, pre);
    if (s != OZC_STATUS_SUCCESS) return s;
    OZC_TRY(launch_mlp_infer(kDims, st->params, st->feat, 1, st->pred, h->stream));
    OZC_TRY(hipMemcpyAsync(st->cls_host, st->pred, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    OZC_TRY(hipEventRecord(st->cls_ready, h->stream));
    *pending = true;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t predict_moduli_wait(ozc_context *h, int *N) {
    MlpState *st = h->mlp;
    if (!st || !st->cls_ready || !st->cls_host) return OZC_STATUS_INVALID_VALUE;
    OZC_TRY(hipEventSynchronize(st->cls_ready));
    const int cls = *(volatile int *)st->cls_host;
    *N = std::min(OZC_MAX_MODULI, std::max(OZC_MIN_MODULI, OZC_MLP_MIN_N + cls + st->margin));
    return OZC_STATUS_SUCCESS;
}

// Predicted N for one product (waits for it).
ozc_status_t predict_moduli(ozc_context *h, bool single, ozc_op_t ta, ozc_op_t tb, int64_t m,
                            int64_t n, int64_t k, const void *A, int64_t lda, const void *B,
                            int64_t ldb, int *N, PreStats *pre) {
    bool pending = false;
    ozc_status_t s = predict_moduli_begin(h, single, ta, tb, m, n, k, A, lda, B, ldb, N, pre, &pending);
    if (s != OZC_STATUS_SUCCESS || !pending) return s;
    return predict_moduli_wait(h, N);
}

// Predicted N for many products at once: one statistics pass over all
// operands (batched launches), one forward pass, one synchronisation.
ozc_status_t predict_moduli_many(ozc_context *h, bool single, const std::vector<OperandView> &va,
                                 const std::vector<OperandView> &vb, std::vector<int> &N) {
    MlpState *st = mlp_state(h);
    if (!st) return OZC_STATUS_ALLOC_FAILED;
    const size_t P = va.size();
    N.assign(P, st->n_fix);
    if (!st->have_params || P == 0) return OZC_STATUS_SUCCESS;
    hipStream_t s = h->stream;
    int64_t rows = 0;
    for (size_t p = 0; p < P; ++p) rows += va[p].rows + vb[p].rows;
    // device scratch: maxbits, sigma, tau per row; zero counters; features; descriptors
    std::vector<BatchOperand> scan(2 * P);
    std::vector<FeatProblem> fprob(P);
    const size_t b_rows = align_up(24 * (size_t)rows), b_zero = align_up(8 * P),
                 b_feat = align_up(4 * P * kDims.F), b_scan = align_up(sizeof(BatchOperand) * 2 * P),
                 b_fprob = align_up(sizeof(FeatProblem) * P), b_pred = align_up(4 * P);
    const size_t total = b_rows + b_zero + b_feat + b_scan + b_fprob + b_pred;
    if (total > st->many_bytes) {
        OZC_TRY(hipStreamSynchronize(s));
        if (st->many) (void)hipFree(st->many);
        st->many = nullptr;
        st->many_bytes = 0;
        if (hipMalloc(&st->many, total) != hipSuccess) {
            st->many = nullptr;
            (void)hipGetLastError();
            return OZC_STATUS_ALLOC_FAILED;
        }
        st->many_bytes = total;
    }
    char *buf = st->many;
    uint64_t *mb = (uint64_t *)buf;
    uint64_t *sig = (uint64_t *)(buf + 8 * (size_t)rows);
    uint64_t *tau = (uint64_t *)(buf + 16 * (size_t)rows);
    uint64_t *zeros = (uint64_t *)(buf + b_rows);
    float *feat = (float *)(buf + b_rows + b_zero);
    char *d = buf + b_rows + b_zero + b_feat;
    BatchOperand *scan_dev = (BatchOperand *)d;
    FeatProblem *fprob_dev = (FeatProblem *)(d + b_scan);
    int *pred = (int *)(d + b_scan + b_fprob);
    int64_t r0 = 0, blk_scan = 0;
    for (size_t p = 0; p < P; ++p) {
        const OperandView *v2[2] = {&va[p], &vb[p]};
        const int64_t rbase[2] = {r0, r0 + va[p].rows};
        for (int q = 0; q < 2; ++q) {
            BatchOperand &b = scan[2 * p + q];
            b = BatchOperand{};
            b.v = *v2[q];
            b.maxbits = mb + rbase[q];
            b.sigma = sig + rbase[q];
            b.tau = tau + rbase[q];
            b.zeros = zeros + p;
            b.blk_scan = blk_scan;
            blk_scan += batch_scan_blocks(b.v);
        }
        FeatProblem &fp = fprob[p];
        fp.s1a = (const unsigned long long *)(tau + rbase[0]);
        fp.s2a = (const unsigned long long *)(sig + rbase[0]);
        fp.ra = va[p].rows;
        fp.s1b = (const unsigned long long *)(tau + rbase[1]);
        fp.s2b = (const unsigned long long *)(sig + rbase[1]);
        fp.rb = vb[p].rows;
        fp.zeros = (const unsigned long long *)(zeros + p);
        fp.m = (double)va[p].rows;
        fp.n = (double)vb[p].rows;
        fp.k = (double)va[p].k;
        fp.out = feat + p * kDims.F;
        r0 += va[p].rows + vb[p].rows;
    }
    OZC_TRY(hipMemcpyAsync(scan_dev, scan.data(), sizeof(BatchOperand) * 2 * P, hipMemcpyHostToDevice, s));
    OZC_TRY(hipMemcpyAsync(fprob_dev, fprob.data(), sizeof(FeatProblem) * P, hipMemcpyHostToDevice, s));
    OZC_TRY(launch_fill_u64(mb, 3 * rows, 0, s));
    OZC_TRY(launch_fill_u64(zeros, (int64_t)P, 0, s));
    OZC_TRY(launch_batch_scan(scan_dev, (int)(2 * P), blk_scan, single, 0, s));
    OZC_TRY(launch_batch_scan(scan_dev, (int)(2 * P), blk_scan, single, 2, s));
    OZC_TRY(launch_batch_feat_reduce(fprob_dev, (int)P, s));
    OZC_TRY(launch_mlp_infer(kDims, st->params, feat, (int)P, pred, s));
    std::vector<int> cls(P);
    OZC_TRY(hipMemcpyAsync(cls.data(), pred, sizeof(int) * P, hipMemcpyDeviceToHost, s));
    OZC_TRY(hipStreamSynchronize(s));
    for (size_t p = 0; p < P; ++p)
        N[p] = std::min(OZC_MAX_MODULI, std::max(OZC_MIN_MODULI, OZC_MLP_MIN_N + cls[p] + st->margin));
    return OZC_STATUS_SUCCESS;
}

}  // namespace ozc

using namespace ozc;

extern "C" {

ozc_status_t ozc_features(ozc_handle_t h, int single, ozc_op_t ta, ozc_op_t tb, int64_t m,
                          int64_t n, int64_t k, const void *A, int64_t lda, const void *B,
                          int64_t ldb, float *features) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    ozc_status_t s = check_args(ta, tb, m, n, k, A, lda, B, ldb, nullptr, m > 1 ? m : 1, true);
    if (s != OZC_STATUS_SUCCESS) return s;
    if (m == 0 || n == 0 || k == 0 || !features) return OZC_STATUS_INVALID_VALUE;
    OZC_TRY(hipSetDevice(h->device));
    return compute_features(h, single != 0, ta, tb, m, n, k, A, lda, B, ldb, features, nullptr);
}

ozc_status_t ozc_mlp_set_params(ozc_handle_t h, const float *params, int count) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (!params || count != mlp_offsets(kDims).total) return OZC_STATUS_INVALID_VALUE;
    const MlpOffsets o = mlp_offsets(kDims);
    for (int i = 0; i < kDims.F; ++i)
        if (!(params[o.sd + i] > 0.f)) return OZC_STATUS_INVALID_VALUE;
    OZC_TRY(hipSetDevice(h->device));
    MlpState *st = mlp_state(h);
    if (!st) return OZC_STATUS_ALLOC_FAILED;
    OZC_TRY(hipMemcpy(st->params, params, sizeof(float) * count, hipMemcpyHostToDevice));
    st->have_params = true;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_mlp_get_params(ozc_handle_t h, float *params, int count) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (!params || count != mlp_offsets(kDims).total) return OZC_STATUS_INVALID_VALUE;
    MlpState *st = mlp_state(h);
    if (!st) return OZC_STATUS_ALLOC_FAILED;
    if (!st->have_params) return OZC_STATUS_INVALID_VALUE;
    OZC_TRY(hipStreamSynchronize(h->stream));
    OZC_TRY(hipMemcpy(params, st->params, sizeof(float) * count, hipMemcpyDeviceToHost));
    return OZC_STATUS_SUCCESS;
}

namespace {
const char kMlpMagic[8] = {'O', 'Z', 'C', 'M', 'L', 'P', '0', '1'};

uint64_t fnv1a64(const void *data, size_t n) {
    const unsigned char *b = static_cast<const unsigned char *>(data);
    uint64_t x = 14695981039346656037ull;
    for (size_t i = 0; i < n; ++i) x = (x ^ b[i]) * 1099511628211ull;
    return x;
}
}  // namespace

ozc_status_t ozc_mlp_save(ozc_handle_t h, const char *path) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (!path) return OZC_STATUS_INVALID_VALUE;
    const int P = mlp_offsets(kDims).total;
    std::vector<float> p(P);
    ozc_status_t s = ozc_mlp_get_params(h, p.data(), P);
    if (s != OZC_STATUS_SUCCESS) return s;
    const int32_t dims[5] = {kDims.F, kDims.H, kDims.C, OZC_MLP_MIN_N, P};
    const uint64_t hash = fnv1a64(p.data(), sizeof(float) * P);
    FILE *f = fopen(path, "wb");
    if (!f) return OZC_STATUS_INVALID_VALUE;
    bool ok = fwrite(kMlpMagic, 1, 8, f) == 8 && fwrite(dims, sizeof(int32_t), 5, f) == 5 &&
              fwrite(p.data(), sizeof(float), P, f) == (size_t)P &&
              fwrite(&hash, sizeof(hash), 1, f) == 1;
    ok = (fclose(f) == 0) && ok;
    return ok ? OZC_STATUS_SUCCESS : OZC_STATUS_INVALID_VALUE;
}

ozc_status_t ozc_mlp_load(ozc_handle_t h, const char *path) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (!path) return OZC_STATUS_INVALID_VALUE;
    const int P = mlp_offsets(kDims).total;
    FILE *f = fopen(path, "rb");
    if (!f) return OZC_STATUS_INVALID_VALUE;
    char magic[8];
    int32_t dims[5];
    std::vector<float> p(P);
    uint64_t hash = 0;
    char extra;
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMlpMagic, 8) == 0 &&
              fread(dims, sizeof(int32_t), 5, f) == 5 && dims[0] == kDims.F &&
              dims[1] == kDims.H && dims[2] == kDims.C && dims[3] == OZC_MLP_MIN_N &&
              dims[4] == P && fread(p.data(), sizeof(float), P, f) == (size_t)P &&
              fread(&hash, sizeof(hash), 1, f) == 1 && fread(&extra, 1, 1, f) == 0;
    fclose(f);
    if (!ok || hash != fnv1a64(p.data(), sizeof(float) * P)) return OZC_STATUS_INVALID_VALUE;
    return ozc_mlp_set_params(h, p.data(), P);  // checks sd > 0 before replacing anything
}

ozc_status_t ozc_mlp_forward(ozc_handle_t h, const float *X, int rows, float *logits) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (rows < 0 || (rows > 0 && (!X || !logits))) return OZC_STATUS_INVALID_VALUE;
    MlpState *st = mlp_state(h);
    if (!st) return OZC_STATUS_ALLOC_FAILED;
    if (!st->have_params) return OZC_STATUS_INVALID_VALUE;
    if (rows == 0) return OZC_STATUS_SUCCESS;
    OZC_TRY(hipSetDevice(h->device));
    ozc_status_t s = ensure_acts(st, rows);
    if (s != OZC_STATUS_SUCCESS) return s;
    MlpActs a = st->a;
    a.z = logits;
    OZC_TRY(launch_mlp_forward(kDims, st->params, X, nullptr, rows, a, h->stream));
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_mlp_predict(ozc_handle_t h, const float *X, int rows, int *classes) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (rows < 0 || (rows > 0 && (!X || !classes))) return OZC_STATUS_INVALID_VALUE;
    MlpState *st = mlp_state(h);
    if (!st) return OZC_STATUS_ALLOC_FAILED;
    if (!st->have_params) return OZC_STATUS_INVALID_VALUE;
    if (rows == 0) return OZC_STATUS_SUCCESS;
    OZC_TRY(hipSetDevice(h->device));
    OZC_TRY(launch_mlp_infer(kDims, st->params, X, rows, classes, h->stream));
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_mlp_grad(ozc_handle_t h, const float *X, const int *y, int rows, float *grad,
                          float *loss) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (rows <= 0 || !X || !y || !grad) return OZC_STATUS_INVALID_VALUE;
    MlpState *st = mlp_state(h);
    if (!st) return OZC_STATUS_ALLOC_FAILED;
    if (!st->have_params) return OZC_STATUS_INVALID_VALUE;
    OZC_TRY(hipSetDevice(h->device));
    ozc_status_t s = ensure_acts(st, rows);
    if (s != OZC_STATUS_SUCCESS) return s;
    OZC_TRY(launch_fill_f32(st->loss_acc, 1, 0.f, h->stream));
    OZC_TRY(launch_mlp_grad(kDims, st->params, X, y, nullptr, rows, st->a, grad, st->loss_acc,
                            h->stream));
    if (loss) {
        OZC_TRY(hipMemcpyAsync(loss, st->loss_acc, sizeof(float), hipMemcpyDeviceToHost, h->stream));
        OZC_TRY(hipStreamSynchronize(h->stream));
    }
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_mlp_train(ozc_handle_t h, const float *X, const int *y, int rows, int epochs,
                           int batch, float lr, uint64_t seed, int init, float *epoch_loss) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (rows <= 0 || epochs < 0 || batch <= 0 || !(lr > 0.f) || !X || !y)
        return OZC_STATUS_INVALID_VALUE;
    OZC_TRY(hipSetDevice(h->device));
    MlpState *st = mlp_state(h);
    if (!st) return OZC_STATUS_ALLOC_FAILED;
    const MlpOffsets o = mlp_offsets(kDims);
    hipStream_t s = h->stream;
    if (init || !st->have_params) {
        // standardisation from the data, He-uniform weights, zero biases
        std::vector<float> hx((size_t)rows * kDims.F);
        OZC_TRY(hipStreamSynchronize(s));
        OZC_TRY(hipMemcpy(hx.data(), X, hx.size() * sizeof(float), hipMemcpyDeviceToHost));
        std::vector<float> p((size_t)o.total, 0.f);
        for (int f = 0; f < kDims.F; ++f) {
            double mean = 0.0, sq = 0.0;
            for (int r = 0; r < rows; ++r) mean += hx[(size_t)r * kDims.F + f];
            mean /= rows;
            for (int r = 0; r < rows; ++r) {
                const double d = hx[(size_t)r * kDims.F + f] - mean;
                sq += d * d;
            }
            const double sd = sqrt(sq / rows);
            p[(size_t)o.mu + f] = (float)mean;
            p[(size_t)o.sd + f] = (float)(sd > 1e-6 ? sd : 1.0);
        }
        uint64_t ctr = 0;
        auto fill = [&](int off, int fan_in, int count) {
            const double lim = sqrt(6.0 / fan_in);
            for (int i = 0; i < count; ++i) p[(size_t)off + i] = (float)((2.0 * uniform01(seed, ctr++) - 1.0) * lim);
        };
        fill(o.W1, kDims.F, kDims.H * kDims.F);
        fill(o.W2, kDims.H, kDims.H * kDims.H);
        fill(o.W3, kDims.H, kDims.C * kDims.H);
        OZC_TRY(hipMemcpy(st->params, p.data(), sizeof(float) * o.total, hipMemcpyHostToDevice));
        st->have_params = true;
    }
    OZC_TRY(launch_fill_f32(st->m, o.total, 0.f, s));
    OZC_TRY(launch_fill_f32(st->v, o.total, 0.f, s));
    const int B = std::min(batch, rows);
    ozc_status_t r = ensure_acts(st, B);
    if (r != OZC_STATUS_SUCCESS) return r;
    if (rows > st->idx_cap) {
        if (st->idx) (void)hipFree(st->idx);
        st->idx = nullptr;
        st->idx_cap = 0;
        if (dev_alloc(&st->idx, (size_t)rows) != hipSuccess) {
            (void)hipGetLastError();
            return OZC_STATUS_ALLOC_FAILED;
        }
        st->idx_cap = rows;
    }
    std::vector<int> perm((size_t)rows);
    const int steps = (rows + B - 1) / B;
    int t = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int i = 0; i < rows; ++i) perm[(size_t)i] = i;
        if (B < rows)  // Fisher-Yates with SplitMix64 draws; a full batch keeps the row order
            for (int i = rows - 1; i > 0; --i) {
                const int j = (int)(splitmix64(seed ^ 0xA5A5A5A5ull, (uint64_t)ep * rows + i) % (uint64_t)(i + 1));
                std::swap(perm[(size_t)i], perm[(size_t)j]);
            }
        OZC_TRY(hipStreamSynchronize(s));  // perm is read by the copy below
        OZC_TRY(hipMemcpy(st->idx, perm.data(), sizeof(int) * rows, hipMemcpyHostToDevice));
        OZC_TRY(launch_fill_f32(st->loss_acc, 1, 0.f, s));
        for (int b = 0; b < steps; ++b) {
            const int r0 = b * B, nb = std::min(B, rows - r0);
            OZC_TRY(launch_mlp_grad(kDims, st->params, X, y, st->idx + r0, nb, st->a, st->grad,
                                    st->loss_acc, s));
            OZC_TRY(launch_adam(st->params, st->grad, st->m, st->v, o.trainable, lr, 0.9f, 0.999f,
                                1e-8f, ++t, s));
        }
        if (epoch_loss) {
            float acc = 0.f;
            OZC_TRY(hipMemcpyAsync(&acc, st->loss_acc, sizeof(float), hipMemcpyDeviceToHost, s));
            OZC_TRY(hipStreamSynchronize(s));
            epoch_loss[ep] = acc / (float)steps;
        }
    }
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_set_auto_moduli(ozc_handle_t h, int fallback, int margin) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (fallback < OZC_MIN_MODULI || fallback > OZC_MAX_MODULI || margin < 0 || margin > 8)
        return OZC_STATUS_INVALID_VALUE;
    OZC_TRY(hipSetDevice(h->device));
    MlpState *st = mlp_state(h);
    if (!st) return OZC_STATUS_ALLOC_FAILED;
    st->n_fix = fallback;
    st->margin = margin;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_predict_moduli(ozc_handle_t h, int single, ozc_op_t ta, ozc_op_t tb, int64_t m,
                                int64_t n, int64_t k, const void *A, int64_t lda, const void *B,
                                int64_t ldb, int *num_moduli) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (!num_moduli) return OZC_STATUS_INVALID_VALUE;
    ozc_status_t s = check_args(ta, tb, m, n, k, A, lda, B, ldb, nullptr, m > 1 ? m : 1, true);
    if (s != OZC_STATUS_SUCCESS) return s;
    OZC_TRY(hipSetDevice(h->device));
    return predict_moduli(h, single != 0, ta, tb, m, n, k, A, lda, B, ldb, num_moduli, nullptr);
}

}  // extern "C"
