// Drop-in redirection of hipBLAS GEMM calls to the emulation (Section III-D: the
// paper's library is activated through LD_PRELOAD and then serves the
// single-, double-, complex- and double-complex GEMM entry points of the vendor
// BLAS).  Loaded before libhipblas, this library defines
//   hipblasSgemm, hipblasDgemm, hipblasCgemm, hipblasZgemm (and their _64 forms)
//   hipblasGemmEx, hipblasGemmEx_64
// and serves them with ozc_sgemm / ozc_dgemm / ozc_cgemm / ozc_zgemm on the
// hipBLAS handle's stream.  hipblasGemmEx is emulated when A, B and C share one
// of the four types above and the compute type is that precision (or its
// "fast" variant); every other combination goes on to the vendor routine.
//
// Scalars follow the handle's pointer mode (device scalars are copied to the
// host on the handle's stream first).  One emulation handle per device and
// host thread.  Settings, read once per process from the environment:
//   OZC_BLAS_DOUBLE_MODULI  moduli for Dgemm / Zgemm (default 14)
//   OZC_BLAS_SINGLE_MODULI  moduli for Sgemm / Cgemm (default 8)
//   OZC_BLAS_MODE           fast | accurate (default fast)
//   OZC_BLAS_ALGO           karatsuba | 4m (default karatsuba)
//   OZC_BLAS_TRACE          1: one line per redirected call on stderr
#include <dlfcn.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>

#include <hip/hip_runtime.h>
#include <hipblas/hipblas.h>

#include "../../include/ozc.h"

namespace {

struct Settings {
    int nd = 14, ns = 8;
    ozc_mode_t mode = OZC_MODE_FAST;
    ozc_algo_t algo = OZC_ALGO_KARATSUBA;
    bool trace = false;
};

int env_int(const char *name, int dflt, int lo, int hi) {
    const char *v = getenv(name);
    if (!v || !*v) return dflt;
    const int x = atoi(v);
    return x >= lo && x <= hi ? x : dflt;
}

const Settings &settings() {
    static const Settings s = [] {
        Settings t;
        t.nd = env_int("OZC_BLAS_DOUBLE_MODULI", 14, OZC_MIN_MODULI, OZC_MAX_MODULI);
        t.ns = env_int("OZC_BLAS_SINGLE_MODULI", 8, OZC_MIN_MODULI, OZC_MAX_MODULI);
        const char *m = getenv("OZC_BLAS_MODE");
        if (m && strcmp(m, "accurate") == 0) t.mode = OZC_MODE_ACCURATE;
        const char *a = getenv("OZC_BLAS_ALGO");
        if (a && strcmp(a, "4m") == 0) t.algo = OZC_ALGO_4M;
        t.trace = env_int("OZC_BLAS_TRACE", 0, 0, 1) == 1;
        return t;
    }();
    return s;
}

// The emulation handle of the current device on this thread (created on first use and
// kept for the thread's lifetime).
ozc_handle_t handle_for_device() {
    thread_local std::map<int, ozc_handle_t> handles;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    auto it = handles.find(dev);
    if (it != handles.end()) return it->second;
    ozc_handle_t h = nullptr;
    if (ozc_create(&h, dev) != OZC_STATUS_SUCCESS) return nullptr;
    handles[dev] = h;
    return h;
}

hipblasStatus_t to_blas(ozc_status_t s) {
    switch (s) {
        case OZC_STATUS_SUCCESS:
        case OZC_STATUS_NONFINITE: return HIPBLAS_STATUS_SUCCESS;
        case OZC_STATUS_INVALID_VALUE: return HIPBLAS_STATUS_INVALID_VALUE;
        case OZC_STATUS_ALLOC_FAILED: return HIPBLAS_STATUS_ALLOC_FAILED;
        case OZC_STATUS_NOT_SUPPORTED: return HIPBLAS_STATUS_NOT_SUPPORTED;
        case OZC_STATUS_INVALID_HANDLE: return HIPBLAS_STATUS_NOT_INITIALIZED;
        default: return HIPBLAS_STATUS_EXECUTION_FAILED;
    }
}

bool to_op(hipblasOperation_t t, ozc_op_t *op) {
    switch (t) {
        case HIPBLAS_OP_N: *op = OZC_OP_N; return true;
        case HIPBLAS_OP_T: *op = OZC_OP_T; return true;
        case HIPBLAS_OP_C: *op = OZC_OP_C; return true;
        default: return false;
    }
}

enum Kind { kZ, kC, kD, kS };

// alpha, beta (bytes each) on the host, following the handle's pointer mode.
hipblasStatus_t host_scalars(hipblasHandle_t bh, hipStream_t stream, const void *alpha,
                             const void *beta, size_t bytes, void *ha, void *hb) {
    if (!alpha || !beta) return HIPBLAS_STATUS_INVALID_VALUE;
    hipblasPointerMode_t pm = HIPBLAS_POINTER_MODE_HOST;
    if (hipblasGetPointerMode(bh, &pm) != HIPBLAS_STATUS_SUCCESS) return HIPBLAS_STATUS_NOT_INITIALIZED;
    if (pm == HIPBLAS_POINTER_MODE_HOST) {
        memcpy(ha, alpha, bytes);
        memcpy(hb, beta, bytes);
        return HIPBLAS_STATUS_SUCCESS;
    }
    if (hipMemcpyAsync(ha, alpha, bytes, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(hb, beta, bytes, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return HIPBLAS_STATUS_EXECUTION_FAILED;
    return HIPBLAS_STATUS_SUCCESS;
}

const char *kind_name(Kind k) {
    return k == kZ ? "zgemm" : k == kC ? "cgemm" : k == kD ? "dgemm" : "sgemm";
}

hipblasStatus_t emulate(Kind kind, hipblasHandle_t bh, hipblasOperation_t transa,
                        hipblasOperation_t transb, int64_t m, int64_t n, int64_t k,
                        const void *alpha, const void *A, int64_t lda, const void *B, int64_t ldb,
                        const void *beta, void *C, int64_t ldc) {
    if (!bh) return HIPBLAS_STATUS_NOT_INITIALIZED;
    ozc_op_t ta, tb;
    if (!to_op(transa, &ta) || !to_op(transb, &tb)) return HIPBLAS_STATUS_INVALID_ENUM;
    hipStream_t stream = nullptr;
    if (hipblasGetStream(bh, &stream) != HIPBLAS_STATUS_SUCCESS) return HIPBLAS_STATUS_NOT_INITIALIZED;
    const Settings &cfg = settings();
    ozc_handle_t h = handle_for_device();
    if (!h) return HIPBLAS_STATUS_ALLOC_FAILED;
    const bool dbl = kind == kZ || kind == kD;
    ozc_status_t st = ozc_set_config(h, dbl ? cfg.nd : cfg.ns, cfg.mode, cfg.algo);
    if (st == OZC_STATUS_SUCCESS) st = ozc_set_stream(h, stream);
    if (st != OZC_STATUS_SUCCESS) return to_blas(st);
    if (cfg.trace)
        fprintf(stderr, "ozc-blas: %s %lld x %lld x %lld, %d moduli\n", kind_name(kind),
                (long long)m, (long long)n, (long long)k, dbl ? cfg.nd : cfg.ns);
    const size_t sb = kind == kZ ? 16 : (kind == kS ? 4 : 8);
    alignas(16) unsigned char ha[16], hb[16];
    const hipblasStatus_t bs = host_scalars(bh, stream, alpha, beta, sb, ha, hb);
    if (bs != HIPBLAS_STATUS_SUCCESS) return bs;
    switch (kind) {
        case kZ:
            st = ozc_zgemm(h, ta, tb, m, n, k, (const double *)ha, A, lda, B, ldb,
                           (const double *)hb, C, ldc);
            break;
        case kC:
            st = ozc_cgemm(h, ta, tb, m, n, k, (const float *)ha, A, lda, B, ldb,
                           (const float *)hb, C, ldc);
            break;
        case kD:
            st = ozc_dgemm(h, ta, tb, m, n, k, (const double *)ha, A, lda, B, ldb,
                           (const double *)hb, C, ldc);
            break;
        case kS:
            st = ozc_sgemm(h, ta, tb, m, n, k, (const float *)ha, A, lda, B, ldb,
                           (const float *)hb, C, ldc);
            break;
    }
    return to_blas(st);
}

// The type handled by the emulation for a GemmEx call, or -1 (vendor routine).
int ex_kind(hipDataType a, hipDataType b, hipDataType c, hipblasComputeType_t ct) {
    if (a != b || a != c) return -1;
    switch (a) {
        case HIP_C_64F: return ct == HIPBLAS_COMPUTE_64F || ct == HIPBLAS_COMPUTE_64F_PEDANTIC ? kZ : -1;
        case HIP_R_64F: return ct == HIPBLAS_COMPUTE_64F || ct == HIPBLAS_COMPUTE_64F_PEDANTIC ? kD : -1;
        case HIP_C_32F: return ct == HIPBLAS_COMPUTE_32F || ct == HIPBLAS_COMPUTE_32F_PEDANTIC ? kC : -1;
        case HIP_R_32F: return ct == HIPBLAS_COMPUTE_32F || ct == HIPBLAS_COMPUTE_32F_PEDANTIC ? kS : -1;
        default: return -1;
    }
}

template <typename F>
F next_symbol(const char *name) {
    return reinterpret_cast<F>(dlsym(RTLD_NEXT, name));
}

}  // namespace

extern "C" {

#define OZC_BLAS_GEMM(NAME, IDX, KIND, T)                                                       \
    hipblasStatus_t NAME(hipblasHandle_t handle, hipblasOperation_t transA,                     \
                         hipblasOperation_t transB, IDX m, IDX n, IDX k, const T *alpha,        \
                         const T *A, IDX lda, const T *B, IDX ldb, const T *beta, T *C, IDX ldc) { \
        return emulate(KIND, handle, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C,    \
                       ldc);                                                                    \
    }

OZC_BLAS_GEMM(hipblasSgemm, int, kS, float)
OZC_BLAS_GEMM(hipblasDgemm, int, kD, double)
OZC_BLAS_GEMM(hipblasCgemm, int, kC, hipComplex)
OZC_BLAS_GEMM(hipblasZgemm, int, kZ, hipDoubleComplex)
OZC_BLAS_GEMM(hipblasSgemm_64, int64_t, kS, float)
OZC_BLAS_GEMM(hipblasDgemm_64, int64_t, kD, double)
OZC_BLAS_GEMM(hipblasCgemm_64, int64_t, kC, hipComplex)
OZC_BLAS_GEMM(hipblasZgemm_64, int64_t, kZ, hipDoubleComplex)
#undef OZC_BLAS_GEMM

hipblasStatus_t hipblasGemmEx(hipblasHandle_t handle, hipblasOperation_t transA,
                              hipblasOperation_t transB, int m, int n, int k, const void *alpha,
                              const void *A, hipDataType aType, int lda, const void *B,
                              hipDataType bType, int ldb, const void *beta, void *C,
                              hipDataType cType, int ldc, hipblasComputeType_t computeType,
                              hipblasGemmAlgo_t algo) {
    const int kind = ex_kind(aType, bType, cType, computeType);
    if (kind >= 0)
        return emulate((Kind)kind, handle, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta,
                       C, ldc);
    using Fn = hipblasStatus_t (*)(hipblasHandle_t, hipblasOperation_t, hipblasOperation_t, int,
                                   int, int, const void *, const void *, hipDataType, int,
                                   const void *, hipDataType, int, const void *, void *,
                                   hipDataType, int, hipblasComputeType_t, hipblasGemmAlgo_t);
    static Fn vendor = next_symbol<Fn>("hipblasGemmEx");
    if (!vendor) return HIPBLAS_STATUS_NOT_SUPPORTED;
    return vendor(handle, transA, transB, m, n, k, alpha, A, aType, lda, B, bType, ldb, beta, C,
                  cType, ldc, computeType, algo);
}

hipblasStatus_t hipblasGemmEx_64(hipblasHandle_t handle, hipblasOperation_t transA,
                                 hipblasOperation_t transB, int64_t m, int64_t n, int64_t k,
                                 const void *alpha, const void *A, hipDataType aType, int64_t lda,
                                 const void *B, hipDataType bType, int64_t ldb, const void *beta,
                                 void *C, hipDataType cType, int64_t ldc,
                                 hipblasComputeType_t computeType, hipblasGemmAlgo_t algo) {
    const int kind = ex_kind(aType, bType, cType, computeType);
    if (kind >= 0)
        return emulate((Kind)kind, handle, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta,
                       C, ldc);
    using Fn = hipblasStatus_t (*)(hipblasHandle_t, hipblasOperation_t, hipblasOperation_t,
                                   int64_t, int64_t, int64_t, const void *, const void *,
                                   hipDataType, int64_t, const void *, hipDataType, int64_t,
                                   const void *, void *, hipDataType, int64_t,
                                   hipblasComputeType_t, hipblasGemmAlgo_t);
    static Fn vendor = next_symbol<Fn>("hipblasGemmEx_64");
    if (!vendor) return HIPBLAS_STATUS_NOT_SUPPORTED;
    return vendor(handle, transA, transB, m, n, k, alpha, A, aType, lda, B, bType, ldb, beta, C,
                  cType, ldc, computeType, algo);
}

}  // extern "C"
