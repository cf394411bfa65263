// Test client of the hipBLAS redirection: an ordinary hipBLAS program (linked to the
// vendor libhipblas) that runs one GEMM on matrices read from files and writes C back.
// Run under LD_PRELOAD of libozc_blas.so, its GEMM calls are served by the emulation.
//
// usage: blas_client KIND API PTRMODE m n k transA transB ar ai br bi lda ldb ldc A B C OUT
//   KIND z | c | d | s; API typed (hipblasXgemm) | ex (hipblasGemmEx) | ex16 (KIND s
//   only: hipblasGemmEx on A, B rounded to half precision with float C and compute type,
//   a combination the emulation leaves to the vendor);
//   PTRMODE host | device; trans N | T | C; A, B, C: files holding the raw column-major
//   element arrays (leading dimensions lda, ldb, ldc); OUT receives C in the same layout.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <hipblas/hipblas.h>

static std::vector<char> read_file(const char *path) {
    std::vector<char> d;
    FILE *f = fopen(path, "rb");
    if (!f) return d;
    fseek(f, 0, SEEK_END);
    long sz = ftell(f);
    fseek(f, 0, SEEK_SET);
    d.resize((size_t)sz);
    if (sz > 0 && fread(d.data(), 1, (size_t)sz, f) != (size_t)sz) d.clear();
    fclose(f);
    return d;
}

static hipblasOperation_t op_of(const char *s) {
    return s[0] == 'T' ? HIPBLAS_OP_T : (s[0] == 'C' ? HIPBLAS_OP_C : HIPBLAS_OP_N);
}

#define CHECK(x)                                                                 \
    do {                                                                         \
        if (!(x)) {                                                              \
            fprintf(stderr, "blas_client: %s failed (line %d)\n", #x, __LINE__); \
            return 1;                                                            \
        }                                                                        \
    } while (0)

int main(int argc, char **argv) {
    if (argc != 20) {
        fprintf(stderr, "blas_client: expected 19 arguments, got %d\n", argc - 1);
        return 2;
    }
    const char kind = argv[1][0];
    const char *api = argv[2];
    const bool dev_ptr = strcmp(argv[3], "device") == 0;
    const int m = atoi(argv[4]), n = atoi(argv[5]), k = atoi(argv[6]);
    const hipblasOperation_t ta = op_of(argv[7]), tb = op_of(argv[8]);
    const double ar = atof(argv[9]), ai = atof(argv[10]), br = atof(argv[11]), bi = atof(argv[12]);
    const int lda = atoi(argv[13]), ldb = atoi(argv[14]), ldc = atoi(argv[15]);
    std::vector<char> hA = read_file(argv[16]), hB = read_file(argv[17]), hC = read_file(argv[18]);
    CHECK(!hA.empty() && !hB.empty() && !hC.empty());
    const size_t es = kind == 'z' ? 16 : (kind == 's' ? 4 : 8);
    const bool half_in = strcmp(api, "ex16") == 0;
    CHECK(!half_in || kind == 's');
    if (half_in) {  // A, B as half-precision elements
        for (std::vector<char> *v : {&hA, &hB}) {
            const size_t cnt = v->size() / 4;
            std::vector<char> h16(cnt * 2);
            for (size_t i = 0; i < cnt; ++i) {
                float x;
                memcpy(&x, v->data() + 4 * i, 4);
                const __half y = __float2half(x);
                memcpy(h16.data() + 2 * i, &y, 2);
            }
            v->swap(h16);
        }
    }
    void *dA = nullptr, *dB = nullptr, *dC = nullptr, *dS = nullptr;
    CHECK(hipMalloc(&dA, hA.size()) == hipSuccess);
    CHECK(hipMalloc(&dB, hB.size()) == hipSuccess);
    CHECK(hipMalloc(&dC, hC.size()) == hipSuccess);
    CHECK(hipMalloc(&dS, 64) == hipSuccess);
    CHECK(hipMemcpy(dA, hA.data(), hA.size(), hipMemcpyHostToDevice) == hipSuccess);
    CHECK(hipMemcpy(dB, hB.data(), hB.size(), hipMemcpyHostToDevice) == hipSuccess);
    CHECK(hipMemcpy(dC, hC.data(), hC.size(), hipMemcpyHostToDevice) == hipSuccess);

    // scalars in the element type, on the host or the device
    alignas(16) unsigned char sa[16] = {}, sb[16] = {};
    if (kind == 'z' || kind == 'd') {
        double a[2] = {ar, ai}, b[2] = {br, bi};
        memcpy(sa, a, es);
        memcpy(sb, b, es);
    } else {
        float a[2] = {(float)ar, (float)ai}, b[2] = {(float)br, (float)bi};
        memcpy(sa, a, es);
        memcpy(sb, b, es);
    }
    hipblasHandle_t h;
    CHECK(hipblasCreate(&h) == HIPBLAS_STATUS_SUCCESS);
    hipStream_t stream;
    CHECK(hipStreamCreate(&stream) == hipSuccess);
    CHECK(hipblasSetStream(h, stream) == HIPBLAS_STATUS_SUCCESS);
    const void *alpha = sa, *beta = sb;
    if (dev_ptr) {
        CHECK(hipMemcpy(dS, sa, 16, hipMemcpyHostToDevice) == hipSuccess);
        CHECK(hipMemcpy((char *)dS + 16, sb, 16, hipMemcpyHostToDevice) == hipSuccess);
        CHECK(hipblasSetPointerMode(h, HIPBLAS_POINTER_MODE_DEVICE) == HIPBLAS_STATUS_SUCCESS);
        alpha = dS;
        beta = (char *)dS + 16;
    }
    hipblasStatus_t st;
    if (strcmp(api, "typed") == 0) {
        switch (kind) {
            case 'z':
                st = hipblasZgemm(h, ta, tb, m, n, k, (const hipDoubleComplex *)alpha,
                                  (const hipDoubleComplex *)dA, lda, (const hipDoubleComplex *)dB, ldb,
                                  (const hipDoubleComplex *)beta, (hipDoubleComplex *)dC, ldc);
                break;
            case 'c':
                st = hipblasCgemm(h, ta, tb, m, n, k, (const hipComplex *)alpha, (const hipComplex *)dA,
                                  lda, (const hipComplex *)dB, ldb, (const hipComplex *)beta,
                                  (hipComplex *)dC, ldc);
                break;
            case 'd':
                st = hipblasDgemm(h, ta, tb, m, n, k, (const double *)alpha, (const double *)dA, lda,
                                  (const double *)dB, ldb, (const double *)beta, (double *)dC, ldc);
                break;
            default:
                st = hipblasSgemm(h, ta, tb, m, n, k, (const float *)alpha, (const float *)dA, lda,
                                  (const float *)dB, ldb, (const float *)beta, (float *)dC, ldc);
                break;
        }
    } else {
        const hipDataType t = kind == 'z' ? HIP_C_64F : kind == 'c' ? HIP_C_32F : kind == 'd' ? HIP_R_64F : HIP_R_32F;
        const hipDataType tab = half_in ? HIP_R_16F : t;
        const hipblasComputeType_t ct = (kind == 'z' || kind == 'd') ? HIPBLAS_COMPUTE_64F : HIPBLAS_COMPUTE_32F;
        st = hipblasGemmEx(h, ta, tb, m, n, k, alpha, dA, tab, lda, dB, tab, ldb, beta, dC, t, ldc,
                           ct, HIPBLAS_GEMM_DEFAULT);
    }
    if (st != HIPBLAS_STATUS_SUCCESS) {
        fprintf(stderr, "blas_client: gemm returned status %d\n", (int)st);
        return 3;
    }
    CHECK(hipStreamSynchronize(stream) == hipSuccess);
    CHECK(hipMemcpy(hC.data(), dC, hC.size(), hipMemcpyDeviceToHost) == hipSuccess);
    FILE *f = fopen(argv[19], "wb");
    CHECK(f != nullptr);
    const size_t wrote = fwrite(hC.data(), 1, hC.size(), f);
    fclose(f);
    CHECK(wrote == hC.size());
    CHECK(hipblasDestroy(h) == HIPBLAS_STATUS_SUCCESS);
    return 0;
}
