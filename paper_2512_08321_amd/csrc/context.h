// Handle state shared by the host runtime files (api.cpp, batched.cpp).
#pragma once

#include <array>
#include <vector>

#include "../../include/ozc.h"
#include "internal.h"

namespace ozc {
struct BatchState;  // batched-call plans and tuning (batched.cpp)
struct MlpState;    // moduli-count predictor (autoN.cpp)
// Scaling statistics a call may take over instead of computing them (row maxima and
// fast-mode sums of squares of op(A) and op(B), the layout of the workspace's own).
struct PreStats {
    const uint64_t *maxA = nullptr, *maxB = nullptr, *sigA = nullptr, *sigB = nullptr;
};
}

struct ozc_context {
    int device = 0;
    hipStream_t stream = nullptr;
    int nmod = 14;
    ozc_mode_t mode = OZC_MODE_FAST;
    ozc_algo_t algo = OZC_ALGO_KARATSUBA;
    void *ws_own = nullptr;
    size_t ws_own_bytes = 0;
    void *ws_user = nullptr;
    size_t ws_user_bytes = 0;
    void *ws_fixed = nullptr;           // this device's fixed workspace array (ozc_zgemm_noalloc)
    bool use_fixed = false;             // set only while ozc_zgemm_noalloc runs
    ozc::NTable *tab_dev = nullptr;          // kMaxModuli tables, index N - 1
    std::vector<ozc::NTable> tab_host;
    uint64_t *status_dev = nullptr;     // bit 0: non-finite input met
    bool keep_status = false;           // k-chunks after the first: keep the flag of earlier chunks
    ozc::PreStats pre{};                // statistics of the predicted-N call in progress (or none)
    void *dd_lo = nullptr;              // set only while ozc_zgemm_dd runs: the low parts
    ozc_info_t last{};
    bool profiling = false;
    // verification
    bool verify = false;
    bool escalate = true;
    double verify_rel = 0.0;
    uint64_t verify_seed = 0x5eed;
    void *vws = nullptr;
    size_t vws_bytes = 0;
    int fault = 0;
    int attempt = 0;
    std::vector<std::array<hipEvent_t, 5>> prof_pending;  // per call: phase boundaries
    std::vector<hipEvent_t> event_pool;
    ozc::BatchState *batch = nullptr;
    ozc::MlpState *mlp = nullptr;
    bool auto_n = false;  // choose N per ozc_zgemm call
};


#define OZC_TRY(expr)                                      \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return OZC_STATUS_HIP_ERROR; \
    } while (0)

namespace ozc {
constexpr size_t kAlign = 256;
inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
OperandView view_A(const void *A, ozc_op_t ta, int64_t m, int64_t k, int64_t lda);
OperandView view_B(const void *B, ozc_op_t tb, int64_t n, int64_t k, int64_t ldb);
ozc_status_t check_args(ozc_op_t ta, ozc_op_t tb, int64_t m, int64_t n, int64_t k, const void *A,
                        int64_t lda, const void *B, int64_t ldb, const void *C, int64_t ldc,
                        bool c_optional);
void batch_release(ozc_context *h);
void mlp_release(ozc_context *h);
ozc_status_t predict_moduli(ozc_context *h, bool single, ozc_op_t ta, ozc_op_t tb, int64_t m,
                            int64_t n, int64_t k, const void *A, int64_t lda, const void *B,
                            int64_t ldb, int *N, PreStats *pre);
// The same in two steps: begin enqueues the prediction (pending: the count is on its way),
// wait delivers the count; the stream may take more work in between.
ozc_status_t predict_moduli_begin(ozc_context *h, bool single, ozc_op_t ta, ozc_op_t tb,
                                  int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                                  const void *B, int64_t ldb, int *N, PreStats *pre, bool *pending);
ozc_status_t predict_moduli_wait(ozc_context *h, int *N);
ozc_status_t predict_moduli_many(ozc_context *h, bool single, const std::vector<OperandView> &va,
                                 const std::vector<OperandView> &vb, std::vector<int> &N);

// Freivalds check (api.cpp): device vectors for products with up to `rows` rows of C and
// inner dimension up to `inner`, carved from one buffer of check_bytes(...) bytes.
struct CheckBufs {
    double2 *y, *yl, *z, *zl, *w, *wl, *v, *vl;
    double *ya, *za, *wa, *va;
    void *scratch;
};
size_t check_bytes(int64_t rows, int64_t inner, size_t scratch_bytes);
ozc_status_t ensure_vws(ozc_context *h, size_t bytes);  // the handle's verification buffer
CheckBufs carve_check(char *base, int64_t rows, int64_t inner);
size_t check_scratch_bytes(ozc_op_t ta, ozc_op_t tb, int64_t m, int64_t n, int64_t k);
// rel: the tolerance relative to the absolute products (the handle's, else 4 k u);
// gam: the relative rounding bound of the double-double evaluation
void check_tolerances(const ozc_context *h, bool single, int64_t n, int64_t k, double *rel,
                      double *gam);
// Enqueues the check of C = alpha op(A) op(B) + beta C_in on stream s; C_in (m x n, leading
// dimension ld_cin) is read only when beta != 0.  word receives (max ratio, failed rows).
ozc_status_t enqueue_check(ozc_context *h, bool single, ozc_op_t ta, ozc_op_t tb, int64_t m,
                           int64_t n, int64_t k, const double alpha[2], const void *A,
                           int64_t lda, const void *B, int64_t ldb, const double beta[2],
                           const void *C, int64_t ldc, const void *cin, int64_t ld_cin,
                           const CheckBufs &b, unsigned long long *word, hipStream_t s);
// Its two parts: the products with the inputs (C_in x, op(B) x, op(A) op(B) x), which
// no rerun changes, and the part that reads the result (C x and the row test).
ozc_status_t enqueue_check_inputs(ozc_context *h, bool single, ozc_op_t ta, ozc_op_t tb,
                                  int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                                  const void *B, int64_t ldb, const double beta[2],
                                  const void *cin, int64_t ld_cin, const CheckBufs &b, hipStream_t s);
ozc_status_t enqueue_check_result(ozc_context *h, bool single, int64_t m, int64_t n, int64_t k,
                                  const double alpha[2], const double beta[2], const void *C,
                                  int64_t ldc, const CheckBufs &b, unsigned long long *word,
                                  hipStream_t s);
}  // namespace ozc
