// Internal definitions shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ozc {

constexpr int kMaxModuli = 24;
constexpr int kChunkBits = 38;      // CRT in FP64 chunks: N * 128 * 2^38 < 2^53 for N <= 24
constexpr int kMaxChunks = 5;       // ceil(bits(P) / 38) for N <= 24 (P below 2^185)
constexpr int kMaxSplitWords = 4;  // residue split: a' as a biased integer of up to 4 32-bit
                                    // words, so |a'| < 2^127 (N <= 24 needs at most 97 bits)
constexpr int kThr = 64;            // threshold table length for the exponent rules
constexpr int kSigmaFracBits = 20;  // fast mode: fixed-point fraction bits of sum of squares
constexpr int kAccuIntBits = 6;     // accurate mode: magnitudes scaled below 2^6
constexpr int16_t kExpZero = -32768;
constexpr int16_t kExpNonfinite = 32767;

// Explicit address spaces for device accesses.  A pointer that a kernel loads from
// memory (the per-problem arguments of the batched kernels) is generic to the
// compiler, which then emits flat accesses, vector loads even for wave-uniform table
// reads; naming the global (1) and constant (4) spaces gives global and scalar loads.
// The constant space is for data that no kernel writes (the moduli tables).
#define OZC_AS_GLOBAL __attribute__((address_space(1)))
#define OZC_AS_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ OZC_AS_GLOBAL T *global_ptr(T *p) {
    return (OZC_AS_GLOBAL T *)(uintptr_t)p;
}
template <typename T>
__device__ __forceinline__ const OZC_AS_CONST T *const_ptr(const T *p) {
    return (const OZC_AS_CONST T *)(uintptr_t)p;
}

// Per-modulus constants.
struct ModConst {
    uint32_t p;                  // modulus
    uint32_t half;               // ceil(p / 2): residues >= half map to r - p
    double schunk[kMaxChunks];   // 38-bit chunks of s_l = (P / p_l) q_l (exact doubles)
    float pf;                    // p
    float ipf;                   // 1 / p rounded to float
    uint32_t wbyte[kMaxSplitWords];  // byte 4 i + b of the words: 2^(8 (4 i + b)) mod p
    uint32_t wbias[kMaxSplitWords];  // entry W - 1: 128 - (2^(32 W - 1) mod p) (two's complement)
    float rbias;                     // 0.5 - 128 ipf (exact)
};

// Constants of one moduli count N.
struct NTable {
    int32_t n;
    int32_t nchunks;              // 38-bit chunks of P (and of every s_l)
    double Pchunk[kMaxChunks];    // 38-bit chunks of P (exact doubles)
    double P_approx;              // P rounded to double
    double inv_P;                 // 1 / P rounded to double
    int32_t fast_tmax;            // largest t with 2^(2t+5) <= P - 1
    int32_t accu_thi;             // largest t with 2 * 4^t <= P - 1
    int32_t max_abits_fast;       // bound on the bit length of |a'| in fast mode
    int32_t max_abits_accu;       // ... in accurate mode
    uint64_t fast_thr[kThr];      // sigma <= fast_thr[d]  <=>  t = fast_tmax - d admissible
    uint64_t accu_thr[kThr];      // X <= accu_thr[d]      <=>  t = accu_thi - d admissible
    ModConst mod[kMaxModuli];
};

// Host: build the tables for N = 1..kMaxModuli (index N-1).
void build_tables(NTable *tables);

// Operand view: `rows` rows of k complex elements; element (r, h) lives at
// base[r * stride_r + h * stride_h] (in complex elements); conj negates Im.
struct OperandView {
    const void *base;
    int64_t rows, k;
    int64_t stride_r, stride_h;
    int conj;
    int contig_h;  // 1 when stride_h == 1 (rows contiguous), 0 when stride_r == 1
};

// Element kind of an operand (the `ek` of the launchers below): complex128,
// complex64 (a bool `single` converts to these two), real float64, real float32.
// OperandView strides count elements of that kind; a real element is handled as a
// complex one with zero imaginary part.
enum ElemKind { kElemZ = 0, kElemC = 1, kElemD = 2, kElemS = 3 };
__host__ __device__ constexpr bool elem_real(int ek) { return ek >= kElemD; }

// Kernel launchers (all asynchronous on `stream`).
hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_row_maxabs(const OperandView &v, int ek, uint64_t *maxbits, hipStream_t s);
// Both operands of one call in one launch: row maxima (sigma = false) or sums of
// squares (sigma = true, maxima final, sigA and sigB zeroed), with tauA, tauB and
// zeros (all or none, zeroed; zeros shared) also the predictor's statistics; the same
// results as launch_row_maxabs / launch_row_sigma on each operand.
hipError_t launch_pair_scans(const OperandView &va, const OperandView &vb, int ek, uint64_t *maxA,
                             uint64_t *maxB, uint64_t *sigA, uint64_t *sigB, bool sigma,
                             hipStream_t s, uint64_t *tauA = nullptr, uint64_t *tauB = nullptr,
                             uint64_t *zeros = nullptr);
// sigma must be zeroed.  With tau and zeros (both or neither, zeroed): also the
// predictor's statistics tau_r = sum ceil(|x| 2^(20 - e_r)) and the zero-real count.
hipError_t launch_row_sigma(const OperandView &v, int ek, const uint64_t *maxbits,
                            uint64_t *sigma, hipStream_t s, uint64_t *tau = nullptr,
                            uint64_t *zeros = nullptr);
hipError_t launch_fast_exponents(const uint64_t *maxbits, const uint64_t *sigma, int64_t rows,
                                 int64_t rows_pad, const NTable *tab, int16_t *mu,
                                 uint32_t *status, hipStream_t s);
// launch_fast_exponents for op(A) (m rows) and op(B) (n columns) in one launch
hipError_t launch_pair_fast_exponents(const uint64_t *maxA, const uint64_t *sigA, int64_t m,
                                      int64_t m_pad, int16_t *mu, const uint64_t *maxB,
                                      const uint64_t *sigB, int64_t n, int64_t n_pad, int16_t *nu,
                                      const NTable *tab, uint32_t *status, hipStream_t s);
// complex: planes Abar_R, Abar_I, Abar_R - Abar_I; real: the plane Abar
hipError_t launch_ceil7(const OperandView &v, int ek, const uint64_t *maxbits,
                        int8_t *dst, int64_t rows_pad, int64_t k_pad, hipStream_t s);
hipError_t launch_accu_exponents(const uint64_t *maxbits, const int32_t *X, int64_t rows,
                                 int64_t rows_pad, const NTable *tab, int16_t *mu,
                                 uint32_t *status, hipStream_t s);
// abits bounds the bit length of |a'| (at most 32 * kMaxSplitWords - 1).  nplanes: 3 (Karatsuba:
// R, I, reduced R + I) or 2 (R, I) for complex operands, 1 (R) for real ones.
hipError_t launch_split(const OperandView &v, int ek, const int16_t *mu, const NTable *tab,
                        int nmod, int nplanes, int abits, int8_t *dst, int64_t rows_pad,
                        int64_t k_pad, hipStream_t s);

struct GemmArgs {
    const int8_t *A;      // [N][planes][k_pad/64][m_pad][64] (slab-major planes)
    const int8_t *B;      // [N][planes][k_pad/64][n_pad][64]
    int64_t m_pad, n_pad, k_pad;
    int nmod;
    int algo;             // 0 Karatsuba, 1 expanded (4 products), 2 real (1 plane, 1 product)
    const NTable *tab;
    int8_t *eprime;       // [N][2][n_pad][m_pad] (real: [N][n_pad][m_pad])
    int32_t *prods;       // optional raw dump [N][nprod][n_pad][m_pad]
    int tile;             // output tile edge (128 or 256); m_pad, n_pad are multiples
};
hipError_t launch_residue_gemm(const GemmArgs &a, hipStream_t s);
// Output tile edge used for an m x n product (the padding of every buffer follows it).
int gemm_tile_for(int64_t m, int64_t n);
// k padding granule of the product kernel for a tile edge (every buffer's k_pad follows it).
int gemm_kstep_for(int tile);
// Output rows (of op(A)) and columns (of op(B)) of one product tile of size class `tile`:
// m_pad and n_pad are multiples of these.
int gemm_tile_rows(int tile);
int gemm_tile_cols(int tile);

// Accurate-mode bound product: X[i] = max_j max(Cbar_R, Cbar_I)_ij, Y[j] likewise.
struct BoundArgs {
    const int8_t *A;      // [3][m_pad][k_pad]: Abar_R, Abar_I, Abar_R - Abar_I (real: [1] Abar)
    const int8_t *B;      // [3][n_pad][k_pad]
    int64_t m_pad, n_pad, k_pad;
    int32_t *X, *Y;       // zero-initialised
    int tile;
    int real;             // 1: real operands, X_i = max_j (Abar Bbar)_ij
};
hipError_t launch_bound_gemm(const BoundArgs &a, hipStream_t s);
// Batched bound products (accurate mode): a persistent kernel over the 128 x 128 tiles of
// all problems, handed out by an atomic counter that must be zero at launch.
struct BatchBound {
    BoundArgs b;
    int64_t item0;          // first work item (tile) of the problem
    int32_t TR, TC;         // tiles per column and per row of the output
};
hipError_t launch_batch_bound(const BatchBound *probs, int nprob, int64_t items,
                              uint32_t *counter, hipStream_t s);

struct CrtArgs {
    const int8_t *eprime;  // [N][2][n_pad][m_pad] (real outputs: [N][n_pad][m_pad])
    int64_t m, n, m_pad, n_pad;
    int nmod;
    int nchunks;           // chunks of P for this N (host copy of tab->nchunks)
    const NTable *tab;     // device pointer
    const int16_t *mu, *nu;
    double alpha_r, alpha_i, beta_r, beta_i;
    void *C;               // column-major, elements of kind `ek` (single: ek of batches)
    int64_t ldc;
    bool single;           // batched launches: complex64 (else complex128)
    int ek;                // single launches: ElemKind of C (real: alpha_i = beta_i = 0)
    void *C_lo;            // complex128 only: double-double output, C the high parts and
                           // C_lo the low parts (alpha = 1, beta = 0); null otherwise
};
hipError_t launch_crt_output(const CrtArgs &a, hipStream_t s);
hipError_t launch_scale_c(void *C, int64_t m, int64_t n, int64_t ldc, int ek, double ar,
                          double ai, double br, double bi, hipStream_t s);

// ---------------------------------------------------------------- batched problems
// Many independent problems share one launch per phase: every block of a
// batched launch first finds its problem (segments are sorted by their first
// block) and then runs the same code as the single-problem kernel.
struct BatchOperand {       // op(A) rows or op(B) columns of one problem
    OperandView v;
    uint64_t *maxbits, *sigma;  // rows_pad entries each, zeroed before the scan
    uint64_t *tau, *zeros;      // scan pass 2 only: predictor statistics (zeroed)
    int16_t *mu;                // rows_pad
    int8_t *res;                // residue planes, slab-major, rows_pad x k_pad each
    const NTable *tab;          // constants of the problem's moduli count
    int8_t *bar;                // accurate mode: the 3 magnitude planes, slab-major
    int32_t *X;                 // accurate mode: bound-product row maxima (rows_pad, zeroed)
    int64_t rows_pad, k_pad;
    int64_t blk_scan, blk_exp;  // first block in the scan and exponent grids
    int64_t blk_ceil7;          // first block in the magnitude grid (accurate mode)
    int64_t blk_split;          // first block in the grid of its split launch
    int32_t nmod;               // the problem's moduli count
};
// Blocks an operand needs in each phase (the host builds the prefix sums with these).
int64_t batch_scan_blocks(const OperandView &v);
int64_t batch_exp_blocks(int64_t rows_pad);
int64_t batch_split_blocks(int64_t rows_pad, int64_t k_pad);
// pass 0: row maxima; 1: sums of squares; 2: sums of squares and the predictor's
// statistics (tau, zeros)
hipError_t launch_batch_scan(const BatchOperand *ops, int nops, int64_t blocks, bool single,
                             int pass, hipStream_t s);
hipError_t launch_batch_fast_exponents(const BatchOperand *ops, int nops, int64_t blocks,
                                       uint32_t *status, hipStream_t s);
// Accurate mode: magnitudes of every operand, then exponents from maxbits and X.
int64_t batch_ceil7_blocks(int64_t rows_pad, int64_t k_pad);
hipError_t launch_batch_ceil7(const BatchOperand *ops, int nops, int64_t blocks, bool single,
                              hipStream_t s);
hipError_t launch_batch_accu_exponents(const BatchOperand *ops, int nops, int64_t blocks,
                                       uint32_t *status, hipStream_t s);
// 32-bit words of the biased form a' + 2^(32 W - 1) of a signed a' with |a'| < 2^abits.
inline int split_words(int abits) { return abits < 32 ? 1 : (abits + 32) / 32; }
constexpr int kMaxSplitBits = 32 * kMaxSplitWords - 1;
// abits: the largest bit length of |a'| among the operands (the chunk count of the launch).
hipError_t launch_batch_split(const BatchOperand *ops, int nops, int64_t blocks, bool single,
                              int nplanes, int abits, hipStream_t s);

struct BatchGemm {          // one problem of a batched product launch
    const int8_t *A, *B;
    int8_t *eprime;
    const NTable *tab;      // constants of the problem's moduli count
    int64_t m_pad, n_pad, k_pad;
    int64_t item0;          // first work item; items run (modulus group, tile row, tile column)
    int32_t TR, TC;         // tiles per column and per row of the output
    int32_t nmod;           // the problem's moduli count
};
// Persistent product kernel over a work queue of (problem, modulus group, tile)
// items, handed out by kBatchQueues atomic counters (one queue per XCD) that must
// be zero at launch.  `group` moduli are computed one after another per item.
// grid_blocks <= 0 picks one wave of resident blocks.
constexpr int kBatchQueues = 8;  // XCDs of an MI355X, each with its own L2
hipError_t launch_batch_gemm(const BatchGemm *probs, int nprob, int64_t items, int tile,
                             int group, int algo, uint32_t *counters, int grid_blocks,
                             hipStream_t s);
// Resident blocks of the persistent product kernel per compute unit, for a tile edge.
int batch_gemm_blocks_per_cu(int tile);

struct BatchCrt {
    CrtArgs a;
    int64_t blk0;
};
int64_t batch_crt_blocks(int64_t m, int64_t n);  // blocks of one problem's reconstruction
hipError_t launch_batch_crt(const BatchCrt *probs, int nprob, int64_t blocks, int nchunks,
                            bool single, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);

// ---------------------------------------------------------------- moduli-count predictor
struct MlpDims {
    int F, H, C;
};
struct MlpOffsets {
    int W1, b1, W2, b2, W3, b3, mu, sd, total, trainable;
};
__host__ __device__ inline MlpOffsets mlp_offsets(const MlpDims &d) {
    MlpOffsets o{};
    o.W1 = 0;
    o.b1 = o.W1 + d.H * d.F;
    o.W2 = o.b1 + d.H;
    o.b2 = o.W2 + d.H * d.H;
    o.W3 = o.b2 + d.H;
    o.b3 = o.W3 + d.C * d.H;
    o.mu = o.b3 + d.C;
    o.sd = o.mu + d.F;
    o.total = o.sd + d.F;
    o.trainable = o.mu;
    return o;
}
struct MlpActs {  // device buffers for `rows` rows
    float *a1, *h1, *a2, *h2, *z, *dz, *loss_r, *d2, *d1, *xs;
};
// Statistics of one product for the predictor: s1 = tau and s2 = sigma of the rows of
// op(A) (a) and the columns of op(B) (b), as the scaling pass computes them.
struct FeatProblem {
    const unsigned long long *s1a, *s2a, *s1b, *s2b;
    int64_t ra, rb;
    const unsigned long long *zeros;
    double m, n, k;
    float *out;  // OZC_MLP_FEATURES floats
};
hipError_t launch_batch_feat_reduce(const FeatProblem *probs, int nprob, hipStream_t s);
hipError_t launch_feat_reduce(const unsigned long long *s1a, const unsigned long long *s2a,
                              int64_t ra, const unsigned long long *s1b,
                              const unsigned long long *s2b, int64_t rb,
                              const unsigned long long *zeros,
                              int64_t m, int64_t n, int64_t k, float *out, hipStream_t s);
hipError_t launch_mlp_forward(const MlpDims &d, const float *params, const float *X, const int *idx,
                              int rows, MlpActs &a, hipStream_t s);
hipError_t launch_mlp_grad(const MlpDims &d, const float *params, const float *X, const int *y,
                           const int *idx, int rows, MlpActs &a, float *grad, float *loss_acc,
                           hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1,
                       float b2, float eps, int t, hipStream_t s);
hipError_t launch_argmax(const float *z, int rows, int C, int *out, hipStream_t s);
// class (argmax of the logits) of each of `rows` feature rows, one fused launch;
// equal to launch_mlp_forward followed by launch_argmax
hipError_t launch_mlp_infer(const MlpDims &d, const float *params, const float *X, int rows,
                            int *cls, hipStream_t s);
hipError_t launch_fill_f32(float *p, int n, float v, hipStream_t s);

// Verification (Freivalds) and test hooks.
hipError_t launch_gemv(const void *M, bool single, int op, int64_t rows, int64_t cols, int64_t ld,
                       const double2 *xv, const double2 *xlo, const double *xa, uint64_t seed,
                       double2 *y, double2 *ylo, double *ya, void *scratch, hipStream_t s);
size_t gemv_scratch_bytes(int64_t rows, int64_t cols);
hipError_t launch_freivalds_rows(const double2 *w, const double2 *wl, const double *wa,
                                 const double2 *z, const double2 *zl, const double *za,
                                 const double2 *v, const double2 *vl, const double *va, int64_t m,
                                 const double alpha[2], const double beta[2], double rel,
                                 double gam, unsigned long long *worst, hipStream_t s);

// One matrix-vector product of a batched check: y = op(M) x as in launch_gemv, with
// x the sign vector of seed (xv == nullptr) or a double-double vector.  make_gemv_task
// fills the column chunking and the partial sums (scratch: gemv_scratch_bytes(rows,
// cols) for op = N, unused otherwise) and appends the task's blocks to the running
// block counts nb[] of the three kernels (partial sums, their reduction, op = T / C).
struct GemvTask {
    const void *M;
    int64_t rows, cols, ld, chunk;
    int32_t op, nchunk;
    const double2 *xv, *xlo;
    const double *xa;
    uint64_t seed;
    double2 *y, *ylo;
    double *ya;
    double2 *ph, *pl;
    double *pa;
    int64_t b0[3];  // first block of this task in each of the three kernels
};
GemvTask make_gemv_task(const void *M, int op, int64_t rows, int64_t cols, int64_t ld,
                        const double2 *xv, const double2 *xlo, const double *xa, uint64_t seed,
                        double2 *y, double2 *ylo, double *ya, void *scratch, int64_t nb[3]);
// tasks: device copy of n tasks whose block counts are nb[]
hipError_t launch_batch_gemv(const GemvTask *tasks, int n, const int64_t nb[3], bool single,
                             hipStream_t s);

// The per-row test of one problem of a batched check (as launch_freivalds_rows; v may
// be null); b0: first block of the problem in the launch.
struct RowsTask {
    const double2 *w, *wl, *z, *zl, *v, *vl;
    const double *wa, *za, *va;
    int64_t m;
    double ar, ai, br, bi, rel, gam;
    unsigned long long *worst;
    int64_t b0;
};
inline int64_t rows_task_blocks(int64_t m) { return (m + 255) / 256; }
// worst[] of every task must be cleared beforehand
hipError_t launch_batch_rows(const RowsTask *tasks, int n, int64_t nblocks, hipStream_t s);
hipError_t launch_debug_xor_byte(int8_t *p, hipStream_t s);
hipError_t launch_debug_add_exp(int16_t *mu, int delta, hipStream_t s);

}  // namespace ozc
