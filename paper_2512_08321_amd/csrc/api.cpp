// C-ABI of the emulated complex GEMM (include/ozc.h): argument checks,
// workspace layout and the order of kernel launches on the caller's stream.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <mutex>
#include <new>
#include <vector>

#include "context.h"

using namespace ozc;

namespace {

// Workspace of ozc_zgemm_noalloc: a fixed array in device memory, one copy per device,
// loaded with the code object and held until the process ends.  Host code never
// uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, looked up once per device (with that device current) when the
// first handle on it is created.
static __device__ __align__(256) unsigned char scratch[OZC_NOALLOC_WORKSPACE];

constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void *g_fixed_ptr[kMaxDevices] = {};

// The calling thread's current device is `device`.
hipError_t fixed_workspace(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_fixed_mu);
    if (!g_fixed_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return e != hipSuccess ? e : hipErrorInvalidSymbol;
        }
        g_fixed_ptr[device] = p;
    }
    *out = g_fixed_ptr[device];
    return hipSuccess;
}


struct Layout {
    int tile;
    int64_t m_pad, n_pad, k_pad;
    int planes, nprod, eplanes;
    size_t maxA, maxB, sigA, sigB, XA, YB, muA, nuB, barA, barB, resA, resB, ep, prods, total;
};

// real: real operands (one residue plane, one product and one E' plane per modulus)
Layout make_layout(const ozc_context *h, int64_t m, int64_t n, int64_t k, bool with_prods,
                   bool real) {
    Layout L{};
    L.tile = gemm_tile_for(m, n);
    L.m_pad = round_up(m > 0 ? m : 1, gemm_tile_rows(L.tile));
    L.n_pad = round_up(n > 0 ? n : 1, gemm_tile_cols(L.tile));
    L.k_pad = round_up(k > 0 ? k : 1, gemm_kstep_for(L.tile));
    L.planes = real ? 1 : (h->algo == OZC_ALGO_KARATSUBA ? 3 : 2);
    L.nprod = real ? 1 : (h->algo == OZC_ALGO_KARATSUBA ? 3 : 4);
    L.eplanes = real ? 1 : 2;
    const size_t N = (size_t)h->nmod;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    // maxA ... YB must stay adjacent and in this order: the scaling phase zeroes them with one fill
    L.maxA = take(8 * (size_t)L.m_pad);
    L.maxB = take(8 * (size_t)L.n_pad);
    L.sigA = take(8 * (size_t)L.m_pad);
    L.sigB = take(8 * (size_t)L.n_pad);
    L.XA = take(4 * (size_t)L.m_pad);
    L.YB = take(4 * (size_t)L.n_pad);
    L.muA = take(2 * (size_t)L.m_pad);
    L.nuB = take(2 * (size_t)L.n_pad);
    const bool accu = h->mode == OZC_MODE_ACCURATE;
    const size_t barp = real ? 1 : 3;  // magnitude planes of the bound product
    L.barA = take(accu ? barp * (size_t)L.m_pad * L.k_pad : 0);
    L.barB = take(accu ? barp * (size_t)L.n_pad * L.k_pad : 0);
    L.resA = take(N * L.planes * (size_t)L.m_pad * L.k_pad);
    L.resB = take(N * L.planes * (size_t)L.n_pad * L.k_pad);
    L.ep = take(N * L.eplanes * (size_t)L.m_pad * L.n_pad);
    L.prods = take(with_prods ? N * L.nprod * 4 * (size_t)L.m_pad * L.n_pad : 0);
    L.total = off;
    return L;
}


ozc_status_t ensure_workspace(ozc_context *h, size_t bytes, char **ws) {
    if (h->use_fixed) {  // checked against the size before any work was enqueued
        if (!h->ws_fixed || bytes > (size_t)OZC_NOALLOC_WORKSPACE) return OZC_STATUS_NOT_SUPPORTED;
        *ws = (char *)h->ws_fixed;
        return OZC_STATUS_SUCCESS;
    }
    if (h->ws_user) {
        if (bytes > h->ws_user_bytes) return OZC_STATUS_ALLOC_FAILED;
        *ws = (char *)h->ws_user;
        return OZC_STATUS_SUCCESS;
    }
    if (bytes > h->ws_own_bytes) {
        if (h->ws_own) {
            OZC_TRY(hipStreamSynchronize(h->stream));
            OZC_TRY(hipFree(h->ws_own));
            h->ws_own = nullptr;
            h->ws_own_bytes = 0;
        }
        if (hipMalloc(&h->ws_own, bytes) != hipSuccess) {
            h->ws_own = nullptr;
            (void)hipGetLastError();
            return OZC_STATUS_ALLOC_FAILED;
        }
        h->ws_own_bytes = bytes;
    }
    *ws = (char *)h->ws_own;
    return OZC_STATUS_SUCCESS;
}

}  // namespace

namespace ozc {

OperandView view_A(const void *A, ozc_op_t ta, int64_t m, int64_t k, int64_t lda) {
    OperandView v{};
    v.base = A;
    v.rows = m;
    v.k = k;
    if (ta == OZC_OP_N) {  // op(A)[i][h] = A[i + h lda]
        v.stride_r = 1;
        v.stride_h = lda;
        v.contig_h = 0;
    } else {               // op(A)[i][h] = A[h + i lda] (conjugated for C)
        v.stride_r = lda;
        v.stride_h = 1;
        v.contig_h = 1;
    }
    v.conj = ta == OZC_OP_C;
    return v;
}

OperandView view_B(const void *B, ozc_op_t tb, int64_t n, int64_t k, int64_t ldb) {
    OperandView v{};
    v.base = B;
    v.rows = n;  // rows of the view = columns of op(B)
    v.k = k;
    if (tb == OZC_OP_N) {  // op(B)[h][j] = B[h + j ldb]
        v.stride_r = ldb;
        v.stride_h = 1;
        v.contig_h = 1;
    } else {               // op(B)[h][j] = B[j + h ldb]
        v.stride_r = 1;
        v.stride_h = ldb;
        v.contig_h = 0;
    }
    v.conj = tb == OZC_OP_C;
    return v;
}

static bool valid_op(ozc_op_t t) { return t == OZC_OP_N || t == OZC_OP_T || t == OZC_OP_C; }

ozc_status_t check_args(ozc_op_t ta, ozc_op_t tb, int64_t m, int64_t n, int64_t k, const void *A,
                        int64_t lda, const void *B, int64_t ldb, const void *C, int64_t ldc,
                        bool c_optional) {
    if (!valid_op(ta) || !valid_op(tb)) return OZC_STATUS_INVALID_VALUE;
    if (m < 0 || n < 0 || k < 0) return OZC_STATUS_INVALID_VALUE;
    const int64_t rowsA = ta == OZC_OP_N ? m : k;
    const int64_t rowsB = tb == OZC_OP_N ? k : n;
    if (lda < (rowsA > 1 ? rowsA : 1)) return OZC_STATUS_INVALID_VALUE;
    if (ldb < (rowsB > 1 ? rowsB : 1)) return OZC_STATUS_INVALID_VALUE;
    if (ldc < (m > 1 ? m : 1)) return OZC_STATUS_INVALID_VALUE;
    if (m > 0 && n > 0 && C == nullptr && !c_optional) return OZC_STATUS_INVALID_VALUE;
    if (m > 0 && n > 0 && k > 0 && (A == nullptr || B == nullptr)) return OZC_STATUS_INVALID_VALUE;
    if (m > ((int64_t)1 << 31) || n > ((int64_t)1 << 31)) return OZC_STATUS_NOT_SUPPORTED;
    return OZC_STATUS_SUCCESS;
}

size_t check_bytes(int64_t rows, int64_t inner, size_t scratch_bytes) {
    const size_t vk = (size_t)(inner > 0 ? inner : 1), vm = (size_t)(rows > 0 ? rows : 1);
    return 3 * align_up(40 * vk) + 9 * align_up(40 * vm) + align_up(scratch_bytes);
}

// Layout: y, yl, ya (inner); then z, zl, za, w, wl, wa, v, vl, va (rows); then scratch.
// The high and low parts are double2 vectors, the absolute sums doubles.
CheckBufs carve_check(char *base, int64_t rows, int64_t inner) {
    const size_t vk = (size_t)(inner > 0 ? inner : 1), vm = (size_t)(rows > 0 ? rows : 1);
    size_t off = 0;
    auto take = [&](size_t b) {
        char *p = base + off;
        off += align_up(b);
        return p;
    };
    CheckBufs c{};
    c.y = (double2 *)take(16 * vk);
    c.yl = (double2 *)take(16 * vk);
    c.ya = (double *)take(8 * vk);
    c.z = (double2 *)take(16 * vm);
    c.zl = (double2 *)take(16 * vm);
    c.za = (double *)take(8 * vm);
    c.w = (double2 *)take(16 * vm);
    c.wl = (double2 *)take(16 * vm);
    c.wa = (double *)take(8 * vm);
    c.v = (double2 *)take(16 * vm);
    c.vl = (double2 *)take(16 * vm);
    c.va = (double *)take(8 * vm);
    c.scratch = base + off;
    return c;
}

size_t check_scratch_bytes(ozc_op_t ta, ozc_op_t tb, int64_t m, int64_t n, int64_t k) {
    size_t scr = gemv_scratch_bytes(m, n);
    if (ta == OZC_OP_N) scr = std::max(scr, gemv_scratch_bytes(m, k));
    if (tb == OZC_OP_N) scr = std::max(scr, gemv_scratch_bytes(k, n));
    return scr;
}

void check_tolerances(const ozc_context *h, bool single, int64_t n, int64_t k, double *rel,
                      double *gam) {
    *rel = h->verify_rel > 0.0 ? h->verify_rel : 4.0 * (double)k * (single ? 0x1p-24 : 0x1p-53);
    *gam = 4.0 * (double)(n + k + 4) * 0x1p-104;  // rounding of the double-double evaluation
}

ozc_status_t enqueue_check_inputs(ozc_context *h, bool single, ozc_op_t ta, ozc_op_t tb,
                                  int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                                  const void *B, int64_t ldb, const double beta[2],
                                  const void *cin, int64_t ld_cin, const CheckBufs &b, hipStream_t s) {
    const uint64_t seed = h->verify_seed;
    const bool beta_zero = beta[0] == 0.0 && beta[1] == 0.0;
    // v = C_in x (m), y = op(B) x (k), z = op(A) y (m)
    if (!beta_zero)
        OZC_TRY(launch_gemv(cin, single, 0, m, n, ld_cin, nullptr, nullptr, nullptr, seed, b.v, b.vl,
                            b.va, b.scratch, s));
    if (tb == OZC_OP_N)
        OZC_TRY(launch_gemv(B, single, 0, k, n, ldb, nullptr, nullptr, nullptr, seed, b.y, b.yl, b.ya,
                            b.scratch, s));
    else
        OZC_TRY(launch_gemv(B, single, (int)tb, n, k, ldb, nullptr, nullptr, nullptr, seed, b.y, b.yl,
                            b.ya, b.scratch, s));
    if (ta == OZC_OP_N)
        OZC_TRY(launch_gemv(A, single, 0, m, k, lda, b.y, b.yl, b.ya, 0, b.z, b.zl, b.za, b.scratch, s));
    else
        OZC_TRY(launch_gemv(A, single, (int)ta, k, m, lda, b.y, b.yl, b.ya, 0, b.z, b.zl, b.za,
                            b.scratch, s));
    return OZC_STATUS_SUCCESS;
}

ozc_status_t enqueue_check_result(ozc_context *h, bool single, int64_t m, int64_t n, int64_t k,
                                  const double alpha[2], const double beta[2], const void *C,
                                  int64_t ldc, const CheckBufs &b, unsigned long long *word,
                                  hipStream_t s) {
    double rel, gam;
    check_tolerances(h, single, n, k, &rel, &gam);
    const bool beta_zero = beta[0] == 0.0 && beta[1] == 0.0;
    // w = C x (m), then the row test against alpha z + beta v
    OZC_TRY(launch_gemv(C, single, 0, m, n, ldc, nullptr, nullptr, nullptr, h->verify_seed, b.w, b.wl,
                        b.wa, b.scratch, s));
    OZC_TRY(launch_freivalds_rows(b.w, b.wl, b.wa, b.z, b.zl, b.za, beta_zero ? nullptr : b.v, b.vl,
                                  b.va, m, alpha, beta, rel, gam, word, s));
    return OZC_STATUS_SUCCESS;
}

ozc_status_t enqueue_check(ozc_context *h, bool single, ozc_op_t ta, ozc_op_t tb, int64_t m,
                           int64_t n, int64_t k, const double alpha[2], const void *A,
                           int64_t lda, const void *B, int64_t ldb, const double beta[2],
                           const void *C, int64_t ldc, const void *cin, int64_t ld_cin,
                           const CheckBufs &b, unsigned long long *word, hipStream_t s) {
    ozc_status_t st = enqueue_check_inputs(h, single, ta, tb, m, n, k, A, lda, B, ldb, beta, cin,
                                           ld_cin, b, s);
    if (st != OZC_STATUS_SUCCESS) return st;
    return enqueue_check_result(h, single, m, n, k, alpha, beta, C, ldc, b, word, s);
}

ozc_status_t ensure_vws(ozc_context *h, size_t bytes) {
    if (bytes <= h->vws_bytes) return OZC_STATUS_SUCCESS;
    if (h->vws) {
        OZC_TRY(hipStreamSynchronize(h->stream));
        OZC_TRY(hipFree(h->vws));
        h->vws = nullptr;
        h->vws_bytes = 0;
    }
    if (hipMalloc(&h->vws, bytes) != hipSuccess) {
        h->vws = nullptr;
        (void)hipGetLastError();
        return OZC_STATUS_ALLOC_FAILED;
    }
    h->vws_bytes = bytes;
    return OZC_STATUS_SUCCESS;
}
}  // namespace ozc

namespace {

// Phase events of one call (a no-op unless profiling is enabled).
struct PhaseEvents {
    ozc_context *h;
    std::array<hipEvent_t, 5> ev{};
    bool on;
    PhaseEvents(ozc_context *ctx) : h(ctx), on(ctx->profiling && !ctx->use_fixed) {
        if (!on) return;
        for (auto &e : ev) {
            if (!h->event_pool.empty()) {
                e = h->event_pool.back();
                h->event_pool.pop_back();
            } else if (hipEventCreate(&e) != hipSuccess) {
                on = false;
                return;
            }
        }
    }
    hipError_t mark(int i) { return on ? hipEventRecord(ev[i], h->stream) : hipSuccess; }
    void commit() {
        if (on) h->prof_pending.push_back(ev);
        on = false;
    }
    ~PhaseEvents() {
        if (on)
            for (auto e : ev) h->event_pool.push_back(e);
    }
};

struct InspectOut {
    int16_t *mu, *nu;
    int8_t *resA, *resB;
    int32_t *prods;
    int8_t *eprime;
};

// ek: ElemKind of A, B and C (a bool `single` selects complex64 over complex128); real
// kinds take real alpha/beta (imaginary parts zero) and treat op C as op T.
ozc_status_t run(ozc_context *h, int ek, ozc_op_t ta, ozc_op_t tb, int64_t m, int64_t n,
                 int64_t k, const double alpha[2], const void *A, int64_t lda, const void *B,
                 int64_t ldb, const double beta[2], void *C, int64_t ldc, const InspectOut *ins) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (ek < kElemZ || ek > kElemS) return OZC_STATUS_INVALID_VALUE;
    const bool real = elem_real(ek);
    if (real) {
        if (ta == OZC_OP_C) ta = OZC_OP_T;
        if (tb == OZC_OP_C) tb = OZC_OP_T;
    }
    ozc_status_t st = check_args(ta, tb, m, n, k, A, lda, B, ldb, C, ldc, ins != nullptr);
    if (st != OZC_STATUS_SUCCESS) return st;
    if (k > OZC_MAX_K) {
        // INT32 accumulation is exact only up to OZC_MAX_K terms (127^2 per term):
        // split k into near-equal chunks, each an emulated product of its own
        // (own exponents), accumulated in C with beta = 1 after the first.
        if (ins) return OZC_STATUS_NOT_SUPPORTED;
        if (m == 0 || n == 0) return OZC_STATUS_SUCCESS;
        const int64_t nc = (k + OZC_MAX_K - 1) / OZC_MAX_K;
        const size_t es = ek == kElemZ ? 16 : (ek == kElemS ? 4 : 8);
        const double one[2] = {1.0, 0.0};
        double ops = 0.0;
        // the non-finite flag is cleared once here and then collects every chunk's
        struct KeepStatus {
            ozc_context *h;
            ~KeepStatus() { h->keep_status = false; }
        } keep{h};
        OZC_TRY(hipSetDevice(h->device));
        OZC_TRY(launch_fill_u64(h->status_dev, 1, 0, h->stream));
        h->keep_status = true;
        for (int64_t c = 0; c < nc; ++c) {
            const int64_t h0 = k * c / nc, h1 = k * (c + 1) / nc;
            const char *Ac = (const char *)A + es * (size_t)(ta == OZC_OP_N ? h0 * lda : h0);
            const char *Bc = (const char *)B + es * (size_t)(tb == OZC_OP_N ? h0 : h0 * ldb);
            st = run(h, ek, ta, tb, m, n, h1 - h0, alpha, Ac, lda, Bc, ldb, c == 0 ? beta : one,
                     C, ldc, nullptr);
            if (st != OZC_STATUS_SUCCESS) return st;
            ops += h->last.int8_ops;
        }
        h->last.k = k;
        h->last.int8_ops = ops;
        return OZC_STATUS_SUCCESS;
    }
    hipStream_t s = h->stream;
    OZC_TRY(hipSetDevice(h->device));
    h->last = ozc_info_t{};
    h->last.num_moduli = h->nmod;
    h->last.mode = h->mode;
    h->last.algo = real ? -1 : h->algo;
    h->last.m = m;
    h->last.n = n;
    h->last.k = k;
    if (!h->keep_status) OZC_TRY(launch_fill_u64(h->status_dev, 1, 0, s));
    if (m == 0 || n == 0) return OZC_STATUS_SUCCESS;
    const bool alpha_zero = alpha[0] == 0.0 && alpha[1] == 0.0;
    if ((alpha_zero || k == 0) && ins == nullptr) {
        OZC_TRY(launch_scale_c(C, m, n, ldc, ek, alpha[0], alpha[1], beta[0], beta[1], s));
        return OZC_STATUS_SUCCESS;
    }
    if (k == 0) return OZC_STATUS_INVALID_VALUE;  // nothing to inspect

    const Layout L = make_layout(h, m, n, k, ins && ins->prods, real);
    char *ws = nullptr;
    st = ensure_workspace(h, L.total, &ws);
    if (st != OZC_STATUS_SUCCESS) return st;
    h->last.workspace = L.total;
    h->last.int8_ops = 2.0 * (double)L.nprod * (double)h->nmod * (double)m * (double)n * (double)k;

    const NTable *tab = h->tab_dev + (h->nmod - 1);
    const NTable &th = h->tab_host[(size_t)h->nmod - 1];
    uint64_t *maxA = (uint64_t *)(ws + L.maxA), *maxB = (uint64_t *)(ws + L.maxB);
    uint64_t *sigA = (uint64_t *)(ws + L.sigA), *sigB = (uint64_t *)(ws + L.sigB);
    int32_t *XA = (int32_t *)(ws + L.XA), *YB = (int32_t *)(ws + L.YB);
    int16_t *muA = (int16_t *)(ws + L.muA), *nuB = (int16_t *)(ws + L.nuB);
    int8_t *resA = (int8_t *)(ws + L.resA), *resB = (int8_t *)(ws + L.resB);
    int8_t *ep = (int8_t *)(ws + L.ep);
    int32_t *prods = ins && ins->prods ? (int32_t *)(ws + L.prods) : nullptr;
    uint32_t *status = (uint32_t *)h->status_dev;

    const OperandView vA = view_A(A, ta, m, k, lda);
    const OperandView vB = view_B(B, tb, n, k, ldb);

    PhaseEvents pe(h);
    if (ins) pe.on = false;
    const int fault = h->fault;
    // Step III: scaling exponents
    OZC_TRY(pe.mark(0));
    // Statistics computed by the moduli-count prediction of this call (same operands,
    // same k) are taken over; otherwise one fill zeroes maxA, maxB, sigA, sigB, XA, YB
    // (adjacent in the layout) and the scans run.
    const bool pre = h->pre.maxA != nullptr && ins == nullptr && !real;
    const uint64_t *cmaxA = pre ? h->pre.maxA : maxA, *cmaxB = pre ? h->pre.maxB : maxB;
    const uint64_t *csigA = pre ? h->pre.sigA : sigA, *csigB = pre ? h->pre.sigB : sigB;
    if (pre) {
        OZC_TRY(launch_fill_u64((uint64_t *)XA, (int64_t)(L.muA - L.XA) / 8, 0, s));
    } else {
        OZC_TRY(launch_fill_u64(maxA, (int64_t)(L.muA - L.maxA) / 8, 0, s));
        OZC_TRY(launch_pair_scans(vA, vB, ek, maxA, maxB, sigA, sigB, false, s));
    }
    int abits;
    if (h->mode == OZC_MODE_FAST) {
        if (!pre) {
            OZC_TRY(launch_pair_scans(vA, vB, ek, maxA, maxB, sigA, sigB, true, s));
        }
        OZC_TRY(launch_pair_fast_exponents(cmaxA, csigA, m, L.m_pad, muA, cmaxB, csigB, n, L.n_pad,
                                           nuB, tab, status, s));
        abits = th.max_abits_fast;
    } else {
        int8_t *barA = (int8_t *)(ws + L.barA), *barB = (int8_t *)(ws + L.barB);
        OZC_TRY(launch_ceil7(vA, ek, cmaxA, barA, L.m_pad, L.k_pad, s));
        OZC_TRY(launch_ceil7(vB, ek, cmaxB, barB, L.n_pad, L.k_pad, s));
        BoundArgs ba{barA, barB, L.m_pad, L.n_pad, L.k_pad, XA, YB, L.tile, real ? 1 : 0};
        OZC_TRY(launch_bound_gemm(ba, s));
        OZC_TRY(launch_accu_exponents(cmaxA, XA, m, L.m_pad, tab, muA, status, s));
        OZC_TRY(launch_accu_exponents(cmaxB, YB, n, L.n_pad, tab, nuB, status, s));
        abits = th.max_abits_accu;
    }
    if (fault == 2) OZC_TRY(launch_debug_add_exp(muA, 12, s));
    if (abits > kMaxSplitBits) return OZC_STATUS_NOT_SUPPORTED;

    // Steps IV, V-i/ii: truncation and residues
    OZC_TRY(pe.mark(1));
    OZC_TRY(launch_split(vA, ek, muA, tab, h->nmod, L.planes, abits, resA, L.m_pad, L.k_pad, s));
    OZC_TRY(launch_split(vB, ek, nuB, tab, h->nmod, L.planes, abits, resB, L.n_pad, L.k_pad, s));

    // Step V-iii/iv: INT8 products and their residues
    OZC_TRY(pe.mark(2));
    const int galgo = real ? 2 : (h->algo == OZC_ALGO_KARATSUBA ? 0 : 1);
    GemmArgs ga{resA, resB, L.m_pad, L.n_pad, L.k_pad, h->nmod, galgo, tab, ep, prods, L.tile};
    OZC_TRY(launch_residue_gemm(ga, s));
    if (fault == 1 && h->attempt == 0) OZC_TRY(launch_debug_xor_byte(ep, s));
    OZC_TRY(pe.mark(3));

    // Steps V-v, V-vi, VI
    if (C) {
        CrtArgs ca{};
        ca.eprime = ep;
        ca.m = m;
        ca.n = n;
        ca.m_pad = L.m_pad;
        ca.n_pad = L.n_pad;
        ca.nmod = h->nmod;
        ca.nchunks = th.nchunks;
        ca.tab = tab;
        ca.mu = muA;
        ca.nu = nuB;
        ca.alpha_r = alpha[0];
        ca.alpha_i = alpha[1];
        ca.beta_r = beta[0];
        ca.beta_i = beta[1];
        ca.C = C;
        ca.ldc = ldc;
        ca.single = ek == kElemC;
        ca.ek = ek;
        ca.C_lo = ek == kElemZ ? h->dd_lo : nullptr;
        OZC_TRY(launch_crt_output(ca, s));
    }
    OZC_TRY(pe.mark(4));
    pe.commit();

    if (ins) {
        if (ins->mu) OZC_TRY(hipMemcpyAsync(ins->mu, muA, 2 * (size_t)m, hipMemcpyDeviceToDevice, s));
        if (ins->nu) OZC_TRY(hipMemcpyAsync(ins->nu, nuB, 2 * (size_t)n, hipMemcpyDeviceToDevice, s));
        const int64_t N = h->nmod;
        // dense copies of padded planes: plane q of `count` planes, `rows` x `width` bytes
        auto planes = [&](void *dst, const void *src, size_t width, size_t src_pitch, int64_t rows,
                          int64_t src_rows, int64_t count) -> hipError_t {
            for (int64_t q = 0; q < count; ++q) {
                hipError_t e = hipMemcpy2DAsync((char *)dst + (size_t)q * rows * width, width,
                                                (const char *)src + (size_t)q * src_rows * src_pitch,
                                                src_pitch, width, (size_t)rows,
                                                hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        };
        // residue planes are stored slab-major: k-slab kb of a plane is rows_pad x 64 bytes
        auto slab_planes = [&](int8_t *dst, const int8_t *src, int64_t rows, int64_t rows_pad,
                               int64_t count) -> hipError_t {
            for (int64_t q = 0; q < count; ++q) {
                for (int64_t kb = 0; kb * 64 < k; ++kb) {
                    const size_t w = (size_t)std::min<int64_t>(64, k - kb * 64);
                    hipError_t e = hipMemcpy2DAsync(
                        dst + (size_t)q * rows * k + kb * 64, (size_t)k,
                        src + (size_t)q * rows_pad * L.k_pad + (size_t)kb * rows_pad * 64, 64, w,
                        (size_t)rows, hipMemcpyDeviceToDevice, s);
                    if (e != hipSuccess) return e;
                }
            }
            return hipSuccess;
        };
        if (ins->resA) OZC_TRY(slab_planes(ins->resA, resA, m, L.m_pad, N * L.planes));
        if (ins->resB) OZC_TRY(slab_planes(ins->resB, resB, n, L.n_pad, N * L.planes));
        if (ins->eprime)
            OZC_TRY(planes(ins->eprime, ep, (size_t)m, (size_t)L.m_pad, n, L.n_pad, N * L.eplanes));
        if (ins->prods)
            OZC_TRY(planes(ins->prods, prods, 4 * (size_t)m, 4 * (size_t)L.m_pad, n, L.n_pad, N * L.nprod));
    }
    return OZC_STATUS_SUCCESS;
}


// One call with the Freivalds check and moduli escalation (see ozc_set_verify).
ozc_status_t run_verified(ozc_context *h, bool single, ozc_op_t ta, ozc_op_t tb, int64_t m,
                          int64_t n, int64_t k, const double alpha[2], const void *A,
                          int64_t lda, const void *B, int64_t ldb, const double beta[2], void *C,
                          int64_t ldc) {
    h->attempt = 0;
    // restores the configured N and drops the prediction's statistics on every exit
    struct RestoreN0 {
        ozc_context *h;
        int n0;
        ~RestoreN0() {
            h->nmod = n0;
            h->pre = PreStats{};
        }
    } restore0{h, h->nmod};
    // The learned count is enqueued first and awaited as late as possible: with the check
    // on, its products with the inputs run while the host waits for the count.
    bool pending = false;
    int N_pred = h->nmod;
    if (h->auto_n) {
        ozc_status_t sa = check_args(ta, tb, m, n, k, A, lda, B, ldb, C, ldc, false);
        if (sa != OZC_STATUS_SUCCESS) return sa;
        N_pred = 9;  // complex64: the fixed count (single-precision level)
        if (!single) {
            OZC_TRY(hipSetDevice(h->device));
            // the prediction's scaling statistics serve every attempt of this call
            sa = predict_moduli_begin(h, single, ta, tb, m, n, k, A, lda, B, ldb, &N_pred, &h->pre,
                                      &pending);
            if (sa != OZC_STATUS_SUCCESS) return sa;
        }
    }
    auto take_count = [&]() -> ozc_status_t {
        if (pending) {
            pending = false;
            ozc_status_t sw = predict_moduli_wait(h, &N_pred);
            if (sw != OZC_STATUS_SUCCESS) return sw;
        }
        h->nmod = N_pred;
        return OZC_STATUS_SUCCESS;
    };
    ozc_status_t st;
    if (!h->verify) {
        if ((st = take_count()) != OZC_STATUS_SUCCESS) return st;
        return run(h, single, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nullptr);
    }
    st = check_args(ta, tb, m, n, k, A, lda, B, ldb, C, ldc, false);
    if (st != OZC_STATUS_SUCCESS) return st;
    const bool alpha_zero = alpha[0] == 0.0 && alpha[1] == 0.0;
    if (m == 0 || n == 0 || k == 0 || alpha_zero) {
        if ((st = take_count()) != OZC_STATUS_SUCCESS) return st;
        return run(h, single, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nullptr);
    }
    hipStream_t s = h->stream;
    OZC_TRY(hipSetDevice(h->device));
    const bool beta_zero = beta[0] == 0.0 && beta[1] == 0.0;
    const size_t es = single ? 8 : 16;
    // check vectors, the result word and (beta != 0) a copy of C_in for the check and reruns
    const size_t cb = check_bytes(m, k, check_scratch_bytes(ta, tb, m, n, k));
    const size_t o_word = cb;
    const size_t o_cin = align_up(o_word + 16);
    const size_t total = o_cin + (beta_zero ? 0 : es * (size_t)m * (size_t)n);
    st = ensure_vws(h, total);
    if (st != OZC_STATUS_SUCCESS) return st;
    char *vw = (char *)h->vws;
    const CheckBufs bufs = carve_check(vw, m, k);
    unsigned long long *word = (unsigned long long *)(vw + o_word);
    void *cin = vw + o_cin;
    if (!beta_zero)
        OZC_TRY(hipMemcpy2DAsync(cin, es * m, C, es * ldc, es * m, n, hipMemcpyDeviceToDevice, s));
    // the check's products with the inputs: once per call (reruns do not change them)
    st = enqueue_check_inputs(h, single, ta, tb, m, n, k, A, lda, B, ldb, beta, cin, m, bufs, s);
    if (st != OZC_STATUS_SUCCESS) return st;
    if ((st = take_count()) != OZC_STATUS_SUCCESS) return st;
    struct RestoreN {
        ozc_context *h;
        int n0;
        ~RestoreN() { h->nmod = n0; }
    } restore{h, h->nmod};
    int N = h->nmod, escalations = 0;
    double ratio = 0.0;
    int64_t failed = 0;
    for (;;) {
        h->nmod = N;
        st = run(h, single, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nullptr);
        if (st != OZC_STATUS_SUCCESS) break;
        st = enqueue_check_result(h, single, m, n, k, alpha, beta, C, ldc, bufs, word, s);
        if (st != OZC_STATUS_SUCCESS) break;
        unsigned long long host[2] = {0, 0};
        OZC_TRY(hipMemcpyAsync(host, word, sizeof(host), hipMemcpyDeviceToHost, s));
        OZC_TRY(hipStreamSynchronize(s));
        memcpy(&ratio, &host[0], sizeof(double));
        failed = (int64_t)host[1];
        if (failed == 0) break;
        if (!h->escalate || N >= OZC_MAX_MODULI) {
            st = OZC_STATUS_VERIFY_FAILED;
            break;
        }
        N = std::min(OZC_MAX_MODULI, N + 2);
        ++escalations;
        ++h->attempt;
        if (!beta_zero)
            OZC_TRY(hipMemcpy2DAsync(C, es * ldc, cin, es * m, es * m, n, hipMemcpyDeviceToDevice, s));
    }
    h->last.verified = 1;
    h->last.escalations = escalations;
    h->last.verify_failed_rows = failed;
    h->last.verify_ratio = ratio;
    return st;
}

}  // namespace

extern "C" {

const char *ozc_status_string(ozc_status_t s) {
    switch (s) {
        case OZC_STATUS_SUCCESS: return "success";
        case OZC_STATUS_INVALID_VALUE: return "invalid value";
        case OZC_STATUS_NOT_SUPPORTED: return "not supported";
        case OZC_STATUS_ALLOC_FAILED: return "device allocation failed";
        case OZC_STATUS_HIP_ERROR: return "HIP runtime error";
        case OZC_STATUS_NONFINITE: return "non-finite input";
        case OZC_STATUS_INVALID_HANDLE: return "invalid handle";
        case OZC_STATUS_VERIFY_FAILED: return "verification failed";
    }
    return "unknown status";
}

ozc_status_t ozc_create(ozc_handle_t *handle, int device) {
    if (!handle) return OZC_STATUS_INVALID_VALUE;
    *handle = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return OZC_STATUS_INVALID_VALUE;
    if (hipSetDevice(device) != hipSuccess) return OZC_STATUS_HIP_ERROR;
    ozc_context *h = new (std::nothrow) ozc_context();
    if (!h) return OZC_STATUS_ALLOC_FAILED;
    h->device = device;
    h->tab_host.resize(kMaxModuli);
    build_tables(h->tab_host.data());
    if (hipMalloc(&h->tab_dev, sizeof(NTable) * kMaxModuli) != hipSuccess ||
        hipMalloc(&h->status_dev, 256) != hipSuccess) {
        if (h->tab_dev) (void)hipFree(h->tab_dev);
        delete h;
        return OZC_STATUS_ALLOC_FAILED;
    }
    if (hipMemcpy(h->tab_dev, h->tab_host.data(), sizeof(NTable) * kMaxModuli,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(h->status_dev, 0, 256) != hipSuccess) {
        (void)hipFree(h->tab_dev);
        (void)hipFree(h->status_dev);
        delete h;
        return OZC_STATUS_HIP_ERROR;
    }
    // The fixed workspace of ozc_zgemm_noalloc; a failed lookup only disables that call.
    if (fixed_workspace(device, &h->ws_fixed) != hipSuccess) h->ws_fixed = nullptr;
    *handle = h;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_destroy(ozc_handle_t h) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    for (auto &ev : h->prof_pending)
        for (auto e : ev) (void)hipEventDestroy(e);
    for (auto e : h->event_pool) (void)hipEventDestroy(e);
    if (h->ws_own) (void)hipFree(h->ws_own);
    if (h->vws) (void)hipFree(h->vws);
    batch_release(h);
    mlp_release(h);
    (void)hipFree(h->tab_dev);
    (void)hipFree(h->status_dev);
    delete h;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_set_stream(ozc_handle_t h, void *stream) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    h->stream = (hipStream_t)stream;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_set_config(ozc_handle_t h, int num_moduli, ozc_mode_t mode, ozc_algo_t algo) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (num_moduli != 0 && (num_moduli < OZC_MIN_MODULI || num_moduli > OZC_MAX_MODULI))
        return OZC_STATUS_INVALID_VALUE;
    if (mode != OZC_MODE_FAST && mode != OZC_MODE_ACCURATE) return OZC_STATUS_INVALID_VALUE;
    if (algo != OZC_ALGO_KARATSUBA && algo != OZC_ALGO_4M) return OZC_STATUS_INVALID_VALUE;
    h->auto_n = num_moduli == 0;
    if (num_moduli != 0) h->nmod = num_moduli;
    h->mode = mode;
    h->algo = algo;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_workspace_size(ozc_handle_t h, ozc_op_t ta, ozc_op_t tb, int64_t m, int64_t n,
                                int64_t k, size_t *bytes) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (!bytes || !valid_op(ta) || !valid_op(tb) || m < 0 || n < 0 || k < 0)
        return OZC_STATUS_INVALID_VALUE;
    const int64_t kc = k > OZC_MAX_K ? (k + (k + OZC_MAX_K - 1) / OZC_MAX_K - 1) /
                                           ((k + OZC_MAX_K - 1) / OZC_MAX_K)
                                     : k;  // largest k chunk
    *bytes = (m == 0 || n == 0 || k == 0) ? 0 : make_layout(h, m, n, kc, false, false).total;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_set_workspace(ozc_handle_t h, void *ptr, size_t bytes) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (ptr && ((uintptr_t)ptr % kAlign)) return OZC_STATUS_INVALID_VALUE;
    h->ws_user = ptr;
    h->ws_user_bytes = ptr ? bytes : 0;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_zgemm(ozc_handle_t h, ozc_op_t ta, ozc_op_t tb, int64_t m, int64_t n, int64_t k,
                       const double alpha[2], const void *A, int64_t lda, const void *B,
                       int64_t ldb, const double beta[2], void *C, int64_t ldc) {
    if (!alpha || !beta) return OZC_STATUS_INVALID_VALUE;
    return run_verified(h, false, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

ozc_status_t ozc_zgemm_noalloc(ozc_handle_t h, ozc_op_t ta, ozc_op_t tb, int64_t m, int64_t n,
                               int64_t k, const double alpha[2], const void *A, int64_t lda,
                               const void *B, int64_t ldb, const double beta[2], void *C,
                               int64_t ldc) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (!alpha || !beta) return OZC_STATUS_INVALID_VALUE;
    ozc_status_t st = check_args(ta, tb, m, n, k, A, lda, B, ldb, C, ldc, false);
    if (st != OZC_STATUS_SUCCESS) return st;
    // the check and the learned count need buffers of their own
    if (h->verify || h->auto_n) return OZC_STATUS_NOT_SUPPORTED;
    if (!h->ws_fixed) return OZC_STATUS_HIP_ERROR;
    size_t need = 0;
    st = ozc_workspace_size(h, ta, tb, m, n, k, &need);
    if (st != OZC_STATUS_SUCCESS) return st;
    if (need > (size_t)OZC_NOALLOC_WORKSPACE) return OZC_STATUS_NOT_SUPPORTED;
    struct UseFixed {
        ozc_context *h;
        ~UseFixed() { h->use_fixed = false; }
    } restore{h};
    h->use_fixed = true;
    return run(h, false, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nullptr);
}

ozc_status_t ozc_cgemm(ozc_handle_t h, ozc_op_t ta, ozc_op_t tb, int64_t m, int64_t n, int64_t k,
                       const float alpha[2], const void *A, int64_t lda, const void *B,
                       int64_t ldb, const float beta[2], void *C, int64_t ldc) {
    if (!alpha || !beta) return OZC_STATUS_INVALID_VALUE;
    const double al[2] = {alpha[0], alpha[1]}, be[2] = {beta[0], beta[1]};
    return run_verified(h, true, ta, tb, m, n, k, al, A, lda, B, ldb, be, C, ldc);
}

ozc_status_t ozc_zgemm_dd(ozc_handle_t h, ozc_op_t ta, ozc_op_t tb, int64_t m, int64_t n,
                          int64_t k, const void *A, int64_t lda, const void *B, int64_t ldb,
                          void *C_hi, void *C_lo, int64_t ldc) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    ozc_status_t st = check_args(ta, tb, m, n, k, A, lda, B, ldb, C_hi, ldc, false);
    if (st != OZC_STATUS_SUCCESS) return st;
    if (m > 0 && n > 0 && !C_lo) return OZC_STATUS_INVALID_VALUE;
    if (k > OZC_MAX_K) return OZC_STATUS_NOT_SUPPORTED;
    const double one[2] = {1.0, 0.0}, zero[2] = {0.0, 0.0};
    if (m == 0 || n == 0) return OZC_STATUS_SUCCESS;
    if (k == 0) {  // the empty product: both parts zero
        OZC_TRY(hipSetDevice(h->device));
        OZC_TRY(launch_scale_c(C_hi, m, n, ldc, kElemZ, 0.0, 0.0, 0.0, 0.0, h->stream));
        OZC_TRY(launch_scale_c(C_lo, m, n, ldc, kElemZ, 0.0, 0.0, 0.0, 0.0, h->stream));
        return OZC_STATUS_SUCCESS;
    }
    struct DdOut {
        ozc_context *h;
        ~DdOut() { h->dd_lo = nullptr; }
    } restore{h};
    h->dd_lo = C_lo;
    return run(h, kElemZ, ta, tb, m, n, k, one, A, lda, B, ldb, zero, C_hi, ldc, nullptr);
}

// Real products: the handle's fixed moduli count and scaling mode; no check, no learned count.
static ozc_status_t run_real(ozc_context *h, int ek, ozc_op_t ta, ozc_op_t tb, int64_t m,
                             int64_t n, int64_t k, double alpha, const void *A, int64_t lda,
                             const void *B, int64_t ldb, double beta, void *C, int64_t ldc) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    const double al[2] = {alpha, 0.0}, be[2] = {beta, 0.0};
    return run(h, ek, ta, tb, m, n, k, al, A, lda, B, ldb, be, C, ldc, nullptr);
}

ozc_status_t ozc_dgemm(ozc_handle_t h, ozc_op_t ta, ozc_op_t tb, int64_t m, int64_t n, int64_t k,
                       const double *alpha, const void *A, int64_t lda, const void *B,
                       int64_t ldb, const double *beta, void *C, int64_t ldc) {
    if (!alpha || !beta) return OZC_STATUS_INVALID_VALUE;
    return run_real(h, kElemD, ta, tb, m, n, k, *alpha, A, lda, B, ldb, *beta, C, ldc);
}

ozc_status_t ozc_sgemm(ozc_handle_t h, ozc_op_t ta, ozc_op_t tb, int64_t m, int64_t n, int64_t k,
                       const float *alpha, const void *A, int64_t lda, const void *B,
                       int64_t ldb, const float *beta, void *C, int64_t ldc) {
    if (!alpha || !beta) return OZC_STATUS_INVALID_VALUE;
    return run_real(h, kElemS, ta, tb, m, n, k, *alpha, A, lda, B, ldb, *beta, C, ldc);
}

ozc_status_t ozc_set_verify(ozc_handle_t h, int enable, double rel, int escalate, uint64_t seed) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (!(rel == rel)) return OZC_STATUS_INVALID_VALUE;
    h->verify = enable != 0;
    h->verify_rel = rel;
    h->escalate = escalate != 0;
    h->verify_seed = seed;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_debug_inject(ozc_handle_t h, int fault) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (fault < 0 || fault > 2) return OZC_STATUS_INVALID_VALUE;
    h->fault = fault;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_inspect(ozc_handle_t h, int single, ozc_op_t ta, ozc_op_t tb, int64_t m,
                         int64_t n, int64_t k, const void *A, int64_t lda, const void *B,
                         int64_t ldb, int16_t *mu, int16_t *nu, int8_t *resA, int8_t *resB,
                         int32_t *prods, int8_t *eprime, void *C, int64_t ldc) {
    const double one[2] = {1.0, 0.0}, zero[2] = {0.0, 0.0};
    InspectOut ins{mu, nu, resA, resB, prods, eprime};
    if (single < kElemZ || single > kElemS) return OZC_STATUS_INVALID_VALUE;
    return run(h, single, ta, tb, m, n, k, one, A, lda, B, ldb, zero, C, ldc, &ins);
}

ozc_status_t ozc_set_profiling(ozc_handle_t h, int enable) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    h->profiling = enable != 0;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_profile_read(ozc_handle_t h, ozc_profile_t *out) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (!out) return OZC_STATUS_INVALID_VALUE;
    *out = ozc_profile_t{};
    if (hipSetDevice(h->device) != hipSuccess) return OZC_STATUS_HIP_ERROR;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return OZC_STATUS_HIP_ERROR;
    ozc_status_t st = OZC_STATUS_SUCCESS;
    for (auto &ev : h->prof_pending) {
        float t[4] = {0, 0, 0, 0}, tot = 0;
        bool ok = true;
        for (int i = 0; i < 4; ++i) ok = ok && hipEventElapsedTime(&t[i], ev[i], ev[i + 1]) == hipSuccess;
        ok = ok && hipEventElapsedTime(&tot, ev[0], ev[4]) == hipSuccess;
        if (!ok) st = OZC_STATUS_HIP_ERROR;
        out->calls += 1;
        out->scale_ms += t[0];
        out->split_ms += t[1];
        out->gemm_ms += t[2];
        out->crt_ms += t[3];
        out->total_ms += tot;
        for (auto e : ev) h->event_pool.push_back(e);
    }
    h->prof_pending.clear();
    return st;
}

ozc_status_t ozc_last_info(ozc_handle_t h, ozc_info_t *info) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (!info) return OZC_STATUS_INVALID_VALUE;
    if (hipSetDevice(h->device) != hipSuccess) return OZC_STATUS_HIP_ERROR;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return OZC_STATUS_HIP_ERROR;
    uint64_t st = 0;
    if (hipMemcpy(&st, h->status_dev, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
        return OZC_STATUS_HIP_ERROR;
    h->last.nonfinite = (int)(st & 1u);
    *info = h->last;
    return h->last.nonfinite ? OZC_STATUS_NONFINITE : OZC_STATUS_SUCCESS;
}

}  // extern "C"
