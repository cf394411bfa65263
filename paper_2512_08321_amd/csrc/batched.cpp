// Batched products (include/ozc.h, "batches"): the plan of one batch (padding,
// workspace layout, per-phase block and work-item numbering), its launch
// sequence, the HIP graph that replays it, and the schedule autotuner.
//
// Every problem goes through the same kernels as a single call (the batched
// kernels only add the lookup of their problem), so the results are
// bit-identical to ozc_zgemm on the same arguments.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "context.h"

namespace ozc {

namespace {

struct Problem {
    ozc_op_t ta, tb;
    int64_t m, n, k, lda, ldb, ldc;
    const void *A, *B;
    void *C;
    double alpha[2], beta[2];
};

}  // namespace

struct BatchPlan {
    // A launch over a contiguous range of descriptors; param = chunk bits (split) or chunks of P (CRT).
    struct Range {
        int first, count;
        int64_t blocks;
        int param;
    };
    std::vector<uint64_t> key;
    bool single = false, accurate = false;
    int algo = 0, planes = 0, group = 1, nmax = 0;
    size_t ws_bytes = 0;
    std::vector<BatchOperand> ops;  // ordered by split launch
    std::vector<Range> splits;      // one split launch per word count
    std::vector<BatchGemm> gm[2];   // [0]: 256 x 256 tiles, [1]: 128 x 128 tiles
    std::vector<BatchCrt> crt;      // ordered by CRT launch
    std::vector<Range> crts;        // one CRT launch per chunk count of P
    std::vector<BatchBound> bound;  // accurate mode: bound products
    int64_t blk_scan = 0, blk_exp = 0, blk_ceil7 = 0, items[2] = {0, 0}, bound_items = 0;
    size_t stats_off = 0, stats_words = 0, counter_off = 0;
    std::vector<Problem> degenerate;  // k == 0 or alpha == 0: C = beta C
    char *desc = nullptr;             // device copy of ops, gm[0], gm[1], crt, bound
    BatchOperand *ops_dev = nullptr;
    BatchGemm *gm_dev[2] = {nullptr, nullptr};
    BatchCrt *crt_dev = nullptr;
    BatchBound *bound_dev = nullptr;
    hipGraphExec_t exec = nullptr;
    double int8_ops = 0.0;
    int64_t sum_m = 0, sum_n = 0, sum_k = 0;

    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (desc) (void)hipFree(desc);
        exec = nullptr;
        desc = nullptr;
    }
};

struct BatchState {
    static constexpr size_t kMaxPlans = 8;
    ozc_batch_policy_t policy{1024, 1, 1};
    std::vector<BatchPlan *> plans;  // most recently used last
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t cap = nullptr;
    int grid[2] = {0, 0};  // resident blocks of the persistent product kernel per tile size
};

void batch_release(ozc_context *h) {
    if (!h->batch) return;
    BatchState *bs = h->batch;
    for (BatchPlan *p : bs->plans) {
        p->release();
        delete p;
    }
    bs->plans.clear();
    if (bs->ws) (void)hipFree(bs->ws);
    if (bs->cap) (void)hipStreamDestroy(bs->cap);
    delete bs;
    h->batch = nullptr;
}

namespace {

BatchState *state_of(ozc_context *h) {
    if (!h->batch) h->batch = new (std::nothrow) BatchState();
    return h->batch;
}

ozc_status_t gather(int count, const ozc_op_t *ta, const ozc_op_t *tb, const int64_t *m,
                    const int64_t *n, const int64_t *k, const double *alpha, const void *const *A,
                    const int64_t *lda, const void *const *B, const int64_t *ldb,
                    const double *beta, void *const *C, const int64_t *ldc, bool need_c,
                    std::vector<Problem> &out) {
    if (count < 0) return OZC_STATUS_INVALID_VALUE;
    if (count == 0) return OZC_STATUS_SUCCESS;
    if (!ta || !tb || !m || !n || !k || !A || !lda || !B || !ldb) return OZC_STATUS_INVALID_VALUE;
    if (need_c && (!alpha || !beta || !C || !ldc)) return OZC_STATUS_INVALID_VALUE;
    out.resize((size_t)count);
    for (int p = 0; p < count; ++p) {
        Problem &q = out[(size_t)p];
        q.ta = ta[p];
        q.tb = tb[p];
        q.m = m[p];
        q.n = n[p];
        q.k = k[p];
        q.lda = lda[p];
        q.ldb = ldb[p];
        q.ldc = need_c ? ldc[p] : (m[p] > 1 ? m[p] : 1);
        q.A = A[p];
        q.B = B[p];
        q.C = need_c ? C[p] : nullptr;
        for (int c = 0; c < 2; ++c) {
            q.alpha[c] = need_c ? alpha[2 * p + c] : (c == 0 ? 1.0 : 0.0);
            q.beta[c] = need_c ? beta[2 * p + c] : 0.0;
        }
        ozc_status_t st = check_args(q.ta, q.tb, q.m, q.n, q.k, q.A, q.lda, q.B, q.ldb, q.C,
                                     q.ldc, !need_c);
        if (st != OZC_STATUS_SUCCESS) return st;
        if (q.k > OZC_MAX_K) return OZC_STATUS_NOT_SUPPORTED;
    }
    return OZC_STATUS_SUCCESS;
}

bool is_degenerate(const Problem &q) {
    return q.k == 0 || (q.alpha[0] == 0.0 && q.alpha[1] == 0.0);
}

std::vector<uint64_t> make_key(const ozc_context *h, bool single, const ozc_batch_policy_t &pol,
                               const std::vector<Problem> &probs, const std::vector<int> &Ns) {
    std::vector<uint64_t> key;
    key.reserve(8 + probs.size() * 16);
    key.push_back(single);
    key.push_back((uint64_t)h->algo);
    key.push_back((uint64_t)h->mode);
    key.push_back((uint64_t)pol.tile_threshold);
    key.push_back((uint64_t)pol.moduli_group);
    key.push_back((uint64_t)pol.use_graph);
    key.push_back(probs.size());
    for (size_t p = 0; p < probs.size(); ++p) {
        const Problem &q = probs[p];
        uint64_t w[16];
        w[0] = (uint64_t)q.ta | ((uint64_t)q.tb << 8);
        w[1] = (uint64_t)q.m;
        w[2] = (uint64_t)q.n;
        w[3] = (uint64_t)q.k;
        w[4] = (uint64_t)q.lda;
        w[5] = (uint64_t)q.ldb;
        w[6] = (uint64_t)q.ldc;
        w[7] = (uint64_t)(uintptr_t)q.A;
        w[8] = (uint64_t)(uintptr_t)q.B;
        w[9] = (uint64_t)(uintptr_t)q.C;
        memcpy(&w[10], q.alpha, 16);
        memcpy(&w[12], q.beta, 16);
        w[14] = (uint64_t)Ns[p];
        w[15] = 0;
        key.insert(key.end(), w, w + 16);
    }
    return key;
}

// Padding, workspace layout and descriptors of a batch (host side only); problem p
// runs with Ns[p] moduli.
ozc_status_t plan_batch(const ozc_context *h, bool single, const ozc_batch_policy_t &pol,
                        const std::vector<Problem> &probs, const std::vector<int> &Ns,
                        BatchPlan &P) {
    P.single = single;
    P.accurate = h->mode == OZC_MODE_ACCURATE;
    P.algo = h->algo == OZC_ALGO_KARATSUBA ? 0 : 1;
    P.planes = P.algo == 0 ? 3 : 2;
    P.group = std::max(1, pol.moduli_group);
    const int nprod = P.algo == 0 ? 3 : 4;

    struct Pad {
        int tile, nmod, nw, nchunks;
        int64_t m_pad, n_pad, k_pad;
        size_t sA, sB, xA, xB, muA, muB, barA, barB, resA, resB, ep;
        size_t p;  // index into probs
    };
    std::vector<Pad> pads;
    size_t stats_words = 0, mu_bytes = 0, bar_bytes = 0, res_bytes = 0, ep_bytes = 0;
    for (size_t p = 0; p < probs.size(); ++p) {
        const Problem &q = probs[p];
        if (q.m == 0 || q.n == 0) continue;
        if (is_degenerate(q)) {
            P.degenerate.push_back(q);
            continue;
        }
        const int N = Ns[p];
        if (N < OZC_MIN_MODULI || N > OZC_MAX_MODULI) return OZC_STATUS_INVALID_VALUE;
        const NTable &th = h->tab_host[(size_t)N - 1];
        const int abits = P.accurate ? th.max_abits_accu : th.max_abits_fast;
        if (abits > kMaxSplitBits) return OZC_STATUS_NOT_SUPPORTED;
        Pad d{};
        d.p = p;
        d.nmod = N;
        d.nw = split_words(abits);
        d.nchunks = th.nchunks;
        d.tile = std::min(q.m, q.n) >= pol.tile_threshold ? 256 : 128;
        d.m_pad = round_up(q.m, gemm_tile_rows(d.tile));
        d.n_pad = round_up(q.n, gemm_tile_cols(d.tile));
        d.k_pad = round_up(q.k, gemm_kstep_for(d.tile));
        d.sA = stats_words;
        stats_words += 2 * (size_t)d.m_pad;  // maxbits, sigma
        d.sB = stats_words;
        stats_words += 2 * (size_t)d.n_pad;
        if (P.accurate) {  // bound maxima X, Y (int32), zeroed with the statistics
            d.xA = stats_words;
            stats_words += ((size_t)d.m_pad + 1) / 2;
            d.xB = stats_words;
            stats_words += ((size_t)d.n_pad + 1) / 2;
            d.barA = bar_bytes;
            bar_bytes = align_up(bar_bytes + 3 * (size_t)d.m_pad * d.k_pad);
            d.barB = bar_bytes;
            bar_bytes = align_up(bar_bytes + 3 * (size_t)d.n_pad * d.k_pad);
        }
        d.muA = mu_bytes;
        mu_bytes = align_up(mu_bytes + 2 * (size_t)d.m_pad);
        d.muB = mu_bytes;
        mu_bytes = align_up(mu_bytes + 2 * (size_t)d.n_pad);
        d.resA = res_bytes;
        res_bytes = align_up(res_bytes + (size_t)N * P.planes * (size_t)d.m_pad * d.k_pad);
        d.resB = res_bytes;
        res_bytes = align_up(res_bytes + (size_t)N * P.planes * (size_t)d.n_pad * d.k_pad);
        d.ep = ep_bytes;
        ep_bytes = align_up(ep_bytes + (size_t)N * 2 * (size_t)d.m_pad * d.n_pad);
        pads.push_back(d);
        P.nmax = std::max(P.nmax, N);
        P.int8_ops += 2.0 * nprod * (double)N * (double)q.m * (double)q.n * (double)q.k;
        P.sum_m += q.m;
        P.sum_n += q.n;
        P.sum_k += q.k;
    }
    size_t off = 0;
    P.counter_off = off;  // 8 work-queue counters per product tile size, 1 for the bounds
    off = align_up(off + 4 * (2 * kBatchQueues + 1));
    P.stats_off = off;
    P.stats_words = stats_words;
    off = align_up(off + 8 * stats_words);
    const size_t mu_off = off;
    off = align_up(off + mu_bytes);
    const size_t bar_off = off;
    off = align_up(off + bar_bytes);
    const size_t res_off = off;
    off = align_up(off + res_bytes);
    const size_t ep_off = off;
    off = align_up(off + ep_bytes);
    P.ws_bytes = off;

    // Descriptors hold offsets from the workspace base (and no tables) until bind().
    P.ops.clear();
    P.crt.clear();
    P.splits.clear();
    P.crts.clear();
    P.bound.clear();
    P.gm[0].clear();
    P.gm[1].clear();
    // operands ordered by word count of the split: one split launch per count
    std::vector<const Pad *> by_nw;
    for (const Pad &d : pads) by_nw.push_back(&d);
    std::stable_sort(by_nw.begin(), by_nw.end(), [](const Pad *x, const Pad *y) { return x->nw < y->nw; });
    for (const Pad *dp : by_nw) {
        const Pad &d = *dp;
        const Problem &q = probs[d.p];
        if (P.splits.empty() || P.splits.back().param != 32 * d.nw - 1)
            P.splits.push_back({(int)P.ops.size(), 0, 0, 32 * d.nw - 1});
        BatchPlan::Range &sr = P.splits.back();
        BatchOperand a{}, b{};
        a.v = view_A(q.A, q.ta, q.m, q.k, q.lda);
        b.v = view_B(q.B, q.tb, q.n, q.k, q.ldb);
        a.maxbits = (uint64_t *)(uintptr_t)(P.stats_off + 8 * d.sA);
        a.sigma = (uint64_t *)(uintptr_t)(P.stats_off + 8 * (d.sA + d.m_pad));
        b.maxbits = (uint64_t *)(uintptr_t)(P.stats_off + 8 * d.sB);
        b.sigma = (uint64_t *)(uintptr_t)(P.stats_off + 8 * (d.sB + d.n_pad));
        a.mu = (int16_t *)(uintptr_t)(mu_off + d.muA);
        b.mu = (int16_t *)(uintptr_t)(mu_off + d.muB);
        a.res = (int8_t *)(uintptr_t)(res_off + d.resA);
        b.res = (int8_t *)(uintptr_t)(res_off + d.resB);
        a.rows_pad = d.m_pad;
        b.rows_pad = d.n_pad;
        a.k_pad = b.k_pad = d.k_pad;
        a.nmod = b.nmod = d.nmod;
        if (P.accurate) {
            a.X = (int32_t *)(uintptr_t)(P.stats_off + 8 * d.xA);
            b.X = (int32_t *)(uintptr_t)(P.stats_off + 8 * d.xB);
            a.bar = (int8_t *)(uintptr_t)(bar_off + d.barA);
            b.bar = (int8_t *)(uintptr_t)(bar_off + d.barB);
            BatchBound bb{};
            bb.b = BoundArgs{a.bar, b.bar, d.m_pad, d.n_pad, d.k_pad, a.X, b.X, 128};
            bb.item0 = P.bound_items;
            bb.TR = (int32_t)(d.m_pad / 128);
            bb.TC = (int32_t)(d.n_pad / 128);
            P.bound_items += (int64_t)bb.TR * bb.TC;
            P.bound.push_back(bb);
        }
        for (BatchOperand *o : {&a, &b}) {
            if (P.accurate) {
                o->blk_ceil7 = P.blk_ceil7;
                P.blk_ceil7 += batch_ceil7_blocks(o->rows_pad, o->k_pad);
            }
            o->blk_scan = P.blk_scan;
            P.blk_scan += batch_scan_blocks(o->v);
            o->blk_exp = P.blk_exp;
            P.blk_exp += batch_exp_blocks(o->rows_pad);
            o->blk_split = sr.blocks;
            sr.blocks += batch_split_blocks(o->rows_pad, o->k_pad);
            ++sr.count;
            P.ops.push_back(*o);
        }
        BatchGemm g{};
        g.A = a.res;
        g.B = b.res;
        g.eprime = (int8_t *)(uintptr_t)(ep_off + d.ep);
        g.m_pad = d.m_pad;
        g.n_pad = d.n_pad;
        g.k_pad = d.k_pad;
        g.TR = (int32_t)(d.m_pad / gemm_tile_rows(d.tile));
        g.TC = (int32_t)(d.n_pad / gemm_tile_cols(d.tile));
        g.nmod = d.nmod;
        P.gm[d.tile == 256 ? 0 : 1].push_back(g);
    }
    // reconstruction ordered by the chunk count of P: one CRT launch per count
    std::vector<const Pad *> by_chunks;
    for (const Pad &d : pads) by_chunks.push_back(&d);
    std::stable_sort(by_chunks.begin(), by_chunks.end(),
                     [](const Pad *x, const Pad *y) { return x->nchunks < y->nchunks; });
    for (const Pad *dp : by_chunks) {
        const Pad &d = *dp;
        const Problem &q = probs[d.p];
        if (P.crts.empty() || P.crts.back().param != d.nchunks)
            P.crts.push_back({(int)P.crt.size(), 0, 0, d.nchunks});
        BatchPlan::Range &cr = P.crts.back();
        BatchCrt c{};
        c.a.eprime = (const int8_t *)(uintptr_t)(ep_off + d.ep);
        c.a.m = q.m;
        c.a.n = q.n;
        c.a.m_pad = d.m_pad;
        c.a.n_pad = d.n_pad;
        c.a.nmod = d.nmod;
        c.a.nchunks = d.nchunks;
        c.a.tab = nullptr;  // bound later
        c.a.mu = (const int16_t *)(uintptr_t)(mu_off + d.muA);
        c.a.nu = (const int16_t *)(uintptr_t)(mu_off + d.muB);
        c.a.alpha_r = q.alpha[0];
        c.a.alpha_i = q.alpha[1];
        c.a.beta_r = q.beta[0];
        c.a.beta_i = q.beta[1];
        c.a.C = q.C;
        c.a.ldc = q.ldc;
        c.a.single = single;
        c.blk0 = cr.blocks;
        cr.blocks += batch_crt_blocks(q.m, q.n);
        ++cr.count;
        P.crt.push_back(c);
    }
    // largest k first, so that the long items start early and the short ones fill the tail
    for (int t = 0; t < 2; ++t) {
        std::stable_sort(P.gm[t].begin(), P.gm[t].end(),
                         [](const BatchGemm &x, const BatchGemm &y) { return x.k_pad > y.k_pad; });
        P.items[t] = 0;
        for (BatchGemm &g : P.gm[t]) {
            g.item0 = P.items[t];
            P.items[t] += (int64_t)((g.nmod + P.group - 1) / P.group) * g.TR * g.TC;
        }
    }
    bool too_big = P.blk_scan >= ((int64_t)1 << 31) || P.items[0] >= ((int64_t)1 << 32) ||
                   P.items[1] >= ((int64_t)1 << 32) || P.blk_ceil7 >= ((int64_t)1 << 31) ||
                   P.bound_items >= ((int64_t)1 << 32);
    for (const BatchPlan::Range &r : P.splits) too_big = too_big || r.blocks >= ((int64_t)1 << 31);
    for (const BatchPlan::Range &r : P.crts) too_big = too_big || r.blocks >= ((int64_t)1 << 31);
    return too_big ? OZC_STATUS_NOT_SUPPORTED : OZC_STATUS_SUCCESS;
}

// Turn workspace offsets into addresses and copy the descriptors to the device.
ozc_status_t bind(const ozc_context *h, BatchPlan &P, char *ws) {
    const uintptr_t base = (uintptr_t)ws;
    for (BatchOperand &o : P.ops) {
        o.maxbits = (uint64_t *)(base + (uintptr_t)o.maxbits);
        o.sigma = (uint64_t *)(base + (uintptr_t)o.sigma);
        o.mu = (int16_t *)(base + (uintptr_t)o.mu);
        o.res = (int8_t *)(base + (uintptr_t)o.res);
        o.tab = h->tab_dev + (o.nmod - 1);
        if (P.accurate) {
            o.X = (int32_t *)(base + (uintptr_t)o.X);
            o.bar = (int8_t *)(base + (uintptr_t)o.bar);
        }
    }
    for (BatchBound &bb : P.bound) {
        bb.b.A = (const int8_t *)(base + (uintptr_t)bb.b.A);
        bb.b.B = (const int8_t *)(base + (uintptr_t)bb.b.B);
        bb.b.X = (int32_t *)(base + (uintptr_t)bb.b.X);
        bb.b.Y = (int32_t *)(base + (uintptr_t)bb.b.Y);
    }
    for (int t = 0; t < 2; ++t)
        for (BatchGemm &g : P.gm[t]) {
            g.A = (const int8_t *)(base + (uintptr_t)g.A);
            g.B = (const int8_t *)(base + (uintptr_t)g.B);
            g.eprime = (int8_t *)(base + (uintptr_t)g.eprime);
            g.tab = h->tab_dev + (g.nmod - 1);
        }
    for (BatchCrt &c : P.crt) {
        c.a.eprime = (const int8_t *)(base + (uintptr_t)c.a.eprime);
        c.a.mu = (const int16_t *)(base + (uintptr_t)c.a.mu);
        c.a.nu = (const int16_t *)(base + (uintptr_t)c.a.nu);
        c.a.tab = h->tab_dev + (c.a.nmod - 1);
    }
    const size_t b_ops = align_up(sizeof(BatchOperand) * P.ops.size());
    const size_t b_g0 = align_up(sizeof(BatchGemm) * P.gm[0].size());
    const size_t b_g1 = align_up(sizeof(BatchGemm) * P.gm[1].size());
    const size_t b_crt = align_up(sizeof(BatchCrt) * P.crt.size());
    const size_t b_bound = align_up(sizeof(BatchBound) * P.bound.size());
    const size_t total = b_ops + b_g0 + b_g1 + b_crt + b_bound;
    if (total == 0) return OZC_STATUS_SUCCESS;
    std::vector<char> host(total, 0);
    memcpy(host.data(), P.ops.data(), sizeof(BatchOperand) * P.ops.size());
    memcpy(host.data() + b_ops, P.gm[0].data(), sizeof(BatchGemm) * P.gm[0].size());
    memcpy(host.data() + b_ops + b_g0, P.gm[1].data(), sizeof(BatchGemm) * P.gm[1].size());
    memcpy(host.data() + b_ops + b_g0 + b_g1, P.crt.data(), sizeof(BatchCrt) * P.crt.size());
    memcpy(host.data() + b_ops + b_g0 + b_g1 + b_crt, P.bound.data(),
           sizeof(BatchBound) * P.bound.size());
    if (hipMalloc(&P.desc, total) != hipSuccess) {
        P.desc = nullptr;
        (void)hipGetLastError();
        return OZC_STATUS_ALLOC_FAILED;
    }
    OZC_TRY(hipMemcpy(P.desc, host.data(), total, hipMemcpyHostToDevice));
    P.ops_dev = (BatchOperand *)P.desc;
    P.gm_dev[0] = (BatchGemm *)(P.desc + b_ops);
    P.gm_dev[1] = (BatchGemm *)(P.desc + b_ops + b_g0);
    P.crt_dev = (BatchCrt *)(P.desc + b_ops + b_g0 + b_g1);
    P.bound_dev = (BatchBound *)(P.desc + b_ops + b_g0 + b_g1 + b_crt);
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ensure_batch_ws(ozc_context *h, BatchState *bs, size_t bytes) {
    if (bytes <= bs->ws_bytes) return OZC_STATUS_SUCCESS;
    OZC_TRY(hipStreamSynchronize(h->stream));
    for (BatchPlan *p : bs->plans) {  // their graphs point into the old workspace
        p->release();
        delete p;
    }
    bs->plans.clear();
    if (bs->ws) (void)hipFree(bs->ws);
    bs->ws = nullptr;
    bs->ws_bytes = 0;
    if (hipMalloc(&bs->ws, bytes) != hipSuccess) {
        bs->ws = nullptr;
        (void)hipGetLastError();
        return OZC_STATUS_ALLOC_FAILED;
    }
    bs->ws_bytes = bytes;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t grid_sizes(ozc_context *h, BatchState *bs) {
    if (bs->grid[0] > 0) return OZC_STATUS_SUCCESS;
    int cus = 0;
    OZC_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    bs->grid[0] = cus * batch_gemm_blocks_per_cu(256);
    bs->grid[1] = cus * batch_gemm_blocks_per_cu(128);
    return OZC_STATUS_SUCCESS;
}

enum { PH_PREP = 1, PH_GEMM = 2, PH_CRT = 4, PH_ALL = 7 };

// The launch sequence of a bound plan (no host synchronisation, no memset nodes).
ozc_status_t launch_batch(ozc_context *h, BatchState *bs, const BatchPlan &P, char *ws,
                          hipStream_t s, int phases, int group) {
    uint32_t *counters = (uint32_t *)(ws + P.counter_off);
    const int nops = (int)P.ops.size();
    if (phases & PH_PREP) {
        OZC_TRY(launch_fill_u64(h->status_dev, 1, 0, s));
        OZC_TRY(launch_fill_u64((uint64_t *)(ws + P.stats_off), (int64_t)P.stats_words, 0, s));
        OZC_TRY(launch_batch_scan(P.ops_dev, nops, P.blk_scan, P.single, 0, s));
        if (P.accurate) {
            OZC_TRY(launch_batch_ceil7(P.ops_dev, nops, P.blk_ceil7, P.single, s));
            uint32_t *bound_counter = counters + 2 * kBatchQueues;
            OZC_TRY(launch_fill_u32(bound_counter, 1, 0, s));
            OZC_TRY(launch_batch_bound(P.bound_dev, (int)P.bound.size(), P.bound_items, bound_counter, s));
            OZC_TRY(launch_batch_accu_exponents(P.ops_dev, nops, P.blk_exp, (uint32_t *)h->status_dev, s));
        } else {
            OZC_TRY(launch_batch_scan(P.ops_dev, nops, P.blk_scan, P.single, 1, s));
            OZC_TRY(launch_batch_fast_exponents(P.ops_dev, nops, P.blk_exp, (uint32_t *)h->status_dev, s));
        }
        for (const BatchPlan::Range &r : P.splits)
            OZC_TRY(launch_batch_split(P.ops_dev + r.first, r.count, r.blocks, P.single, P.planes,
                                       r.param, s));
    }
    if (phases & PH_GEMM) {
        OZC_TRY(launch_fill_u32(counters, 2 * kBatchQueues, 0, s));
        const int tiles[2] = {256, 128};
        for (int t = 0; t < 2; ++t) {
            if (P.items[t] == 0) continue;
            OZC_TRY(launch_batch_gemm(P.gm_dev[t], (int)P.gm[t].size(), P.items[t], tiles[t], group,
                                      P.algo, counters + kBatchQueues * t, bs->grid[t], s));
        }
    }
    if (phases & PH_CRT) {
        for (const BatchPlan::Range &r : P.crts)
            OZC_TRY(launch_batch_crt(P.crt_dev + r.first, r.count, r.blocks, r.param, P.single, s));
        for (const Problem &q : P.degenerate)
            OZC_TRY(launch_scale_c(q.C, q.m, q.n, q.ldc, P.single, q.alpha[0], q.alpha[1], q.beta[0],
                                   q.beta[1], s));
    }
    return OZC_STATUS_SUCCESS;
}

ozc_status_t record_graph(ozc_context *h, BatchState *bs, BatchPlan &P) {
    if (!bs->cap) OZC_TRY(hipStreamCreateWithFlags(&bs->cap, hipStreamNonBlocking));
    OZC_TRY(hipStreamBeginCapture(bs->cap, hipStreamCaptureModeThreadLocal));
    ozc_status_t st = launch_batch(h, bs, P, bs->ws, bs->cap, PH_ALL, P.group);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(bs->cap, &g);
    if (st == OZC_STATUS_SUCCESS && e != hipSuccess) st = OZC_STATUS_HIP_ERROR;
    if (st == OZC_STATUS_SUCCESS && hipGraphInstantiate(&P.exec, g, nullptr, nullptr, 0) != hipSuccess) {
        P.exec = nullptr;
        st = OZC_STATUS_HIP_ERROR;
    }
    if (g) (void)hipGraphDestroy(g);
    return st;
}

// One batch, problem p with Ns[p] moduli: plan lookup (or build and record), launch.
ozc_status_t run_plan(ozc_context *h, BatchState *bs, bool single,
                      const std::vector<Problem> &probs, const std::vector<int> &Ns) {
    const ozc_batch_policy_t pol = bs->policy;
    std::vector<uint64_t> key = make_key(h, single, pol, probs, Ns);
    BatchPlan *P = nullptr;
    for (size_t i = 0; i < bs->plans.size(); ++i)
        if (bs->plans[i]->key == key) {
            P = bs->plans[i];
            bs->plans.erase(bs->plans.begin() + (long)i);
            bs->plans.push_back(P);
            break;
        }
    if (!P) {
        BatchPlan *Q = new (std::nothrow) BatchPlan();
        if (!Q) return OZC_STATUS_ALLOC_FAILED;
        ozc_status_t st = plan_batch(h, single, pol, probs, Ns, *Q);
        if (st == OZC_STATUS_SUCCESS) st = ensure_batch_ws(h, bs, Q->ws_bytes);
        if (st == OZC_STATUS_SUCCESS) st = bind(h, *Q, bs->ws);
        if (st == OZC_STATUS_SUCCESS && pol.use_graph) st = record_graph(h, bs, *Q);
        if (st != OZC_STATUS_SUCCESS) {
            Q->release();
            delete Q;
            return st;
        }
        Q->key = std::move(key);
        if (bs->plans.size() >= BatchState::kMaxPlans) {  // evict the least recently used
            OZC_TRY(hipStreamSynchronize(h->stream));
            bs->plans.front()->release();
            delete bs->plans.front();
            bs->plans.erase(bs->plans.begin());
        }
        bs->plans.push_back(Q);
        P = Q;
    }
    if (P->exec) OZC_TRY(hipGraphLaunch(P->exec, h->stream));
    else {
        ozc_status_t st = launch_batch(h, bs, *P, bs->ws, h->stream, PH_ALL, P->group);
        if (st != OZC_STATUS_SUCCESS) return st;
    }
    h->last.m += P->sum_m;
    h->last.n += P->sum_n;
    h->last.k += P->sum_k;
    h->last.workspace = std::max(h->last.workspace, P->ws_bytes);
    h->last.int8_ops += P->int8_ops;
    h->last.num_moduli = std::max(h->last.num_moduli, P->nmax);
    return OZC_STATUS_SUCCESS;
}

// A batch with the Freivalds check per problem (see ozc_set_verify): problems that fail
// are rerun as a smaller batch with two more moduli, up to OZC_MAX_MODULI.
// Workspace of one problem's check: its vectors (carve_check) with scratch for the
// partial sums of the gemvs that run together (C_in x, op(B) x and C x), later reused
// by op(A) y.
size_t problem_check_bytes(const Problem &q, bool has_cin) {
    size_t first = align_up(gemv_scratch_bytes(q.m, q.n));  // C x
    if (has_cin) first += align_up(gemv_scratch_bytes(q.m, q.n));
    if (q.tb == OZC_OP_N) first += align_up(gemv_scratch_bytes(q.k, q.n));
    const size_t second = q.ta == OZC_OP_N ? gemv_scratch_bytes(q.m, q.k) : 0;
    return align_up(check_bytes(q.m, q.k, std::max(first, second)));
}

ozc_status_t run_plan_verified(ozc_context *h, BatchState *bs, bool single,
                               const std::vector<Problem> &probs, std::vector<int> Ns) {
    hipStream_t s = h->stream;
    const size_t es = single ? 8 : 16;
    auto has_cin = [&](const Problem &q) { return q.beta[0] != 0.0 || q.beta[1] != 0.0; };
    std::vector<size_t> chk;                    // checked problems
    std::vector<size_t> slot(probs.size(), 0);  // their index in chk
    std::vector<size_t> cin_off(probs.size(), 0), chk_off(probs.size(), 0);
    size_t cin_bytes = 0, chk_bytes = 0;
    for (size_t p = 0; p < probs.size(); ++p) {
        const Problem &q = probs[p];
        if (q.m == 0 || q.n == 0 || is_degenerate(q)) continue;
        slot[p] = chk.size();
        chk.push_back(p);
        chk_off[p] = chk_bytes;
        chk_bytes += problem_check_bytes(q, has_cin(q));
        if (has_cin(q)) {
            cin_off[p] = cin_bytes;
            cin_bytes = align_up(cin_bytes + es * (size_t)q.m * (size_t)q.n);
        }
    }
    // words (max ratio, failed rows) per checked problem | task descriptors | per-problem
    // check buffers | saved C_in
    const size_t nchk = std::max<size_t>(1, chk.size());
    const size_t o_desc = align_up(16 * nchk);
    const size_t desc_bytes = align_up(nchk * (4 * sizeof(GemvTask) + sizeof(RowsTask)));
    const size_t o_chk = o_desc + desc_bytes;
    const size_t o_cin = o_chk + chk_bytes;
    ozc_status_t st = ensure_vws(h, o_cin + cin_bytes);
    if (st != OZC_STATUS_SUCCESS) return st;
    char *vw = (char *)h->vws;
    unsigned long long *words = (unsigned long long *)vw;
    for (size_t p : chk) {  // C_in for the check and for reruns
        const Problem &q = probs[p];
        if (has_cin(q))
            OZC_TRY(hipMemcpy2DAsync(vw + o_cin + cin_off[p], es * q.m, q.C, es * q.ldc, es * q.m, q.n,
                                     hipMemcpyDeviceToDevice, s));
    }
    st = run_plan(h, bs, single, probs, Ns);
    if (st != OZC_STATUS_SUCCESS) return st;
    std::vector<size_t> todo = chk;
    std::vector<double> ratio(chk.size(), 0.0);
    std::vector<int64_t> failed(chk.size(), 0);
    int rounds = 0;
    const uint64_t seed = h->verify_seed;
    for (;;) {
        // The checks of all pending problems in five launches: w = C x, y = op(B) x and
        // v = C_in x together, then z = op(A) y, then the row tests.
        std::vector<GemvTask> first, second;
        std::vector<RowsTask> rows;
        int64_t nb1[3] = {0, 0, 0}, nb2[3] = {0, 0, 0}, nbr = 0;
        for (size_t p : todo) {
            const Problem &q = probs[p];
            const CheckBufs b = carve_check(vw + o_chk + chk_off[p], q.m, q.k);
            char *sc = (char *)b.scratch;
            first.push_back(make_gemv_task(q.C, 0, q.m, q.n, q.ldc, nullptr, nullptr, nullptr, seed, b.w,
                                           b.wl, b.wa, sc, nb1));
            sc += align_up(gemv_scratch_bytes(q.m, q.n));
            if (has_cin(q)) {
                first.push_back(make_gemv_task(vw + o_cin + cin_off[p], 0, q.m, q.n, q.m, nullptr, nullptr,
                                               nullptr, seed, b.v, b.vl, b.va, sc, nb1));
                sc += align_up(gemv_scratch_bytes(q.m, q.n));
            }
            if (q.tb == OZC_OP_N)
                first.push_back(make_gemv_task(q.B, 0, q.k, q.n, q.ldb, nullptr, nullptr, nullptr, seed,
                                               b.y, b.yl, b.ya, sc, nb1));
            else
                first.push_back(make_gemv_task(q.B, (int)q.tb, q.n, q.k, q.ldb, nullptr, nullptr, nullptr,
                                               seed, b.y, b.yl, b.ya, nullptr, nb1));
            if (q.ta == OZC_OP_N)
                second.push_back(make_gemv_task(q.A, 0, q.m, q.k, q.lda, b.y, b.yl, b.ya, 0, b.z, b.zl,
                                                b.za, b.scratch, nb2));
            else
                second.push_back(make_gemv_task(q.A, (int)q.ta, q.k, q.m, q.lda, b.y, b.yl, b.ya, 0, b.z,
                                                b.zl, b.za, nullptr, nb2));
            RowsTask r{};
            r.w = b.w;
            r.wl = b.wl;
            r.wa = b.wa;
            r.z = b.z;
            r.zl = b.zl;
            r.za = b.za;
            if (has_cin(q)) {
                r.v = b.v;
                r.vl = b.vl;
                r.va = b.va;
            }
            r.m = q.m;
            r.ar = q.alpha[0];
            r.ai = q.alpha[1];
            r.br = q.beta[0];
            r.bi = q.beta[1];
            check_tolerances(h, single, q.n, q.k, &r.rel, &r.gam);
            r.worst = words + 2 * slot[p];
            r.b0 = nbr;
            nbr += rows_task_blocks(q.m);
            rows.push_back(r);
        }
        if (std::max({nb1[0], nb1[1], nb1[2], nb2[0], nb2[1], nb2[2], nbr}) > INT32_MAX)
            return OZC_STATUS_NOT_SUPPORTED;
        // descriptors: first | second | rows (the host copy lives until the synchronisation)
        std::vector<char> desc(first.size() * sizeof(GemvTask) + second.size() * sizeof(GemvTask) +
                               rows.size() * sizeof(RowsTask));
        memcpy(desc.data(), first.data(), first.size() * sizeof(GemvTask));
        memcpy(desc.data() + first.size() * sizeof(GemvTask), second.data(),
               second.size() * sizeof(GemvTask));
        memcpy(desc.data() + (first.size() + second.size()) * sizeof(GemvTask), rows.data(),
               rows.size() * sizeof(RowsTask));
        const GemvTask *d_first = (const GemvTask *)(vw + o_desc);
        const GemvTask *d_second = d_first + first.size();
        const RowsTask *d_rows = (const RowsTask *)(d_second + second.size());
        OZC_TRY(hipMemcpyAsync(vw + o_desc, desc.data(), desc.size(), hipMemcpyHostToDevice, s));
        OZC_TRY(launch_fill_u64((uint64_t *)words, 2 * (int64_t)nchk, 0, s));
        OZC_TRY(launch_batch_gemv(d_first, (int)first.size(), nb1, single, s));
        OZC_TRY(launch_batch_gemv(d_second, (int)second.size(), nb2, single, s));
        OZC_TRY(launch_batch_rows(d_rows, (int)rows.size(), nbr, s));
        std::vector<unsigned long long> host(2 * std::max<size_t>(1, chk.size()), 0);
        OZC_TRY(hipMemcpyAsync(host.data(), words, 16 * chk.size(), hipMemcpyDeviceToHost, s));
        OZC_TRY(hipStreamSynchronize(s));
        std::vector<size_t> again;
        bool stuck = false;
        for (size_t p : todo) {
            const size_t i = slot[p];
            memcpy(&ratio[i], &host[2 * i], sizeof(double));
            failed[i] = (int64_t)host[2 * i + 1];
            if (failed[i] == 0) continue;
            if (h->escalate && Ns[p] < OZC_MAX_MODULI) again.push_back(p);
            else stuck = true;
        }
        if (stuck) st = OZC_STATUS_VERIFY_FAILED;
        if (again.empty()) break;
        ++rounds;
        std::vector<Problem> sub;
        std::vector<int> subN;
        for (size_t p : again) {
            const Problem &q = probs[p];
            Ns[p] = std::min(OZC_MAX_MODULI, Ns[p] + 2);
            if (has_cin(q))
                OZC_TRY(hipMemcpy2DAsync(q.C, es * q.ldc, vw + o_cin + cin_off[p], es * q.m, es * q.m,
                                         q.n, hipMemcpyDeviceToDevice, s));
            sub.push_back(q);
            subN.push_back(Ns[p]);
        }
        ozc_status_t sr = run_plan(h, bs, single, sub, subN);
        if (sr != OZC_STATUS_SUCCESS) return sr;
        todo = again;
    }
    h->last.verified = 1;
    h->last.escalations = rounds;
    h->last.verify_failed_rows = 0;
    h->last.verify_ratio = 0.0;
    for (size_t i = 0; i < chk.size(); ++i) {
        h->last.verify_failed_rows += failed[i];
        h->last.verify_ratio = std::max(h->last.verify_ratio, ratio[i]);
    }
    return st;
}

ozc_status_t run_vbatched(ozc_context *h, bool single, int count, const ozc_op_t *ta,
                          const ozc_op_t *tb, const int64_t *m, const int64_t *n,
                          const int64_t *k, const double *alpha, const void *const *A,
                          const int64_t *lda, const void *const *B, const int64_t *ldb,
                          const double *beta, void *const *C, const int64_t *ldc) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    std::vector<Problem> probs;
    ozc_status_t st = gather(count, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, true, probs);
    if (st != OZC_STATUS_SUCCESS) return st;
    OZC_TRY(hipSetDevice(h->device));
    BatchState *bs = state_of(h);
    if (!bs) return OZC_STATUS_ALLOC_FAILED;
    OZC_TRY(launch_fill_u64(h->status_dev, 1, 0, h->stream));
    h->last = ozc_info_t{};
    h->last.num_moduli = h->nmod;
    h->last.mode = h->mode;
    h->last.algo = h->algo;
    if (probs.empty()) return OZC_STATUS_SUCCESS;
    st = grid_sizes(h, bs);
    if (st != OZC_STATUS_SUCCESS) return st;
    std::vector<int> Ns(probs.size(), h->nmod);
    if (!h->auto_n)
        return h->verify ? run_plan_verified(h, bs, single, probs, Ns)
                         : run_plan(h, bs, single, probs, Ns);

    // Learned N per problem (complex64: the fixed count), all in one batch.
    h->last.num_moduli = 0;
    if (single) {
        std::fill(Ns.begin(), Ns.end(), 9);
    } else {
        std::vector<OperandView> va, vb;
        std::vector<size_t> which;
        for (size_t p = 0; p < probs.size(); ++p) {
            const Problem &q = probs[p];
            if (q.m == 0 || q.n == 0 || is_degenerate(q)) continue;
            va.push_back(view_A(q.A, q.ta, q.m, q.k, q.lda));
            vb.push_back(view_B(q.B, q.tb, q.n, q.k, q.ldb));
            which.push_back(p);
        }
        std::vector<int> pred;
        st = predict_moduli_many(h, single, va, vb, pred);
        if (st != OZC_STATUS_SUCCESS) return st;
        for (size_t i = 0; i < which.size(); ++i) Ns[which[i]] = pred[i];
    }
    // num_moduli: the largest count used
    return h->verify ? run_plan_verified(h, bs, single, probs, Ns) : run_plan(h, bs, single, probs, Ns);
}

// Median of the product phase over `reps` runs.
ozc_status_t time_gemm(ozc_context *h, BatchState *bs, const BatchPlan &P, int group, int reps,
                       float *ms) {
    hipEvent_t e0, e1;
    OZC_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return OZC_STATUS_HIP_ERROR;
    }
    std::vector<float> t;
    ozc_status_t st = launch_batch(h, bs, P, bs->ws, h->stream, PH_GEMM, group);  // warm-up
    for (int r = 0; r < reps && st == OZC_STATUS_SUCCESS; ++r) {
        float x = 0.f;
        if (hipEventRecord(e0, h->stream) != hipSuccess) st = OZC_STATUS_HIP_ERROR;
        if (st == OZC_STATUS_SUCCESS) st = launch_batch(h, bs, P, bs->ws, h->stream, PH_GEMM, group);
        if (st == OZC_STATUS_SUCCESS && (hipEventRecord(e1, h->stream) != hipSuccess ||
                                         hipEventSynchronize(e1) != hipSuccess ||
                                         hipEventElapsedTime(&x, e0, e1) != hipSuccess))
            st = OZC_STATUS_HIP_ERROR;
        t.push_back(x);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != OZC_STATUS_SUCCESS) return st;
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return OZC_STATUS_SUCCESS;
}

}  // namespace

}  // namespace ozc

using namespace ozc;

extern "C" {

ozc_status_t ozc_zgemm_vbatched(ozc_handle_t h, int count, const ozc_op_t *transa,
                                const ozc_op_t *transb, const int64_t *m, const int64_t *n,
                                const int64_t *k, const double *alpha, const void *const *A,
                                const int64_t *lda, const void *const *B, const int64_t *ldb,
                                const double *beta, void *const *C, const int64_t *ldc) {
    return run_vbatched(h, false, count, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

ozc_status_t ozc_cgemm_vbatched(ozc_handle_t h, int count, const ozc_op_t *transa,
                                const ozc_op_t *transb, const int64_t *m, const int64_t *n,
                                const int64_t *k, const float *alpha, const void *const *A,
                                const int64_t *lda, const void *const *B, const int64_t *ldb,
                                const float *beta, void *const *C, const int64_t *ldc) {
    if (count < 0) return OZC_STATUS_INVALID_VALUE;
    if (count > 0 && (!alpha || !beta)) return OZC_STATUS_INVALID_VALUE;
    std::vector<double> al((size_t)2 * (count > 0 ? count : 0)), be(al.size());
    for (size_t i = 0; i < al.size(); ++i) {
        al[i] = (double)alpha[i];
        be[i] = (double)beta[i];
    }
    return run_vbatched(h, true, count, transa, transb, m, n, k, al.data(), A, lda, B, ldb,
                        be.data(), C, ldc);
}

ozc_status_t ozc_set_batch_policy(ozc_handle_t h, const ozc_batch_policy_t *policy) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (!policy || policy->tile_threshold < 0 || policy->moduli_group < 1)
        return OZC_STATUS_INVALID_VALUE;
    BatchState *bs = state_of(h);
    if (!bs) return OZC_STATUS_ALLOC_FAILED;
    bs->policy = *policy;
    if (bs->policy.tile_threshold == 0) bs->policy.tile_threshold = 1024;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_get_batch_policy(ozc_handle_t h, ozc_batch_policy_t *policy) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    if (!policy) return OZC_STATUS_INVALID_VALUE;
    BatchState *bs = state_of(h);
    if (!bs) return OZC_STATUS_ALLOC_FAILED;
    *policy = bs->policy;
    return OZC_STATUS_SUCCESS;
}

ozc_status_t ozc_batch_tune(ozc_handle_t h, int single, int count, const ozc_op_t *transa,
                            const ozc_op_t *transb, const int64_t *m, const int64_t *n,
                            const int64_t *k, const void *const *A, const int64_t *lda,
                            const void *const *B, const int64_t *ldb, ozc_batch_policy_t *chosen) {
    if (!h) return OZC_STATUS_INVALID_HANDLE;
    std::vector<Problem> probs;
    ozc_status_t st = gather(count, transa, transb, m, n, k, nullptr, A, lda, B, ldb, nullptr,
                             nullptr, nullptr, false, probs);
    if (st != OZC_STATUS_SUCCESS) return st;
    OZC_TRY(hipSetDevice(h->device));
    BatchState *bs = state_of(h);
    if (!bs) return OZC_STATUS_ALLOC_FAILED;
    st = grid_sizes(h, bs);
    if (st != OZC_STATUS_SUCCESS) return st;
    ozc_batch_policy_t best = bs->policy;
    float best_ms = -1.f;
    const int thresholds[] = {256, 512, 1024, 2048, 1 << 30};
    const int groups[] = {1, 2, 4, h->nmod};
    for (int thr : thresholds) {
        ozc_batch_policy_t pol = bs->policy;
        pol.tile_threshold = thr;
        pol.moduli_group = 1;
        BatchPlan P;
        st = plan_batch(h, single != 0, pol, probs, std::vector<int>(probs.size(), h->nmod), P);
        if (st == OZC_STATUS_SUCCESS) st = ensure_batch_ws(h, bs, P.ws_bytes);
        if (st == OZC_STATUS_SUCCESS) st = bind(h, P, bs->ws);
        if (st == OZC_STATUS_SUCCESS) st = launch_batch(h, bs, P, bs->ws, h->stream, PH_PREP, 1);
        for (int g : groups) {
            if (st != OZC_STATUS_SUCCESS) break;
            if (g < 1 || g > h->nmod) continue;
            float ms = 0.f;
            st = time_gemm(h, bs, P, g, 3, &ms);
            if (st == OZC_STATUS_SUCCESS && (best_ms < 0.f || ms < best_ms)) {
                best_ms = ms;
                best = pol;
                best.moduli_group = g;
            }
        }
        if (hipStreamSynchronize(h->stream) != hipSuccess && st == OZC_STATUS_SUCCESS)
            st = OZC_STATUS_HIP_ERROR;
        P.release();
        if (st != OZC_STATUS_SUCCESS) return st;
    }
    bs->policy = best;
    if (chosen) *chosen = best;
    return OZC_STATUS_SUCCESS;
}

}  // extern "C"
