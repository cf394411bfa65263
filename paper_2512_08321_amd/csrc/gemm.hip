// Per-modulus complex INT8 products on the gfx950 matrix cores with INT32
// accumulation (Section III-A; Algorithm 1 Step V-iii/iv).
//
// One block computes a TM x TN output tile of one modulus l with WM x WN
// waves; each wave owns (BM*32) x (BN*32) outputs as BM x BN blocks of
// v_mfma_i32_32x32x32_i8 (large problems: 256 x 256 tiles, 8 waves of
// 128 x 64, two waves per SIMD; small problems: 128 x 128, 4 waves of
// 64 x 64).  The products of the chosen algorithm run one after another over
// the same tile, each as a k-loop over a ring of LDS buffers that the load
// units fill straight from global memory a few 64-wide k-slabs ahead of the
// matrix cores (one barrier per k-slab).  Between products
// the INT32 accumulators are reduced to symmetric residues in registers; one
// packed INT8 carry per output survives to the next product, and E'_R, E'_I
// are stored as soon as they are final, so only INT8 data leaves the chip:
//   Karatsuba (eq. (10)): D = R.R, E = I.I, F = S.S (S = reduced R + I):
//                         E'_R = mod(D - E), E'_I = mod(F - mod(D + E))
//   expanded  (eq. (7)):  E'_R = mod(RR - II), E'_I = mod(RI + IR)
// A third plan computes the accurate-mode bound product (Section III-B):
//   Cbar_I = Abar_I Bbar_R + Abar_R Bbar_I, Cbar_R = Cbar_I + (Abar_R - Abar_I)(Bbar_R - Bbar_I),
// folded on the fly into row and column maxima (Cbar is never stored).
// Real matrices (Algorithm 1 as stated for real A, B) take one product per
// modulus, E' = mod(A'_l B'_l), and one real bound product Abar Bbar.
//
// Block order: block ids are dealt round-robin to the 8 XCDs; ids are
// remapped so that each XCD walks its own contiguous part of the
// (modulus, tile) sequence, tiles grouped 4 rows at a time, so that the
// blocks resident on one XCD share A and B panels in that XCD's L2.
//
// MFMA operand layout: lane l of a 32x32x32 instruction supplies 16 bytes of
// row (l mod 32) of the A block and of column (l mod 32) of the B block, at
// k-offset 16 * (l / 32); both operands use the same k assignment, so the
// product does not depend on how the hardware orders k inside the 32-wide
// step.  Accumulator register r of lane l holds row 8(r/4) + 4(l/32) + (r mod 4),
// column (l mod 32).
#include <utility>

#include "internal.h"

namespace ozc {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int BK = 64;

enum { KIND_KARATSUBA = 0, KIND_4M = 1, KIND_BOUND = 2, KIND_REAL = 3, KIND_BOUND_REAL = 4 };

// Products of each plan as (A plane, B plane) pairs, in execution order.
template <int KIND>
struct Plan {
    static constexpr bool real = KIND == KIND_REAL || KIND == KIND_BOUND_REAL;
    static constexpr bool bound = KIND == KIND_BOUND || KIND == KIND_BOUND_REAL;
    static constexpr int nseg = real ? 1 : (KIND == KIND_4M ? 4 : 3);
    static constexpr int nplanes = real ? 1 : (KIND == KIND_4M ? 2 : 3);
    static constexpr int eplanes = real ? 1 : 2;  // E' planes per modulus
    // Karatsuba: RR, II, SS.  Expanded: RR, II, RI, IR.  Bound: I.R, R.I, D.D (D = R - I).
    // Real products and the real bound: the one product R.R.
    __device__ static constexpr int pa(int s) {
        return KIND == KIND_BOUND ? (s == 0 ? 1 : (s == 1 ? 0 : 2)) : (KIND == KIND_4M ? (s & 1) : s);
    }
    __device__ static constexpr int pb(int s) {
        return KIND == KIND_4M ? (s == 2 ? 1 : (s == 3 ? 0 : s)) : s;
    }
};

// Symmetric residue of an INT32 accumulator, or of an accumulator plus or minus a
// residue, in FP64: q = rint(x (1/p)) is the nearest integer to x / p (|x| < 2^31, so
// the rounded product is off by less than 2^-22, and x / p lies at least 1/(2p) from a
// half-integer unless p = 256, where 1/p is exact), and x - q p is exact.  For p = 256
// a tie gives +128 instead of -128: the same byte.  The argument stays in INT32: an
// accumulator is bounded by k 127^2 (odd p; k <= 2^17) and the residues added to it
// (at most three times 127) keep it below 2^31 - p; for p = 256 the wrap-around modulo
// 2^32 leaves the residue unchanged.
// Five FP64 instructions, against two quarter-rate integer multiplies and fix-ups for
// a Barrett reduction (2.5% faster batches, 1.5% at 4096^3).
__device__ __forceinline__ int reduce_fp(int x, double pd, double ipd) {
    const double xd = (double)x;
    return (int)fma(-rint(xd * ipd), pd, xd);
}

__device__ __forceinline__ uint32_t pack4(const int (&v)[4]) {
    return (uint32_t)(v[0] & 0xff) | ((uint32_t)(v[1] & 0xff) << 8) |
           ((uint32_t)(v[2] & 0xff) << 16) | ((uint32_t)(v[3] & 0xff) << 24);
}

__device__ __forceinline__ int byte_of(uint32_t w, int u) { return (int)(int8_t)(w >> (8 * u)); }

// LDS tile layout: 64-byte rows of four 16-byte granules; granule g of row r is
// stored at position g ^ sw(r).  With sw(r) = r2 | (r1 ^ r3) << 1 (ri = bit i of
// r), 8 and 16 consecutive rows read at one granule position hit distinct bank
// groups (32- and 64-bank LDS), and so do the row-major 16-byte stores.
__device__ __forceinline__ int swz_bits(int row) {
    return ((row >> 2) & 1) | ((((row >> 1) ^ (row >> 3)) & 1) << 1);
}
__device__ __forceinline__ int swz(int row, int seg) { return row * 4 + (seg ^ swz_bits(row)); }

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0..N-1, so that
// register arrays are only ever indexed by constants.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ void map_tile(int64_t L, int64_t TR, int64_t TC, int64_t total, int &l,
                                         int64_t &ti, int64_t &tj) {
    int64_t q = L;
    if ((total & 7) == 0) q = (L & 7) * (total >> 3) + (L >> 3);  // XCD x -> contiguous part x
    const int64_t T = TR * TC;
    l = (int)(q / T);
    const int64_t t = q - (int64_t)l * T;
    constexpr int64_t G = 4;
    const int64_t grp = t / (G * TC);
    const int64_t rem = t - grp * (G * TC);
    const int64_t rows = min(G, TR - grp * G);
    ti = grp * G + rem % rows;
    tj = rem / rows;
}

// WM x WN waves of BM x BN blocks; KS 64-byte k sub-slabs per pipeline stage.
// k-slabs are copied global -> LDS by the load units directly (gfx950
// global_load_lds_dwordx4) into a ring of NSTAGE buffers, NSTAGE - 1 slabs
// ahead of the matrix cores.  REG_CARRY: the residue carried between the
// products of a modulus stays in registers; otherwise it is parked in the
// thread's own E'_I words.  PREFETCH: the next product's first stages are
// queued before the current product's epilogue; otherwise each product
// starts its own ring after the epilogue.  Both pay where k is short (4096^3:
// 15% faster products); for long k the plain schedule keeps the tiles of an
// XCD in step (16384^3: L2 hit rate 84% against 65%, 2.6% faster).
template <int WM_, int WN_, int BM_, int BN_, int KS_, int NSTAGE_, bool REG_CARRY_, bool PREFETCH_>
struct TileCfg {
    static constexpr int WM = WM_, WN = WN_, BM = BM_, BN = BN_, KS = KS_;
    static constexpr int NSTAGE = NSTAGE_;
    static constexpr bool REG_CARRY = REG_CARRY_, PREFETCH = PREFETCH_;
    static constexpr int TM = WM * BM * 32, TN = WN * BN * 32;
    static constexpr int THREADS = 64 * WM * WN;
    static constexpr int STAGE = (TM + TN) * 4;   // uint4 per sub-slab in LDS
    static constexpr int KSTEP = BK * KS;
};
using CfgLarge = TileCfg<2, 4, 4, 2, 1, 4, false, false>;  // 256 x 256 output tiles, 512 threads, 128 KB LDS
using CfgSmall = TileCfg<2, 2, 2, 2, 1, 4, true, true>;    // 128 x 128, 256 threads, 64 KB LDS
// 256 x 256 tiles with the short-k schedule: single calls with k_pad < kLongK and batches.
using CfgLargeShortK = TileCfg<2, 4, 4, 2, 1, 4, true, true>;
static_assert(CfgLargeShortK::TM == CfgLarge::TM && CfgLargeShortK::TN == CfgLarge::TN &&
                  CfgLargeShortK::KSTEP == CfgLarge::KSTEP,
              "both large-tile schedules share the operand padding");
constexpr int64_t kLongK = 16384;  // measured: short-k faster up to 12288^3, plain at 16384^3

// One wave copies 64 x 16 bytes from global memory straight into 1 KB of LDS:
// lane i reads sbase + voff_i + OFF and writes lds_base + OFF + 16 i (the
// instruction offset applies to both addresses).  The base address and the
// LDS base are wave-uniform scalars and the per-lane offset is fixed for the
// whole kernel, so a copy costs no vector instructions.  Issued as inline
// assembly so that the compiler does not serialise later LDS reads behind it;
// completion is tracked explicitly with vmcnt_wait() before the barrier.
// M0 is written only here in these kernels (checked in the generated code); the
// clobber entry documents it although the compiler treats M0 as reserved.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
template <int OFF>
__device__ __forceinline__ void dma16(const int8_t *sbase, uint32_t voff, uint32_t lds_base) {
    static_assert(OFF >= 0 && OFF < 4096, "instruction offset range");
    asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %0, %1 offset:%3" ::"v"(voff),
                 "s"(sbase), "s"(lds_base), "n"(OFF)
                 : "memory", "m0");
}
#pragma clang diagnostic pop
// A wave-uniform pointer forced into scalar registers.
__device__ __forceinline__ const int8_t *uniform_ptr(const int8_t *p) {
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const int8_t *)(uintptr_t)(((uint64_t)hi << 32) | lo);
}
template <int N>
__device__ __forceinline__ void vmcnt_wait() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
__device__ __forceinline__ void block_barrier() { __builtin_amdgcn_s_barrier(); }

// One output tile (ti, tj) of modulus l: all products of the plan and their epilogues.
// Ends with a block barrier, so a caller may run the next tile right away.
template <int KIND, typename C, bool DUMP>
__device__ __forceinline__ void gemm_tile(const GemmArgs &a, const BoundArgs &b, int l, int64_t ti,
                                          int64_t tj) {
    using P = Plan<KIND>;
    constexpr int TM = C::TM, TN = C::TN, BM = C::BM, BN = C::BN, KS = C::KS;
    constexpr int WTM = BM * 32, WTN = BN * 32;  // wave tile
    __shared__ uint4 lds[C::NSTAGE][KS * C::STAGE];  // [buffer][sub-slab][A rows, B rows]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % C::WM, wn = wave / C::WM;

    constexpr bool bound = P::bound;
    const int64_t m_pad = bound ? b.m_pad : a.m_pad;
    const int64_t n_pad = bound ? b.n_pad : a.n_pad;
    const int64_t k_pad = bound ? b.k_pad : a.k_pad;
    const int64_t i0 = ti * TM, j0 = tj * TN;

    // planes are slab-major: k-slab s (64 wide) of a plane is m_pad x 64 bytes at s * slabA
    const int64_t planeA = m_pad * k_pad, planeB = n_pad * k_pad;
    const int64_t slabA = m_pad * BK, slabB = n_pad * BK;
    const int8_t *baseA = (bound ? b.A : a.A) + (int64_t)l * P::nplanes * planeA + i0 * BK;
    const int8_t *baseB = (bound ? b.B : a.B) + (int64_t)l * P::nplanes * planeB + j0 * BK;

    const int nk = (int)(k_pad / C::KSTEP);

    ModConst mc;
    if constexpr (!bound) mc = a.tab->mod[l];
    const double pd = bound ? 1.0 : (double)mc.p, ipd = 1.0 / pd;
    const int64_t planeC = bound ? 0 : a.n_pad * a.m_pad;

    // Each wave fills whole 1 KB chunks (16 rows) of the A and B slabs: lane i of a
    // chunk writes LDS granule i, i.e. row 16c + i/4 at position i mod 4, which holds
    // the swizzled global granule (i mod 4) ^ swz_bits(row).  A ring stage holds KS
    // consecutive 64-wide k-slabs.
    constexpr int CA = TM / 16, CB = TN / 16, NW = C::WM * C::WN;
    static_assert(CA % NW == 0 && CB % NW == 0, "chunks per wave");
    // a stage is waited for one stage before it is consumed and issued AHEAD >= 2
    // stages ahead, so its buffer was released by the barrier of the stage before
    static_assert(C::NSTAGE >= 3, "DMA ring needs at least three buffers");
    constexpr int QA = CA / NW, QB = CB / NW, NLOAD = KS * (QA + QB);  // loads per wave per stage
    static_assert(QA <= 4 && QB <= 4, "chunk offsets must fit the instruction offset");
    constexpr int AHEAD = C::NSTAGE - 1, NH = 2 * KS;
    const int crow = lane >> 2;
    const int cg = (lane & 3) ^ swz_bits(crow);  // chunk rows start at multiples of 16
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    // per-lane offsets inside the wave's first chunk (same for every stage and product)
    const uint32_t voffA = (uint32_t)(wv * QA * 1024 + crow * BK + cg * 16);
    const uint32_t voffB = (uint32_t)(wv * QB * 1024 + crow * BK + cg * 16);
    const uint32_t lbase = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint4 *)(&lds[0][0]);
    // plane bases of product g (wave-uniform)
    auto pa_of = [&](int g) { return uniform_ptr(baseA + (int64_t)P::pa(g) * planeA); };
    auto pb_of = [&](int g) { return uniform_ptr(baseB + (int64_t)P::pb(g) * planeB); };
    auto issue_from = [&](const int8_t *sa, const int8_t *sb_, int st) {  // stage st -> buffer st % NSTAGE
        const uint32_t buf = lbase + (uint32_t)((st % C::NSTAGE) * KS * C::STAGE * 16);
        static_for<KS>([&](auto ks) {
            const int64_t ks_idx = (int64_t)st * KS + ks;
            const uint32_t la = buf + (uint32_t)(ks * C::STAGE * 16 + wv * QA * 1024);
            const uint32_t lb = buf + (uint32_t)(ks * C::STAGE * 16 + TM * 64 + wv * QB * 1024);
            static_for<QA>([&](auto q) { dma16<q * 1024>(sa + ks_idx * slabA, voffA, la); });
            static_for<QB>([&](auto q) { dma16<q * 1024>(sb_ + ks_idx * slabB, voffB, lb); });
        });
    };
    // The first AHEAD stages of a product.  Those of product g + 1 are issued right
    // after product g's last barrier, so they load while g's epilogue runs.
    auto issue_first = [&](int g) {
        const int8_t *sa = pa_of(g), *sb_ = pb_of(g);
        static_for<AHEAD>([&](auto st) {
            if (st < nk) issue_from(sa, sb_, st);
        });
    };

    v16i acc[BM][BN];
    uint32_t cw[BM][BN][4];  // packed carry residues (kept here, or reloaded from E'_I)
    uint32_t cr[BM][BN][4];  // Karatsuba, carry in registers, small tiles: E'_R, kept for E'_I
    if constexpr (C::PREFETCH) issue_first(0);

#pragma unroll 1
    for (int sgi = 0; sgi < P::nseg; ++sgi) {
        if (!bound || sgi == 0) {
            static_for<BM>([&](auto bi) { static_for<BN>([&](auto bj) { acc[bi][bj] = v16i{}; }); });
        }
        // Fragments of one 32-wide half (kk) of a 64-wide k-slab held in LDS buffer Lbuf.
        auto read_frags = [&](const uint4 *Lbuf, int kk, v4i (&fa)[BM], v4i (&fb)[BN]) {
            // fragment rows are (multiple of 32) + (lane mod 32): the swizzle depends on the lane only
            const int g = (kk * 2 + (lane >> 5)) ^ swz_bits(lane & 31);
            const uint4 *FA = Lbuf + (wm * WTM + (lane & 31)) * 4 + g;
            const uint4 *FB = Lbuf + TM * 4 + (wn * WTN + (lane & 31)) * 4 + g;
            // issue order B0 A0 B1 A1 A2 ...: the MFMAs (A-block outer, B-block inner) can
            // start after the first two reads and consume the rest as they arrive
            constexpr int NR = BM > BN ? BM : BN;
            static_for<NR>([&](auto i) {
                if constexpr (i < BN) {
                    const uint4 t = FB[i * 32 * 4];
                    fb[i] = v4i{(int)t.x, (int)t.y, (int)t.z, (int)t.w};
                }
                if constexpr (i < BM) {
                    const uint4 t = FA[i * 32 * 4];
                    fa[i] = v4i{(int)t.x, (int)t.y, (int)t.z, (int)t.w};
                }
            });
        };
        auto mfmas = [&](const v4i (&fa)[BM], const v4i (&fb)[BN]) {
            static_for<BM>([&](auto bi) {
                static_for<BN>([&](auto bj) {
                    acc[bi][bj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[bi], fb[bj], acc[bi][bj], 0, 0, 0);
                });
            });
        };
        {
            const int8_t *sa = pa_of(sgi), *sb_ = pb_of(sgi);
            auto issue = [&](int st) { issue_from(sa, sb_, st); };
            // Software pipeline over half-slabs (32-wide k): the fragments of the next half
            // are read while the current half's matrix instructions run.  The one barrier
            // per stage sits before the last half's MFMAs, after the wait for the next
            // stage, so queued MFMAs keep the matrix pipe busy while the waves meet; after
            // it the oldest buffer is free and receives the stage AHEAD steps ahead.
            // stages 1 .. AHEAD-1 may stay in flight, except when this product's first
            // stages were queued before the previous epilogue's stores: then wait for all
            if constexpr (!C::PREFETCH) issue_first(sgi);
            const bool fresh = !C::PREFETCH || sgi == 0;
            if (fresh && nk > 2 && AHEAD >= 3) vmcnt_wait<2 * NLOAD>();
            else if (fresh && nk > 1 && AHEAD >= 2) vmcnt_wait<NLOAD>();
            else vmcnt_wait<0>();
            block_barrier();
            v4i fa[2][BM], fb[2][BN];
            read_frags(lds[0], 0, fa[0], fb[0]);
            // The fragment reads of the next half are interleaved with this half's matrix
            // instructions (MFMA, read, MFMA, read, ...) so that they are all in flight
            // early; otherwise the scheduler tends to sink them behind the MFMAs and the
            // LDS latency shows at the start of the next half.
            auto interleave = [&]() {
                static_for<BM + BN>([&](auto) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
                });
                __builtin_amdgcn_sched_group_barrier(0x008, BM * BN - (BM + BN), 0);
            };
            static_assert(BM * BN >= BM + BN, "interleave needs an MFMA per fragment read");
            // HANDOVER: wait for stage s+1 (WAIT loads of later stages may stay in flight),
            // then ISSUE stage s + AHEAD into the buffer released by the barrier.
            auto stage = [&](int s, auto handover_tag, auto issue_tag, auto wait_tag) {
                constexpr bool HANDOVER = decltype(handover_tag)::value;
                constexpr bool ISSUE = decltype(issue_tag)::value;
                const uint4 *cur = lds[s % C::NSTAGE];
                static_for<NH>([&](auto h) {
                    constexpr int nb = (h + 1) & 1;
                    if constexpr (h + 1 < NH) {
                        read_frags(cur + ((h + 1) / 2) * C::STAGE, (h + 1) & 1, fa[nb], fb[nb]);
                        mfmas(fa[h & 1], fb[h & 1]);
                        interleave();
                    } else if constexpr (HANDOVER) {
                        vmcnt_wait<decltype(wait_tag)::value>();
                        block_barrier();  // stage s+1 visible; stage s-1's buffer free
                        if constexpr (ISSUE) issue(s + AHEAD);
                        read_frags(lds[(s + 1) % C::NSTAGE], 0, fa[0], fb[0]);
                        mfmas(fa[h & 1], fb[h & 1]);
                        interleave();
                    } else {
                        mfmas(fa[h & 1], fb[h & 1]);
                    }
                });
            };
            using T = std::true_type;
            using F = std::false_type;
            // stages issued after stage s+1 when it is awaited: min(AHEAD - 2, nk - 2 - s)
            constexpr int LATER = AHEAD >= 2 ? AHEAD - 2 : 0;
            using WL = std::integral_constant<int, LATER * NLOAD>;
            using W0 = std::integral_constant<int, 0>;
            int s = 0;
            for (; s + AHEAD < nk; ++s) stage(s, T{}, T{}, WL{});
            for (; s + 1 + LATER < nk; ++s) stage(s, T{}, F{}, WL{});
            for (; s + 1 < nk; ++s) stage(s, T{}, F{}, W0{});
            stage(s, F{}, F{}, W0{});
            block_barrier();  // all waves done with the ring before it is refilled
        }

        // ------------------------------------------------ per-product epilogue
        // (compile-time loops only: the accumulators must stay in registers)
        // The residue carried from one product to the next (mod(D) then mod(D + E) for
        // Karatsuba, mod(RR) and mod(RI) for the expanded form) stays in registers, or
        // is parked in this thread's own E'_I words, which receive the final E'_I last
        // (each lane re-reads only what it wrote, so no synchronisation is needed).
        // With the carry in registers and small tiles, Karatsuba keeps mod(D) and E'_R
        // instead of mod(D + E): three reductions per output rather than four.
        // Parked carries are loaded and awaited first; then the next product's first
        // stages are queued, so that their copies overlap the rest of this epilogue.
        constexpr bool karatsuba = KIND == KIND_KARATSUBA;
        // the E'_R registers fit beside small tiles' accumulators only
        constexpr bool keep_er = karatsuba && C::REG_CARRY && C::BM * C::BN <= 4;
        auto eword = [&](int8_t *E, int bi, int bj, int g) {
            const int64_t i = i0 + wm * WTM + bi * 32 + 8 * g + 4 * (lane >> 5);
            const int64_t j = j0 + wn * WTN + bj * 32 + (lane & 31);
            return reinterpret_cast<uint32_t *>(E + j * a.m_pad + i);
        };
        int8_t *ER = nullptr, *EI = nullptr;
        if constexpr (!bound) {
            ER = a.eprime + (int64_t)l * P::eplanes * planeC;
            EI = ER + planeC;  // not used by real products
            if (C::PREFETCH && !C::REG_CARRY && sgi >= 1 && (karatsuba || sgi != 2)) {
                static_for<BM>([&](auto bi) {
                    static_for<BN>([&](auto bj) {
                        static_for<4>([&](auto g) { cw[bi][bj][g] = *eword(EI, bi, bj, g); });
                    });
                });
                __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the carries are in registers
            }
        }
        if constexpr (C::PREFETCH) {
            if (sgi + 1 < P::nseg) issue_first(sgi + 1);
        }
        if constexpr (DUMP) {
            int32_t *D = a.prods + ((int64_t)l * P::nseg + sgi) * planeC;
            static_for<BM>([&](auto bi) {
                static_for<BN>([&](auto bj) {
                    static_for<16>([&](auto r) {
                        const int64_t i = i0 + wm * WTM + bi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                        const int64_t j = j0 + wn * WTN + bj * 32 + (lane & 31);
                        D[j * a.m_pad + i] = acc[bi][bj][(int)r];
                    });
                });
            });
        }
        if constexpr (bound) {
            // complex: acc holds Cbar_I after the second product, Cbar_R after the third;
            // real: Abar Bbar after the one product
            if (P::real || sgi >= 1) {
                static_for<BM>([&](auto bi) {
                    static_for<16>([&](auto r) {
                        int x = acc[bi][0][(int)r];
                        static_for<BN>([&](auto bj) { x = max(x, acc[bi][bj][(int)r]); });
#pragma unroll
                        for (int off = 16; off >= 1; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
                        if ((lane & 31) == 0 && x > 0) {
                            const int64_t i = i0 + wm * WTM + bi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                            atomicMax(&b.X[i], x);
                        }
                    });
                });
                static_for<BN>([&](auto bj) {
                    int y = 0;
                    static_for<BM>([&](auto bi) { static_for<16>([&](auto r) { y = max(y, acc[bi][bj][(int)r]); }); });
                    y = max(y, __shfl_xor(y, 32, 64));
                    if (lane < 32 && y > 0) atomicMax(&b.Y[j0 + wn * WTN + bj * 32 + lane], y);
                });
            }
        } else if constexpr (P::real) {
            // E' = mod(A'_l B'_l): one reduction per output (Algorithm 1 Step V-iv)
            static_for<BM>([&](auto bi) {
                static_for<BN>([&](auto bj) {
                    static_for<4>([&](auto g) {
                        int o[4];
                        static_for<4>([&](auto u) { o[u] = reduce_fp(acc[bi][bj][4 * (int)g + u], pd, ipd); });
                        *eword(ER, bi, bj, g) = pack4(o);
                    });
                });
            });
        } else {
            static_for<BM>([&](auto bi) {
                // A parked carry is read back one row of blocks at a time (BN * 4 words in one
                // burst of loads) before that row's stores: a load after a store is not moved
                // above it (they might alias), so word-by-word read-back waited for a memory
                // round trip per word.  Reading all BM rows before any store was no faster
                // overall (fewer E' write-backs, but more operand misses in L2).
                if (!C::PREFETCH && !C::REG_CARRY && sgi >= 1 && (karatsuba || sgi != 2)) {
                    static_for<BN>([&](auto bj) {
                        static_for<4>([&](auto g) { cw[bi][bj][g] = *eword(EI, bi, bj, g); });
                    });
                }
                static_for<BN>([&](auto bj) {
                    static_for<4>([&](auto g) {
                        uint32_t *er = eword(ER, bi, bj, g);
                        uint32_t *ei = eword(EI, bi, bj, g);
                        // The first product of a pair is reduced and carried; the second
                        // enters the reduction unreduced (accumulator +- carried residue
                        // stays in range, see reduce_fp): 4 reductions per output and
                        // modulus in both forms, 3 for Karatsuba with keep_er.
                        int o[4];
                        auto acc_u = [&](int u) { return acc[bi][bj][4 * (int)g + u]; };
                        if (sgi == 0 || (!karatsuba && sgi == 2)) {
                            static_for<4>([&](auto u) { o[u] = reduce_fp(acc_u(u), pd, ipd); });
                            if constexpr (C::REG_CARRY) cw[bi][bj][g] = pack4(o);
                            else *ei = pack4(o);
                        } else if (sgi == 1) {
                            // Karatsuba: E'_R = mod(D - E), carry mod(D + E); expanded: E'_R = mod(RR - II)
                            const uint32_t w = cw[bi][bj][g];
                            static_for<4>([&](auto u) { o[u] = reduce_fp(byte_of(w, u) - acc_u(u), pd, ipd); });
                            *er = pack4(o);
                            if constexpr (keep_er) {
                                cr[bi][bj][g] = pack4(o);
                            } else if constexpr (karatsuba) {
                                static_for<4>([&](auto u) { o[u] = reduce_fp(byte_of(w, u) + acc_u(u), pd, ipd); });
                                if constexpr (C::REG_CARRY) cw[bi][bj][g] = pack4(o);
                                else *ei = pack4(o);
                            }
                        } else if constexpr (keep_er) {
                            // E'_I = mod(F - D - E) = mod(F - 2 mod(D) + E'_R), since
                            // D + E = 2 D - (D - E): one reduction fewer than carrying mod(D + E)
                            const uint32_t w = cw[bi][bj][g], r = cr[bi][bj][g];
                            static_for<4>([&](auto u) {
                                o[u] = reduce_fp(acc_u(u) - 2 * byte_of(w, u) + byte_of(r, u), pd, ipd);
                            });
                            *ei = pack4(o);
                        } else {
                            // Karatsuba: E'_I = mod(F - mod(D + E)); expanded: E'_I = mod(RI + IR)
                            const uint32_t w = cw[bi][bj][g];
                            static_for<4>([&](auto u) {
                                o[u] = reduce_fp(karatsuba ? acc_u(u) - byte_of(w, u) : byte_of(w, u) + acc_u(u), pd, ipd);
                            });
                            *ei = pack4(o);
                        }
                    });
                });
            });
        }
    }
}

template <int KIND, typename C, bool DUMP>
__global__ __launch_bounds__(C::THREADS) void residue_gemm_kernel(GemmArgs a, BoundArgs b) {
    constexpr bool bound = Plan<KIND>::bound;
    const int64_t TR = (bound ? b.m_pad : a.m_pad) / C::TM, TC = (bound ? b.n_pad : a.n_pad) / C::TN;
    const int nmod = bound ? 1 : a.nmod;
    int l;
    int64_t ti, tj;
    map_tile((int64_t)blockIdx.x, TR, TC, (int64_t)nmod * TR * TC, l, ti, tj);
    gemm_tile<KIND, C, DUMP>(a, b, l, ti, tj);
}

// Persistent kernel over the work queue of a batch: each block takes the next
// item from the counter until the queue is empty.  Items of one problem are
// numbered (modulus group, tile row, tile column); problems are ordered by the
// host (largest k first).
template <int KIND, typename C>
__global__ __launch_bounds__(C::THREADS) void batch_gemm_kernel(const BatchGemm *probs, int nprob,
                                                                int64_t items, int group,
                                                                uint32_t *counters, int64_t chunk) {
    __shared__ int64_t item_s;
    // Work-groups are dispatched to the XCDs in turn (block b on XCD b mod 8).  The
    // item sequence is cut into chunks of `chunk` items (the blocks one XCD holds at a
    // time), dealt to the XCDs in turn, each XCD with its own counter: the tiles that
    // run together on an XCD are neighbours of one product and share their operand
    // panels in that XCD's L2.  A block whose queue is empty takes items from the
    // other queues.  Any dispatch order gives the same results.
    // Per item the block needs the queue's counter and its problem's record, each a
    // round trip to L2: the next item is claimed as soon as the current one is known
    // (the atomic returns while this item computes), and the problem is looked up
    // first where the previous item was (a block's items rise within a queue, and a
    // problem has many items), with a binary search only when that misses.  Item
    // numbers are below 2^32 (the counters are 32-bit), so the index arithmetic is
    // 32-bit.  The counter address is offset by a zero the compiler cannot see through:
    // for a uniform address it combines the lanes' atomics into one and reads the
    // result back at once, which would wait for the round trip right there.
    const int64_t nchunks = items / chunk, rem = items - nchunks * chunk;
    const uint32_t ch = (uint32_t)chunk;
    const int home = (int)(blockIdx.x % kBatchQueues);
    int lo = 0;          // problem of the previous item
    uint32_t ahead = 0;  // thread 0: the item claimed for the next round
    uint32_t zero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    for (int qs = 0; qs < kBatchQueues; ++qs) {
        const int q = (home + qs) % kBatchQueues;
        const int64_t nq = (nchunks / kBatchQueues + (q < nchunks % kBatchQueues ? 1 : 0)) * chunk +
                           (nchunks % kBatchQueues == q ? rem : 0);
        if (threadIdx.x == 0) ahead = atomicAdd(&counters[q], 1u);
        for (;;) {
            if (threadIdx.x == 0) item_s = (int64_t)ahead;
            __syncthreads();
            const int64_t j = item_s;
            __syncthreads();
            if (j >= nq) break;
            if (threadIdx.x == 0) ahead = atomicAdd(&counters[q] + zero, 1u);
            const uint32_t j32 = (uint32_t)j, jc = j32 / ch;
            const int64_t w = ((int64_t)jc * kBatchQueues + q) * ch + (j32 - jc * ch);
            const int64_t f0 = probs[lo].item0;
            const int64_t f1 = lo + 1 < nprob ? probs[lo + 1].item0 : items;
            if (w < f0 || w >= f1) {  // last problem whose first item is <= w
                int hi = w < f0 ? lo - 1 : nprob - 1;
                lo = w < f0 ? 0 : lo + 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (probs[mid].item0 <= w) lo = mid;
                    else hi = mid - 1;
                }
            }
            const BatchGemm &pb = probs[lo];
            const uint32_t T = (uint32_t)pb.TR * (uint32_t)pb.TC, local = (uint32_t)(w - pb.item0);
            const int lg = (int)(local / T);
            const uint32_t t = local - (uint32_t)lg * T;
            const int64_t ti = t / (uint32_t)pb.TC, tj = t - (uint32_t)ti * (uint32_t)pb.TC;
            GemmArgs a{pb.A, pb.B, pb.m_pad, pb.n_pad, pb.k_pad, pb.nmod, KIND == KIND_4M ? 1 : 0,
                       pb.tab, pb.eprime, nullptr, C::TM};
            const int l1 = min(pb.nmod, (lg + 1) * group);
            for (int l = lg * group; l < l1; ++l) gemm_tile<KIND, C, false>(a, BoundArgs{}, l, ti, tj);
        }
    }
}

// Persistent kernel over the tiles of a batch's bound products (accurate mode).
template <typename C>
__global__ __launch_bounds__(C::THREADS) void batch_bound_kernel(const BatchBound *probs, int nprob,
                                                                int64_t items, uint32_t *counter) {
    __shared__ int64_t item_s;
    for (;;) {
        if (threadIdx.x == 0) item_s = (int64_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int64_t w = item_s;
        __syncthreads();
        if (w >= items) break;
        int lo = 0, hi = nprob - 1;  // last problem whose first item is <= w
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (probs[mid].item0 <= w) lo = mid;
            else hi = mid - 1;
        }
        const BatchBound &pb = probs[lo];
        const int64_t t = w - pb.item0;
        const int64_t ti = t / pb.TC, tj = t - ti * pb.TC;
        gemm_tile<KIND_BOUND, C, false>(GemmArgs{}, pb.b, 0, ti, tj);
    }
}

template <int KIND, typename C>
void launch_batch_kind(const BatchGemm *probs, int nprob, int64_t items, int group,
                       uint32_t *counters, int grid, hipStream_t s) {
    const int64_t chunk = grid >= kBatchQueues ? grid / kBatchQueues : 1;  // resident blocks per XCD
    hipLaunchKernelGGL((batch_gemm_kernel<KIND, C>), dim3((unsigned)grid), dim3(C::THREADS), 0, s,
                       probs, nprob, items, group, counters, chunk);
}

template <int KIND, typename C>
int blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_gemm_kernel<KIND, C>, C::THREADS, 0) !=
        hipSuccess)
        n = 1;
    return n > 0 ? n : 1;
}

template <int KIND, typename C>
void launch_kind(const GemmArgs &a, const BoundArgs &b, bool dump, int64_t blocks, hipStream_t s) {
    if (dump) hipLaunchKernelGGL((residue_gemm_kernel<KIND, C, true>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s, a, b);
    else hipLaunchKernelGGL((residue_gemm_kernel<KIND, C, false>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s, a, b);
}

}  // namespace

int gemm_tile_for(int64_t m, int64_t n) { return (m >= 1024 && n >= 1024) ? 256 : 128; }
int gemm_kstep_for(int tile) { return tile == 256 ? CfgLarge::KSTEP : CfgSmall::KSTEP; }
int gemm_tile_rows(int tile) { return tile == 256 ? CfgLarge::TM : CfgSmall::TM; }
int gemm_tile_cols(int tile) { return tile == 256 ? CfgLarge::TN : CfgSmall::TN; }

hipError_t launch_residue_gemm(const GemmArgs &a, hipStream_t s) {
    const int tile = a.tile;
    if (tile != 128 && tile != 256) return hipErrorInvalidValue;
    const int tr = gemm_tile_rows(tile), tc = gemm_tile_cols(tile);
    if (a.m_pad % tr || a.n_pad % tc || a.k_pad % gemm_kstep_for(tile) || a.nmod < 1)
        return hipErrorInvalidValue;
    const int64_t blocks = (int64_t)a.nmod * (a.m_pad / tr) * (a.n_pad / tc);
    if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    BoundArgs none{};
    const bool dump = a.prods != nullptr;
    if (a.algo < 0 || a.algo > 2) return hipErrorInvalidValue;
    // one product per modulus: the long-k schedule keeps no carry, so it serves every k
    if (a.algo == 2) {
        if (tile == 256) launch_kind<KIND_REAL, CfgLarge>(a, none, dump, blocks, s);
        else launch_kind<KIND_REAL, CfgSmall>(a, none, dump, blocks, s);
        return hipGetLastError();
    }
    if (tile == 256) {
        if (a.k_pad >= kLongK) {
            if (a.algo == 0) launch_kind<KIND_KARATSUBA, CfgLarge>(a, none, dump, blocks, s);
            else launch_kind<KIND_4M, CfgLarge>(a, none, dump, blocks, s);
        } else {
            if (a.algo == 0) launch_kind<KIND_KARATSUBA, CfgLargeShortK>(a, none, dump, blocks, s);
            else launch_kind<KIND_4M, CfgLargeShortK>(a, none, dump, blocks, s);
        }
    } else {
        if (a.algo == 0) launch_kind<KIND_KARATSUBA, CfgSmall>(a, none, dump, blocks, s);
        else launch_kind<KIND_4M, CfgSmall>(a, none, dump, blocks, s);
    }
    return hipGetLastError();
}

// The bound product is 1/N of the work; it always runs on 128 x 128 tiles
// (valid for buffers padded to 128 or 256).
hipError_t launch_bound_gemm(const BoundArgs &b, hipStream_t s) {
    constexpr int tile = 128;
    if (b.m_pad % tile || b.n_pad % tile || b.k_pad % BK) return hipErrorInvalidValue;
    const int64_t blocks = (b.m_pad / tile) * (b.n_pad / tile);
    GemmArgs none{};
    if (b.real) launch_kind<KIND_BOUND_REAL, CfgSmall>(none, b, false, blocks, s);
    else launch_kind<KIND_BOUND, CfgSmall>(none, b, false, blocks, s);
    return hipGetLastError();
}

hipError_t launch_batch_bound(const BatchBound *probs, int nprob, int64_t items,
                              uint32_t *counter, hipStream_t s) {
    if (items <= 0 || nprob <= 0) return hipSuccess;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_bound_kernel<CfgSmall>,
                                                     CfgSmall::THREADS, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int64_t grid = (int64_t)cus * per_cu;
    if (grid > items) grid = items;
    hipLaunchKernelGGL((batch_bound_kernel<CfgSmall>), dim3((unsigned)grid), dim3(CfgSmall::THREADS), 0,
                       s, probs, nprob, items, counter);
    return hipGetLastError();
}

int batch_gemm_blocks_per_cu(int tile) {
    return tile == 256 ? blocks_per_cu<KIND_KARATSUBA, CfgLargeShortK>() : blocks_per_cu<KIND_KARATSUBA, CfgSmall>();
}

hipError_t launch_batch_gemm(const BatchGemm *probs, int nprob, int64_t items, int tile, int group,
                             int algo, uint32_t *counters, int grid_blocks, hipStream_t s) {
    if (items <= 0 || nprob <= 0) return hipSuccess;
    if ((tile != 128 && tile != 256) || group < 1) return hipErrorInvalidValue;
    if (grid_blocks <= 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        grid_blocks = cus * batch_gemm_blocks_per_cu(tile);
    }
    if ((int64_t)grid_blocks > items) grid_blocks = (int)items;
    if (tile == 256) {
        if (algo == 0) launch_batch_kind<KIND_KARATSUBA, CfgLargeShortK>(probs, nprob, items, group, counters, grid_blocks, s);
        else launch_batch_kind<KIND_4M, CfgLargeShortK>(probs, nprob, items, group, counters, grid_blocks, s);
    } else {
        if (algo == 0) launch_batch_kind<KIND_KARATSUBA, CfgSmall>(probs, nprob, items, group, counters, grid_blocks, s);
        else launch_batch_kind<KIND_4M, CfgSmall>(probs, nprob, items, group, counters, grid_blocks, s);
    }
    return hipGetLastError();
}

}  // namespace ozc
