// Per-modulus complex INT8 products on the gfx950 matrix cores with INT32
// accumulation (Section III-A; Algorithm 1 Step V-iii/iv).
//
// One block computes a TM x TN output tile of one modulus l with WM x WN
// waves; each wave owns (BM*32) x (BN*32) outputs as BM x BN blocks of
// v_mfma_i32_32x32x32_i8 (large problems: 256 x 256 tiles, 8 waves of
// 128 x 64, two waves per SIMD; small problems: 128 x 128, 4 waves of 64 x 64).  The products of the chosen algorithm run one after
// another over the same tile, each as a k-loop over double-buffered LDS
// tiles (one barrier per 64-wide k-step, the next tile prefetched into
// registers while the current one feeds the matrix cores).  Between products
// the INT32 accumulators are reduced to symmetric residues in registers; one
// packed INT8 carry per output survives to the next product, and E'_R, E'_I
// are stored as soon as they are final, so only INT8 data leaves the chip:
//   Karatsuba (eq. (10)): D = R.R, E = I.I, F = S.S (S = reduced R + I):
//                         E'_R = mod(D - E), E'_I = mod(F - mod(D + E))
//   expanded  (eq. (7)):  E'_R = mod(RR - II), E'_I = mod(RI + IR)
// A third plan computes the accurate-mode bound product (Section III-B):
//   Cbar_I = Abar_I Bbar_R + Abar_R Bbar_I, Cbar_R = Cbar_I + (Abar_R - Abar_I)(Bbar_R - Bbar_I),
// folded on the fly into row and column maxima (Cbar is never stored).
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
#include "internal.h"

namespace ozc {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int BK = 64;

enum { KIND_KARATSUBA = 0, KIND_4M = 1, KIND_BOUND = 2 };

// Products of each plan as (A plane, B plane) pairs, in execution order.
template <int KIND>
struct Plan {
    static constexpr int nseg = KIND == KIND_4M ? 4 : 3;
    static constexpr int nplanes = KIND == KIND_4M ? 2 : 3;
    // Karatsuba: RR, II, SS.  Expanded: RR, II, RI, IR.  Bound: I.R, R.I, D.D (D = R - I).
    __device__ static constexpr int pa(int s) {
        return KIND == KIND_BOUND ? (s == 0 ? 1 : (s == 1 ? 0 : 2)) : (KIND == KIND_4M ? (s & 1) : s);
    }
    __device__ static constexpr int pb(int s) {
        return KIND == KIND_4M ? (s == 2 ? 1 : (s == 3 ? 0 : s)) : s;
    }
};

// Symmetric residue of an INT32 accumulator: for odd p the accumulator is
// bounded by k * 127^2 < 2^31 and koff (a multiple of p >= 2^31) makes it
// non-negative; for p = 256 the wrap-around modulo 2^32 is harmless.
__device__ __forceinline__ int reduce_acc(int x, const ModConst &mc) {
    uint32_t u = (uint32_t)x + mc.koff;
    uint32_t r = u - __umulhi(u, mc.barrett) * mc.p;
    if (r >= mc.p) r -= mc.p;
    int s = (int)r;
    if (r >= mc.half) s -= (int)mc.p;
    return s;
}

__device__ __forceinline__ uint32_t pack4(const int (&v)[4]) {
    return (uint32_t)(v[0] & 0xff) | ((uint32_t)(v[1] & 0xff) << 8) |
           ((uint32_t)(v[2] & 0xff) << 16) | ((uint32_t)(v[3] & 0xff) << 24);
}

__device__ __forceinline__ int byte_of(uint32_t w, int u) { return (int)(int8_t)(w >> (8 * u)); }

__device__ __forceinline__ int swz(int row, int seg) { return row * 4 + (seg ^ ((row >> 1) & 3)); }

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

template <int WM_, int WN_, int BM_, int BN_>
struct TileCfg {
    static constexpr int WM = WM_, WN = WN_, BM = BM_, BN = BN_;
    static constexpr int TM = WM * BM * 32, TN = WN * BN * 32;
    static constexpr int THREADS = 64 * WM * WN;
    static constexpr int NLA = TM * 4 / THREADS;  // 16-byte loads per thread per k-step (A)
    static constexpr int NLB = TN * 4 / THREADS;  // (B)
    static constexpr int ROWS_PER_LOAD = THREADS / 4;
};
using CfgLarge = TileCfg<2, 4, 4, 2>;  // 256 x 256, 512 threads
using CfgSmall = TileCfg<2, 2, 2, 2>;  // 128 x 128, 256 threads

template <int KIND, typename C, bool DUMP>
__global__ __launch_bounds__(C::THREADS) void residue_gemm_kernel(GemmArgs a, BoundArgs b) {
    using P = Plan<KIND>;
    constexpr int TM = C::TM, TN = C::TN, BM = C::BM, BN = C::BN;
    constexpr int WTM = BM * 32, WTN = BN * 32;  // wave tile
    __shared__ uint4 lds[2][(TM + TN) * 4];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % C::WM, wn = wave / C::WM;

    const bool bound = KIND == KIND_BOUND;
    const int64_t m_pad = bound ? b.m_pad : a.m_pad;
    const int64_t n_pad = bound ? b.n_pad : a.n_pad;
    const int64_t k_pad = bound ? b.k_pad : a.k_pad;
    const int64_t TR = m_pad / TM, TC = n_pad / TN;
    const int nmod = bound ? 1 : a.nmod;
    int l;
    int64_t ti, tj;
    map_tile((int64_t)blockIdx.x, TR, TC, (int64_t)nmod * TR * TC, l, ti, tj);
    const int64_t i0 = ti * TM, j0 = tj * TN;

    const int64_t planeA = m_pad * k_pad, planeB = n_pad * k_pad;
    const int8_t *baseA = (bound ? b.A : a.A) + (int64_t)l * P::nplanes * planeA + i0 * k_pad;
    const int8_t *baseB = (bound ? b.B : a.B) + (int64_t)l * P::nplanes * planeB + j0 * k_pad;

    const int lrow = tid >> 2, lseg = tid & 3;
    const int nk = (int)(k_pad / BK);
    const int64_t rstep = (int64_t)C::ROWS_PER_LOAD * k_pad;

    ModConst mc;
    if constexpr (!bound) mc = a.tab->mod[l];
    const int64_t planeC = bound ? 0 : a.n_pad * a.m_pad;

    uint32_t keep[BM][BN][4];
    v16i acc[BM][BN];

#pragma unroll 1
    for (int sgi = 0; sgi < P::nseg; ++sgi) {
        const int8_t *Ap = baseA + (int64_t)P::pa(sgi) * planeA + (int64_t)lrow * k_pad + lseg * 16;
        const int8_t *Bp = baseB + (int64_t)P::pb(sgi) * planeB + (int64_t)lrow * k_pad + lseg * 16;
        if (!bound || sgi == 0) {
#pragma unroll
            for (int bi = 0; bi < BM; ++bi)
#pragma unroll
                for (int bj = 0; bj < BN; ++bj) acc[bi][bj] = v16i{};
        }
        // two 16-byte loads per thread per operand and k-step (both tile shapes);
        // named registers rather than arrays keep them out of scratch memory
        static_assert(C::NLA == 2 && C::NLB == 2, "loader assumes two loads per operand");
        const int r1 = lrow + C::ROWS_PER_LOAD;
        uint4 ra0 = *reinterpret_cast<const uint4 *>(Ap);
        uint4 ra1 = *reinterpret_cast<const uint4 *>(Ap + rstep);
        uint4 rb0 = *reinterpret_cast<const uint4 *>(Bp);
        uint4 rb1 = *reinterpret_cast<const uint4 *>(Bp + rstep);
        lds[0][swz(lrow, lseg)] = ra0;
        lds[0][swz(r1, lseg)] = ra1;
        lds[0][TM * 4 + swz(lrow, lseg)] = rb0;
        lds[0][TM * 4 + swz(r1, lseg)] = rb1;
        __syncthreads();

        for (int s = 0; s < nk; ++s) {
            const int cur = s & 1;
            const bool more = s + 1 < nk;
            if (more) {
                const int64_t ko = (int64_t)(s + 1) * BK;
                ra0 = *reinterpret_cast<const uint4 *>(Ap + ko);
                ra1 = *reinterpret_cast<const uint4 *>(Ap + rstep + ko);
                rb0 = *reinterpret_cast<const uint4 *>(Bp + ko);
                rb1 = *reinterpret_cast<const uint4 *>(Bp + rstep + ko);
            }
            const uint4 *LA = lds[cur];
            const uint4 *LB = lds[cur] + TM * 4;
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int seg = kk * 2 + (lane >> 5);
                v4i fa[BM], fb[BN];
#pragma unroll
                for (int bi = 0; bi < BM; ++bi) {
                    const uint4 t = LA[swz(wm * WTM + bi * 32 + (lane & 31), seg)];
                    fa[bi] = v4i{(int)t.x, (int)t.y, (int)t.z, (int)t.w};
                }
#pragma unroll
                for (int bj = 0; bj < BN; ++bj) {
                    const uint4 t = LB[swz(wn * WTN + bj * 32 + (lane & 31), seg)];
                    fb[bj] = v4i{(int)t.x, (int)t.y, (int)t.z, (int)t.w};
                }
#pragma unroll
                for (int bi = 0; bi < BM; ++bi)
#pragma unroll
                    for (int bj = 0; bj < BN; ++bj)
                        acc[bi][bj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[bi], fb[bj],
                                                                           acc[bi][bj], 0, 0, 0);
            }
            if (more) {
                lds[cur ^ 1][swz(lrow, lseg)] = ra0;
                lds[cur ^ 1][swz(r1, lseg)] = ra1;
                lds[cur ^ 1][TM * 4 + swz(lrow, lseg)] = rb0;
                lds[cur ^ 1][TM * 4 + swz(r1, lseg)] = rb1;
            }
            __syncthreads();
        }

        // ------------------------------------------------ per-product epilogue
        if constexpr (DUMP) {
            int32_t *D = a.prods + ((int64_t)l * P::nseg + sgi) * planeC;
#pragma unroll
            for (int bi = 0; bi < BM; ++bi)
#pragma unroll
                for (int bj = 0; bj < BN; ++bj)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int64_t i = i0 + wm * WTM + bi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                        const int64_t j = j0 + wn * WTN + bj * 32 + (lane & 31);
                        D[j * a.m_pad + i] = acc[bi][bj][r];
                    }
        }
        if constexpr (bound) {
            if (sgi >= 1) {  // acc holds Cbar_I after the second product, Cbar_R after the third
#pragma unroll
                for (int bi = 0; bi < BM; ++bi)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        int x = acc[bi][0][r];
#pragma unroll
                        for (int bj = 1; bj < BN; ++bj) x = max(x, acc[bi][bj][r]);
#pragma unroll
                        for (int off = 16; off >= 1; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
                        if ((lane & 31) == 0 && x > 0) {
                            const int64_t i = i0 + wm * WTM + bi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                            atomicMax(&b.X[i], x);
                        }
                    }
#pragma unroll
                for (int bj = 0; bj < BN; ++bj) {
                    int y = 0;
#pragma unroll
                    for (int bi = 0; bi < BM; ++bi)
#pragma unroll
                        for (int r = 0; r < 16; ++r) y = max(y, acc[bi][bj][r]);
                    y = max(y, __shfl_xor(y, 32, 64));
                    if (lane < 32 && y > 0) atomicMax(&b.Y[j0 + wn * WTN + bj * 32 + lane], y);
                }
            }
        } else {
            int8_t *ER = a.eprime + (int64_t)l * 2 * planeC;
            int8_t *EI = ER + planeC;
            const bool karatsuba = KIND == KIND_KARATSUBA;
#pragma unroll
            for (int bi = 0; bi < BM; ++bi)
#pragma unroll
                for (int bj = 0; bj < BN; ++bj)
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const int64_t i = i0 + wm * WTM + bi * 32 + 8 * g + 4 * (lane >> 5);
                        const int64_t j = j0 + wn * WTN + bj * 32 + (lane & 31);
                        int v[4], o[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) v[u] = reduce_acc(acc[bi][bj][4 * g + u], mc);
                        const uint32_t w = keep[bi][bj][g];
                        if (sgi == 0 || (!karatsuba && sgi == 2)) {
                            keep[bi][bj][g] = pack4(v);
                        } else if (sgi == 1) {
                            // Karatsuba: E'_R = mod(D - E), carry mod(D + E); expanded: E'_R = mod(RR - II)
#pragma unroll
                            for (int u = 0; u < 4; ++u) o[u] = reduce_acc(byte_of(w, u) - v[u], mc);
                            *reinterpret_cast<uint32_t *>(ER + j * a.m_pad + i) = pack4(o);
                            if (karatsuba) {
#pragma unroll
                                for (int u = 0; u < 4; ++u) o[u] = reduce_acc(byte_of(w, u) + v[u], mc);
                                keep[bi][bj][g] = pack4(o);
                            }
                        } else {
                            // Karatsuba: E'_I = mod(F - mod(D + E)); expanded: E'_I = mod(RI + IR)
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                o[u] = reduce_acc(karatsuba ? v[u] - byte_of(w, u) : byte_of(w, u) + v[u], mc);
                            *reinterpret_cast<uint32_t *>(EI + j * a.m_pad + i) = pack4(o);
                        }
                    }
        }
    }
}

template <int KIND, typename C>
void launch_kind(const GemmArgs &a, const BoundArgs &b, bool dump, int64_t blocks, hipStream_t s) {
    if (dump) hipLaunchKernelGGL((residue_gemm_kernel<KIND, C, true>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s, a, b);
    else hipLaunchKernelGGL((residue_gemm_kernel<KIND, C, false>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s, a, b);
}

}  // namespace

int gemm_tile_for(int64_t m, int64_t n) { return (m >= 1024 && n >= 1024) ? 256 : 128; }

hipError_t launch_residue_gemm(const GemmArgs &a, hipStream_t s) {
    const int tile = a.tile;
    if ((tile != 128 && tile != 256) || a.m_pad % tile || a.n_pad % tile || a.k_pad % BK || a.nmod < 1)
        return hipErrorInvalidValue;
    const int64_t blocks = (int64_t)a.nmod * (a.m_pad / tile) * (a.n_pad / tile);
    if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    BoundArgs none{};
    const bool dump = a.prods != nullptr;
    if (tile == 256) {
        if (a.algo == 0) launch_kind<KIND_KARATSUBA, CfgLarge>(a, none, dump, blocks, s);
        else launch_kind<KIND_4M, CfgLarge>(a, none, dump, blocks, s);
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
    launch_kind<KIND_BOUND, CfgSmall>(none, b, false, blocks, s);
    return hipGetLastError();
}

}  // namespace ozc
