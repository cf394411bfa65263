// Per-modulus complex INT8 products on the gfx950 matrix cores with INT32
// accumulation (Section III-A; Algorithm 1 Step V-iii/iv).
//
// One block computes a 128 x 128 output tile of one modulus l (grid z).  The
// products of the chosen algorithm run one after another over the same tile,
// each as a k-loop of v_mfma_i32_32x32x32_i8 over LDS-staged residue tiles;
// between products the INT32 accumulators are reduced to symmetric residues
// in registers, so only the INT8 result E'_l ever leaves the chip:
//   Karatsuba (eq. (10)): D = R.R, E = I.I, F = S.S (S = reduced R + I),
//                         E'_R = mod(D - E), E'_I = mod(F - D - E)
//   expanded  (eq. (7)):  E'_R = mod(RR - II), E'_I = mod(RI + IR)
// A third plan computes the accurate-mode bound product (Section III-B):
//   Cbar_I = Abar_I Bbar_R + Abar_R Bbar_I, Cbar_R = Cbar_I + (Abar_R - Abar_I)(Bbar_R - Bbar_I),
// reduced on the fly to row and column maxima (Cbar is never stored).
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

constexpr int TM = 128, TN = 128, BK = 64;

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

__device__ __forceinline__ uint32_t pack4(int a, int b, int c, int d) {
    return (uint32_t)(a & 0xff) | ((uint32_t)(b & 0xff) << 8) | ((uint32_t)(c & 0xff) << 16) |
           ((uint32_t)(d & 0xff) << 24);
}

__device__ __forceinline__ int swz(int row, int seg) { return row * 4 + (seg ^ ((row >> 1) & 3)); }

template <int KIND, bool DUMP>
__global__ __launch_bounds__(256) void residue_gemm_kernel(GemmArgs a, BoundArgs b) {
    using P = Plan<KIND>;
    __shared__ uint4 ldsA[TM * 4];
    __shared__ uint4 ldsB[TN * 4];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int l = KIND == KIND_BOUND ? 0 : (int)blockIdx.z;
    const int64_t i0 = (int64_t)blockIdx.x * TM, j0 = (int64_t)blockIdx.y * TN;

    const int8_t *Abase = KIND == KIND_BOUND ? b.A : a.A;
    const int8_t *Bbase = KIND == KIND_BOUND ? b.B : a.B;
    const int64_t m_pad = KIND == KIND_BOUND ? b.m_pad : a.m_pad;
    const int64_t n_pad = KIND == KIND_BOUND ? b.n_pad : a.n_pad;
    const int64_t k_pad = KIND == KIND_BOUND ? b.k_pad : a.k_pad;
    const int64_t planeA = m_pad * k_pad, planeB = n_pad * k_pad;
    const int8_t *baseA = Abase + (int64_t)l * P::nplanes * planeA + i0 * k_pad;
    const int8_t *baseB = Bbase + (int64_t)l * P::nplanes * planeB + j0 * k_pad;

    const int lrow = tid >> 2, lseg = tid & 3;
    const int st0 = swz(lrow, lseg), st1 = swz(lrow + 64, lseg);

    ModConst mc;
    if constexpr (KIND != KIND_BOUND) mc = a.tab->mod[l];

    int keep1[2][2][16], keep2[2][2][16];
    v16i acc[2][2];
    int snap[2][2][16];

#pragma unroll 1
    for (int sgi = 0; sgi < P::nseg; ++sgi) {
        const int8_t *Ap = baseA + (int64_t)P::pa(sgi) * planeA + (int64_t)lrow * k_pad + lseg * 16;
        const int8_t *Bp = baseB + (int64_t)P::pb(sgi) * planeB + (int64_t)lrow * k_pad + lseg * 16;
        const int64_t off64 = 64 * k_pad;
        if (KIND != KIND_BOUND || sgi == 0) {
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v16i{};
        }
        uint4 ga0 = *reinterpret_cast<const uint4 *>(Ap);
        uint4 ga1 = *reinterpret_cast<const uint4 *>(Ap + off64);
        uint4 gb0 = *reinterpret_cast<const uint4 *>(Bp);
        uint4 gb1 = *reinterpret_cast<const uint4 *>(Bp + off64);
        for (int64_t k0 = 0; k0 < k_pad; k0 += BK) {
            ldsA[st0] = ga0;
            ldsA[st1] = ga1;
            ldsB[st0] = gb0;
            ldsB[st1] = gb1;
            __syncthreads();
            if (k0 + BK < k_pad) {
                ga0 = *reinterpret_cast<const uint4 *>(Ap + k0 + BK);
                ga1 = *reinterpret_cast<const uint4 *>(Ap + off64 + k0 + BK);
                gb0 = *reinterpret_cast<const uint4 *>(Bp + k0 + BK);
                gb1 = *reinterpret_cast<const uint4 *>(Bp + off64 + k0 + BK);
            }
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int seg = kk * 2 + (lane >> 5);
                v4i fa[2], fb[2];
#pragma unroll
                for (int bi = 0; bi < 2; ++bi) {
                    const int r = wm * 64 + bi * 32 + (lane & 31);
                    const uint4 t = ldsA[swz(r, seg)];
                    fa[bi] = v4i{(int)t.x, (int)t.y, (int)t.z, (int)t.w};
                }
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    const int r = wn * 64 + bj * 32 + (lane & 31);
                    const uint4 t = ldsB[swz(r, seg)];
                    fb[bj] = v4i{(int)t.x, (int)t.y, (int)t.z, (int)t.w};
                }
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj)
                        acc[bi][bj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[bi], fb[bj],
                                                                           acc[bi][bj], 0, 0, 0);
            }
            __syncthreads();
        }

        // ------------------------------------------------ per-product epilogue
        if constexpr (DUMP) {
            const int nprod = P::nseg;
            const int64_t planeC = a.n_pad * a.m_pad;
            int32_t *D = a.prods + ((int64_t)l * nprod + sgi) * planeC;
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int64_t i = i0 + wm * 64 + bi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                        const int64_t j = j0 + wn * 64 + bj * 32 + (lane & 31);
                        D[j * a.m_pad + i] = acc[bi][bj][r];
                    }
        }
        if constexpr (KIND == KIND_KARATSUBA) {
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int v = reduce_acc(acc[bi][bj][r], mc);
                        if (sgi == 0) {
                            keep1[bi][bj][r] = v;                          // D
                        } else if (sgi == 1) {
                            keep2[bi][bj][r] = keep1[bi][bj][r] + v;       // D + E
                            keep1[bi][bj][r] = reduce_acc(keep1[bi][bj][r] - v, mc);  // E'_R
                        } else {
                            keep2[bi][bj][r] = reduce_acc(v - keep2[bi][bj][r], mc);  // E'_I
                        }
                    }
        } else if constexpr (KIND == KIND_4M) {
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int v = reduce_acc(acc[bi][bj][r], mc);
                        if (sgi == 0) keep1[bi][bj][r] = v;
                        else if (sgi == 1) keep1[bi][bj][r] = reduce_acc(keep1[bi][bj][r] - v, mc);
                        else if (sgi == 2) keep2[bi][bj][r] = v;
                        else keep2[bi][bj][r] = reduce_acc(keep2[bi][bj][r] + v, mc);
                    }
        } else {
            if (sgi == 1) {
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                        for (int r = 0; r < 16; ++r) snap[bi][bj][r] = acc[bi][bj][r];  // Cbar_I
            }
        }
    }

    if constexpr (KIND == KIND_BOUND) {
        // v = max(Cbar_R, Cbar_I); X_i = max over j, Y_j = max over i
        int v[2][2][16];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int r = 0; r < 16; ++r) v[bi][bj][r] = max(acc[bi][bj][r], snap[bi][bj][r]);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int x = max(v[bi][0][r], v[bi][1][r]);
#pragma unroll
                for (int off = 16; off >= 1; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
                if ((lane & 31) == 0 && x > 0) {
                    const int64_t i = i0 + wm * 64 + bi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    atomicMax(&b.X[i], x);
                }
            }
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            int y = 0;
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int r = 0; r < 16; ++r) y = max(y, v[bi][bj][r]);
            y = max(y, __shfl_xor(y, 32, 64));
            if (lane < 32 && y > 0) atomicMax(&b.Y[j0 + wn * 64 + bj * 32 + lane], y);
        }
    } else {
        const int64_t planeC = a.n_pad * a.m_pad;
        int8_t *ER = a.eprime + (int64_t)l * 2 * planeC;
        int8_t *EI = ER + planeC;
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int64_t i = i0 + wm * 64 + bi * 32 + 8 * g + 4 * (lane >> 5);
                    const int64_t j = j0 + wn * 64 + bj * 32 + (lane & 31);
                    const int *k1 = &keep1[bi][bj][4 * g];
                    const int *k2 = &keep2[bi][bj][4 * g];
                    *reinterpret_cast<uint32_t *>(ER + j * a.m_pad + i) = pack4(k1[0], k1[1], k1[2], k1[3]);
                    *reinterpret_cast<uint32_t *>(EI + j * a.m_pad + i) = pack4(k2[0], k2[1], k2[2], k2[3]);
                }
    }
}

}  // namespace

hipError_t launch_residue_gemm(const GemmArgs &a, hipStream_t s) {
    if (a.m_pad % TM || a.n_pad % TN || a.k_pad % BK || a.nmod < 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)(a.m_pad / TM), (unsigned)(a.n_pad / TN), (unsigned)a.nmod);
    BoundArgs none{};
    if (a.algo == 0) {
        if (a.prods) hipLaunchKernelGGL((residue_gemm_kernel<KIND_KARATSUBA, true>), grid, dim3(256), 0, s, a, none);
        else hipLaunchKernelGGL((residue_gemm_kernel<KIND_KARATSUBA, false>), grid, dim3(256), 0, s, a, none);
    } else {
        if (a.prods) hipLaunchKernelGGL((residue_gemm_kernel<KIND_4M, true>), grid, dim3(256), 0, s, a, none);
        else hipLaunchKernelGGL((residue_gemm_kernel<KIND_4M, false>), grid, dim3(256), 0, s, a, none);
    }
    return hipGetLastError();
}

hipError_t launch_bound_gemm(const BoundArgs &b, hipStream_t s) {
    if (b.m_pad % TM || b.n_pad % TN || b.k_pad % BK) return hipErrorInvalidValue;
    dim3 grid((unsigned)(b.m_pad / TM), (unsigned)(b.n_pad / TN), 1);
    GemmArgs none{};
    hipLaunchKernelGGL((residue_gemm_kernel<KIND_BOUND, false>), grid, dim3(256), 0, s, none, b);
    return hipGetLastError();
}

}  // namespace ozc
