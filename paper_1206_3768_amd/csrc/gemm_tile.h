// The complex MFMA tile shared by the single-problem GEMM / filter kernels (gemm.hip) and the
// persistent multi-problem filter kernel (batched.hip).
//
// Complex products run as three real products (GAUSS3 below) on v_mfma_f64_16x16x4f64 (FP64) or
// v_mfma_f32_16x16x4f32 (FP32).  The MFMA is used "transposed": its A operand carries op(B)
// (row index = output column j) and its B operand carries op(A) (column index = output row i),
// so that each lane ends up owning output elements of one output row i, and 16 lanes store 16
// consecutive rows of one column: 256 contiguous bytes per store instruction for complex128.
//
// Workgroup = 4 waves (256 threads) computing a BM x BN complex output tile, each wave a
// (BM/2) x (BN/2) sub-tile of 16x16 MFMA blocks.  Operands are staged through LDS in k-stages of
// 16 complex elements, double buffered with one barrier per stage: the global loads of stage s+1
// are in flight while the MFMAs of stage s run.
#pragma once
#include "common.h"

namespace chfsi_tile {

template <typename T> struct CT;
template <> struct CT<double> { typedef double2 c; typedef d4 acc; };
template <> struct CT<float> { typedef float2 c; typedef f4 acc; };

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

template <typename C2> __device__ __forceinline__ C2 cconj(C2 v) { v.y = -v.y; return v; }

// Complex products as three real products (Gauss): re = ArBr - AiBi, im = (Ar + Ai)(Br + Bi) - ArBr -
// AiBi, three MFMAs per complex multiply-add instead of four.  The error bound of the imaginary part
// grows from (|Ar||Bi| + |Ai||Br|) to about (|Ar| + |Ai|)(|Br| + |Bi|) times the same multiple of the
// unit roundoff (Higham, Accuracy and Stability of Numerical Algorithms, section 23.2.4): at most a
// factor 2 on the rounding error of a product, FP64 or FP32.
#ifdef CHFSI_TILE_FOUR_PRODUCTS
constexpr bool GAUSS3 = false;
#else
constexpr bool GAUSS3 = true;
#endif

// Row of the 16x16 MFMA result held in register r of lane l.  Measured on gfx950:
// v_mfma_f32_16x16x4f32 holds row 4 (l/16) + r, v_mfma_f64_16x16x4f64 holds row 4 r + l/16;
// both hold column l % 16.
__device__ __forceinline__ int drow(double, int lane, int r) { return 4 * r + (lane >> 4); }
__device__ __forceinline__ int drow(float, int lane, int r) { return 4 * (lane >> 4) + r; }

template <typename T, int BM, int BN> struct TileShape {
    static constexpr int BK = 16;
    static constexpr int LDA_S = BM + 1, LDB_S = BN + 1;   // +1 element: conflict-free transposed stores
    static constexpr int NPA = BM * BK / 256, NPB = BN * BK / 256;
    static constexpr int MI = BM / 32, NJ = BN / 32;
    static constexpr int AS_ELEMS = BK * LDA_S, BS_ELEMS = BK * LDB_S;   // one LDS buffer
};

// acc[bi][bj] (real and imaginary parts) += op(A)[i0 + rows of the wave, kb:ke] op(B)[kb:ke, j0 + cols]
// for the BM x BN tile at (i0, j0).  As/Bs: two LDS buffers each (2 * AS_ELEMS, 2 * BS_ELEMS).
// Every global load is clamped into the matrix and masked to zero outside it, so any tile
// position and any [kb, ke) inside [0, K) is safe.  Ends without a barrier: a caller that reuses
// As/Bs for another tile must __syncthreads() first.
template <typename T, int OPA, int OPB, int BM, int BN>
__device__ __forceinline__ void tile_mainloop(const typename CT<T>::c* __restrict__ A, int lda, int M,
                                              const typename CT<T>::c* __restrict__ B, int ldb, int N, int i0,
                                              int j0, int kb, int ke, typename CT<T>::c* As,
                                              typename CT<T>::c* Bs,
                                              typename CT<T>::acc (&accr)[BM / 32][BN / 32],
                                              typename CT<T>::acc (&acci)[BM / 32][BN / 32])
{
    typedef typename CT<T>::c C2;
    typedef TileShape<T, BM, BN> S;
    constexpr int BK = S::BK, LDA_S = S::LDA_S, LDB_S = S::LDB_S, NPA = S::NPA, NPB = S::NPB;
    constexpr int MI = S::MI, NJ = S::NJ;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave & 1) * (BM / 2), wc = (wave >> 1) * (BN / 2);
    const int nstages = ke > kb ? (ke - kb + BK - 1) / BK : 0;

    typename CT<T>::acc acc2[MI][NJ];   // T2 of the three-product form (unused with four products)
#pragma unroll
    for (int bi = 0; bi < MI; ++bi)
#pragma unroll
        for (int bj = 0; bj < NJ; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) { accr[bi][bj][r] = 0; acci[bi][bj][r] = 0; acc2[bi][bj][r] = 0; }

    C2 ra[NPA], rb[NPB];

    // element p of a stage tile handled by this thread: op(A) row ai(p), column ak(p); op(B) row
    // bk(p), column bj(p).  Consecutive threads walk the contiguous dimension of the stored matrix.
#define AI(p) ((OPA == OP_N) ? (tid + 256 * (p)) % BM : (tid + 256 * (p)) / BK)
#define AK(p) ((OPA == OP_N) ? (tid + 256 * (p)) / BM : (tid + 256 * (p)) % BK)
#define BJ(p) ((OPB == OP_N) ? (tid + 256 * (p)) / BK : (tid + 256 * (p)) % BN)
#define BKK(p) ((OPB == OP_N) ? (tid + 256 * (p)) % BK : (tid + 256 * (p)) / BN)
#define GEMM_GLOAD(k0)                                                                                    \
    {                                                                                                     \
        _Pragma("unroll") for (int p = 0; p < NPA; ++p) {                                                 \
            const int ci = min(i0 + AI(p), M - 1), ck = min((k0) + AK(p), ke - 1);   /* clamped */       \
            ra[p] = A[(OPA == OP_N) ? (size_t)ci + (size_t)ck * lda : (size_t)ck + (size_t)ci * lda];      \
        }                                                                                                 \
        _Pragma("unroll") for (int p = 0; p < NPB; ++p) {                                                 \
            const int cj = min(j0 + BJ(p), N - 1), ck = min((k0) + BKK(p), ke - 1);                      \
            rb[p] = B[(OPB == OP_N) ? (size_t)ck + (size_t)cj * ldb : (size_t)cj + (size_t)ck * ldb];      \
        }                                                                                                 \
    }
    // the loaded values are masked (outside the matrix or beyond ke: zero) and conjugated only when
    // they are stored to LDS, one stage later, so that no instruction waits on the global loads
    // before the MFMAs of the current stage have been issued
#define GEMM_SSTORE(buf, k0)                                                                              \
    {                                                                                                     \
        _Pragma("unroll") for (int p = 0; p < NPA; ++p) {                                                 \
            const bool ok = i0 + AI(p) < M && (k0) + AK(p) < ke;                                          \
            C2 v;                                                                                         \
            v.x = ok ? ra[p].x : T(0);                                                                    \
            v.y = ok ? ((OPA == OP_N) ? ra[p].y : -ra[p].y) : T(0);                                       \
            As[(buf) * S::AS_ELEMS + AK(p) * LDA_S + AI(p)] = v;                                          \
        }                                                                                                 \
        _Pragma("unroll") for (int p = 0; p < NPB; ++p) {                                                 \
            const bool ok = j0 + BJ(p) < N && (k0) + BKK(p) < ke;                                        \
            C2 v;                                                                                         \
            v.x = ok ? rb[p].x : T(0);                                                                    \
            v.y = ok ? ((OPB == OP_N) ? rb[p].y : -rb[p].y) : T(0);                                       \
            Bs[(buf) * S::BS_ELEMS + BKK(p) * LDB_S + BJ(p)] = v;                                         \
        }                                                                                                 \
    }

    if (nstages > 0) GEMM_GLOAD(kb);
    for (int s = 0; s < nstages; ++s) {
        const int buf = s & 1;
        GEMM_SSTORE(buf, kb + s * BK);
        __syncthreads();
        // the next stage's loads (the last stage reloads itself: in bounds, never stored) are issued
        // unconditionally so that they overlap the MFMAs below
        GEMM_GLOAD(kb + min(s + 1, nstages - 1) * BK);
        asm volatile("" ::: "memory");   // keeps the compiler from sinking the loads below the MFMAs
        const C2* as = As + buf * S::AS_ELEMS;
        const C2* bs = Bs + buf * S::BS_ELEMS;
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            C2 a[MI], b[NJ];
#pragma unroll
            for (int bi = 0; bi < MI; ++bi) a[bi] = as[kr * LDA_S + wr + bi * 16 + (lane & 15)];
#pragma unroll
            for (int bj = 0; bj < NJ; ++bj) b[bj] = bs[kr * LDB_S + wc + bj * 16 + (lane & 15)];
            if constexpr (GAUSS3) {
                // T1 += Bre Are (accr), T2 += Bim Aim (acc2), T3 += (Bre + Bim)(Are + Aim) (acci)
                T as_[MI], bs_[NJ];
#pragma unroll
                for (int bi = 0; bi < MI; ++bi) as_[bi] = a[bi].x + a[bi].y;
#pragma unroll
                for (int bj = 0; bj < NJ; ++bj) bs_[bj] = b[bj].x + b[bj].y;
#pragma unroll
                for (int bi = 0; bi < MI; ++bi)
#pragma unroll
                    for (int bj = 0; bj < NJ; ++bj) {
                        accr[bi][bj] = mfma16(b[bj].x, a[bi].x, accr[bi][bj]);
                        acc2[bi][bj] = mfma16(b[bj].y, a[bi].y, acc2[bi][bj]);
                        acci[bi][bj] = mfma16(bs_[bj], as_[bi], acci[bi][bj]);
                    }
            } else {
                // re += Bre Are ; im += Bim Are   (all blocks), then re -= Bim Aim ; im += Bre Aim
#pragma unroll
                for (int bi = 0; bi < MI; ++bi)
#pragma unroll
                    for (int bj = 0; bj < NJ; ++bj) {
                        accr[bi][bj] = mfma16(b[bj].x, a[bi].x, accr[bi][bj]);
                        acci[bi][bj] = mfma16(b[bj].y, a[bi].x, acci[bi][bj]);
                    }
#pragma unroll
                for (int bi = 0; bi < MI; ++bi)
#pragma unroll
                    for (int bj = 0; bj < NJ; ++bj) {
                        accr[bi][bj] = mfma16(-b[bj].y, a[bi].y, accr[bi][bj]);
                        acci[bi][bj] = mfma16(b[bj].x, a[bi].y, acci[bi][bj]);
                    }
            }
        }
    }
    if constexpr (GAUSS3) {   // re = T1 - T2, im = T3 - T1 - T2
#pragma unroll
        for (int bi = 0; bi < MI; ++bi)
#pragma unroll
            for (int bj = 0; bj < NJ; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const T t1 = accr[bi][bj][r], t2 = acc2[bi][bj][r];
                    accr[bi][bj][r] = t1 - t2;
                    acci[bi][bj][r] = acci[bi][bj][r] - t1 - t2;
                }
    }
#undef GEMM_GLOAD
#undef GEMM_SSTORE
#undef AI
#undef AK
#undef BJ
#undef BKK
}

// output element (i, j) of accumulator register r of block (bi, bj) held by this lane
template <typename T, int BM, int BN>
__device__ __forceinline__ int tile_row(int i0, int bi)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    return i0 + (wave & 1) * (BM / 2) + bi * 16 + (lane & 15);
}
template <typename T, int BM, int BN>
__device__ __forceinline__ int tile_col(int j0, int bj, int r)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    return j0 + (wave >> 1) * (BN / 2) + bj * 16 + drow(T(0), lane, r);
}

}  // namespace chfsi_tile
