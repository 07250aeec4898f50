// Inverse of a 64 x 64 lower-triangular block held in LDS, for the diagonal blocks of the Cholesky
// factorisation and the triangular solves, blockwise with 16 x 16 blocks:
//   X_kk = L_kk^{-1}                                   (k = 0 .. 3: one wave each, a 16-step
//                                                      substitution with the given reciprocals)
//   X_ij = -X_ii  sum_{k = j}^{i - 1} L_ik X_kj        (i > j, by increasing distance i - j, one
//                                                      wave per block, on MFMA)
#pragma once
#include "common.h"
#include "gemm_tile.h"

namespace tri64 {

constexpr int N = 64, P = 65, B = 16;

// v from lane ^ 1 and lane ^ 2 of the same quad (DPP quad permutations [1,0,3,2], [2,3,0,1])
template <int CTRL> __device__ inline double quad_perm(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// L: lower triangle with zeros above the diagonal (pitch P); rinv[k] = 1 / L_kk (L's diagonal is
// real).  X receives L^{-1} in its lower block triangle: the diagonal 16 x 16 blocks in full (zeros
// above their diagonal), the blocks below them; the blocks above are not written.  256 threads;
// ends with a barrier.
__device__ __forceinline__ void lower_inverse(const zd* L, const double* rinv, zd* X)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // diagonal blocks: wave w substitutes block w; lane = 4 c + t takes column c and, of the
    // column's entries x_r, the ones with r % 4 == t (in registers; zero until computed, so that the
    // sums need no bounds)
    {
        const int o = wave * B, c = lane >> 2, t = lane & 3;
        zd x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < B; ++i) {
            double ar = 0.0, ai = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const zd l = L[(o + i) * P + o + 4 * q + t];
                ar = __builtin_fma(l.x, x[q].x, ar);
                ar = __builtin_fma(-l.y, x[q].y, ar);
                ai = __builtin_fma(l.x, x[q].y, ai);
                ai = __builtin_fma(l.y, x[q].x, ai);
            }
            ar += quad_perm<0xB1>(ar);
            ai += quad_perm<0xB1>(ai);
            ar += quad_perm<0x4E>(ar);
            ai += quad_perm<0x4E>(ai);
            const double d = rinv[o + i];
            const bool live = i >= c, mine = (i & 3) == t;
            const double vr = live ? ((i == c ? 1.0 : 0.0) - ar) * d : 0.0;
            const double vi = live ? -ai * d : 0.0;
            x[i >> 2].x = mine ? vr : x[i >> 2].x;
            x[i >> 2].y = mine ? vi : x[i >> 2].y;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) X[(o + 4 * q + t) * P + o + c] = x[q];
    }
    __syncthreads();
    // off-diagonal blocks.  T = sum_k L_ik X_kj is formed transposed (T^T = sum_k X_kj^T L_ik^T),
    // which leaves in register r of lane l the entry T[4 r + (l >> 4)][l & 15]: the B operand of
    // step r of the product X_ii T.
    const int lr = lane & 15, lk = lane >> 4;
    for (int dist = 1; dist < 4; ++dist) {
        if (wave < 4 - dist) {
            const int jb = wave, ib = wave + dist;
            d4 tr, ti;
#pragma unroll
            for (int r = 0; r < 4; ++r) { tr[r] = 0.0; ti[r] = 0.0; }
            for (int kb = jb; kb < ib; ++kb)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 4 * kk + lk;
                    const zd a = X[(kb * B + k) * P + jb * B + lr];   // (X_kj^T)[lr][k]
                    const zd b = L[(ib * B + lr) * P + kb * B + k];   // (L_ik^T)[k][lr]
                    tr = chfsi_tile::mfma16(b.x, a.x, tr);
                    tr = chfsi_tile::mfma16(-b.y, a.y, tr);
                    ti = chfsi_tile::mfma16(b.y, a.x, ti);
                    ti = chfsi_tile::mfma16(b.x, a.y, ti);
                }
            d4 xr, xi;
#pragma unroll
            for (int r = 0; r < 4; ++r) { xr[r] = 0.0; xi[r] = 0.0; }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const zd a = X[(ib * B + lr) * P + ib * B + 4 * kk + lk];   // X_ii[lr][k]
                xr = chfsi_tile::mfma16(tr[kk], a.x, xr);
                xr = chfsi_tile::mfma16(-ti[kk], a.y, xr);
                xi = chfsi_tile::mfma16(ti[kk], a.x, xi);
                xi = chfsi_tile::mfma16(tr[kk], a.y, xi);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                X[(ib * B + lr) * P + jb * B + 4 * r + lk] = make_double2(-xr[r], -xi[r]);
        }
        __syncthreads();
    }
}

}  // namespace tri64
