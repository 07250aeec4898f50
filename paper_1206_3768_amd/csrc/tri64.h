// Inverse of a 64 x 64 lower-triangular block held in LDS, for the diagonal blocks of the Cholesky
// factorisation and the triangular solves: blockwise with 16 x 16 blocks, so that the sequential
// part is a 16-step substitution per diagonal block (one wave each, register resident) and the rest
// is small matrix products over all 256 threads.
//   X_kk = L_kk^{-1}                                   (k = 0 .. 3, one wave per block)
//   X_ij = -X_ii  sum_{k = j}^{i - 1} L_ik X_kj        (i > j, by increasing distance i - j)
#pragma once
#include "common.h"

namespace tri64 {

constexpr int N = 64, P = 65, B = 16;

__device__ inline zd cmul(zd a, zd b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline zd cadd(zd a, zd b) { return make_double2(a.x + b.x, a.y + b.y); }

// v from lane ^ 1 and lane ^ 2 of the same quad (DPP quad permutations [1,0,3,2], [2,3,0,1])
template <int CTRL> __device__ inline double quad_perm(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// L: lower triangle read (pitch P); X: receives L^{-1}, lower, zeros above the diagonal.  L's
// diagonal must be real and nonzero.  256 threads; ends with a barrier.
__device__ inline void lower_inverse(const zd* L, zd* X)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // zero the strict upper triangle and the off-diagonal blocks' upper parts
#pragma unroll
    for (int e = tid; e < N * N; e += 256) {
        const int i = e % N, j = e / N;
        if (i < j) X[i * P + j] = make_double2(0.0, 0.0);
    }
    // diagonal 16 x 16 blocks: wave w inverts block w; lane = 4 c + t handles column c, and of the
    // column's entries x_r the ones with r % 4 == t (kept in registers)
    {
        const int o = wave * B, c = lane >> 2, t = lane & 3;
        zd x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < B; ++i) {
            zd acc = make_double2(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int l = 4 * q + t;
                if (l < i && l >= c) acc = cadd(acc, cmul(L[(o + i) * P + o + l], x[q]));
            }
            acc.x += quad_perm<0xB1>(acc.x);
            acc.y += quad_perm<0xB1>(acc.y);
            acc.x += quad_perm<0x4E>(acc.x);
            acc.y += quad_perm<0x4E>(acc.y);
            const double d = 1.0 / L[(o + i) * P + o + i].x;
            const zd v = (i < c) ? make_double2(0.0, 0.0)
                                 : make_double2(((i == c ? 1.0 : 0.0) - acc.x) * d, -acc.y * d);
            if ((i & 3) == t) x[i >> 2] = v;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) X[(o + 4 * q + t) * P + o + c] = x[q];
    }
    __syncthreads();
    // off-diagonal blocks by distance: T = sum_k L_ik X_kj, then X_ij = -X_ii T
    __shared__ zd Tb[3 * B * B];
    // (each thread takes elements tid, tid + 256, tid + 512 of the nblk blocks at once, and each sum
    // runs in two halves, so that several independent chains of LDS reads and FMAs are in flight)
    for (int dist = 1; dist < 4; ++dist) {
        const int nblk = 4 - dist;                    // blocks (i, j) = (j + dist, j), j < nblk
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int e = tid + 256 * s;
            if (e < nblk * B * B) {
                const int jb = e / (B * B), r = (e / B) % B, c = e % B;
                const int ib = jb + dist;
                zd acc0 = make_double2(0.0, 0.0), acc1 = acc0;
                for (int kb = jb; kb < ib; ++kb)
#pragma unroll
                    for (int k = 0; k < B; k += 2) {
                        acc0 = cadd(acc0, cmul(L[(ib * B + r) * P + kb * B + k], X[(kb * B + k) * P + jb * B + c]));
                        acc1 = cadd(acc1, cmul(L[(ib * B + r) * P + kb * B + k + 1],
                                               X[(kb * B + k + 1) * P + jb * B + c]));
                    }
                Tb[e] = cadd(acc0, acc1);
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int e = tid + 256 * s;
            if (e < nblk * B * B) {
                const int jb = e / (B * B), r = (e / B) % B, c = e % B;
                const int ib = jb + dist;
                zd acc0 = make_double2(0.0, 0.0), acc1 = acc0;
#pragma unroll
                for (int k = 0; k < B; k += 2) {
                    acc0 = cadd(acc0, cmul(X[(ib * B + r) * P + ib * B + k], Tb[jb * B * B + k * B + c]));
                    acc1 = cadd(acc1, cmul(X[(ib * B + r) * P + ib * B + k + 1], Tb[jb * B * B + (k + 1) * B + c]));
                }
                const zd acc = cadd(acc0, acc1);
                X[(ib * B + r) * P + jb * B + c] = make_double2(-acc.x, -acc.y);
            }
        }
        __syncthreads();
    }
}

}  // namespace tri64
