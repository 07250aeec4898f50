// Triangular solves with the Cholesky factor L (lower, n x n) of the reduction to standard form
// and of Cholesky QR: blocked substitution with 64 x 64 diagonal blocks (inverted in LDS, then
// applied as a product) and the off-diagonal updates on the MFMA complex GEMM of gemm.hip.
//   trsm_left_lower   L X = B          (H = L^{-1} A, first half of the reduction)
//   trsm_left_lower_h L^H X = B        (X = L^{-H} V, back-transform of the eigenvectors)
//   trsm_right_lower_h X L^H = B       (H = W L^{-H}, second half; Q = Y R^{-1} of Cholesky QR)
// Each solve runs over the 64-blocks of the triangular dimension in dependency order: the
// diagonal-block kernel solves one block row (or column) of B, then one GEMM subtracts its
// contribution from the rest.  Only the lower triangle of L is read.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "tri64.h"

namespace {

constexpr int TB = 64;        // block size
constexpr int TP = TB + 1;    // LDS pitch

enum { RL_C = 0, LL_N = 1, LL_C = 2 };

__device__ inline zd zfma(zd acc, zd a, zd b, double sgn)   // acc + sgn a b
{
    acc.x += sgn * (a.x * b.x - a.y * b.y);
    acc.y += sgn * (a.x * b.y + a.y * b.x);
    return acc;
}
__device__ inline zd zc(zd a) { return make_double2(a.x, -a.y); }

// Solves the diagonal block k0 .. k0 + nb of L against 64 vectors of B per workgroup.
//   RL_C: vectors are rows r of B(:, k0:k0+nb):   x L_kk^H = b,  x_v = sum_l b_l conj(X_vl)
//   LL_N: vectors are columns c of B(k0:k0+nb, :): L_kk x = b,    x_v = sum_l X_vl b_l
//   LL_C: vectors are columns c of B(k0:k0+nb, :): L_kk^H x = b,  x_v = sum_l conj(X_lv) b_l
// with X = L_kk^{-1} (tri64.h).  nvec: number of vectors (rows of B for RL_C, columns for LL_*).
// Each thread computes a 4 x 4 block of (vector, position) outputs.
template <int MODE>
__global__ __launch_bounds__(256) void k_trsm_diag(int k0, int nb, int nvec, const zd* __restrict__ L, int ldl,
                                                   zd* __restrict__ B, int ldb)
{
    __shared__ zd T[TB * TP];   // L_kk (lower, identity padding), then the coefficient table
    __shared__ zd X[TB * TP];   // L_kk^{-1}, then the vectors: X[u][v]
    const int tid = threadIdx.x;
    const int v0 = blockIdx.x * TB;
    const int nv = min(TB, nvec - v0);
    #pragma unroll
    for (int e = tid; e < TB * TB; e += 256) {
        const int i = e % TB, j = e / TB;
        zd t = make_double2(i == j ? 1.0 : 0.0, 0.0);
        if (i < nb && j < nb && i >= j) t = L[(size_t)(k0 + i) + (size_t)(k0 + j) * ldl];
        T[i * TP + j] = t;
    }
    __syncthreads();
    tri64::lower_inverse(T, X);
    // coefficient table C[l][v] (contiguous in v for the product below):
    //   LL_N: X[v][l],  LL_C: conj(X[l][v]),  RL_C: conj(X[v][l])
    #pragma unroll
    for (int e = tid; e < TB * TB; e += 256) {
        const int v = e % TB, l = e / TB;
        T[l * TP + v] = (MODE == LL_N) ? X[v * TP + l] : (MODE == LL_C) ? zc(X[l * TP + v]) : zc(X[v * TP + l]);
    }
    __syncthreads();
    #pragma unroll
    for (int e = tid; e < TB * TB; e += 256) {   // vector u = i, position v = j into X; consecutive
        // threads walk the contiguous dimension of B (vectors for RL_C, positions for LL_*)
        const int i = (MODE == RL_C) ? e % TB : e / TB, j = (MODE == RL_C) ? e / TB : e % TB;
        zd b = make_double2(0.0, 0.0);
        if (i < nv && j < nb)
            b = (MODE == RL_C) ? B[(size_t)(v0 + i) + (size_t)(k0 + j) * ldb] : B[(size_t)(k0 + j) + (size_t)(v0 + i) * ldb];
        X[i * TP + j] = b;
    }
    __syncthreads();
    const int ug = (tid >> 4) * 4, vg = (tid & 15) * 4;
    zd acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = make_double2(0.0, 0.0);
    for (int l = 0; l < TB; ++l) {
        zd bv[4], cf[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) bv[a] = X[(ug + a) * TP + l];
#pragma unroll
        for (int c = 0; c < 4; ++c) cf[c] = T[l * TP + vg + c];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][c] = zfma(acc[a][c], cf[c], bv[a], 1.0);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = ug + a, j = vg + c;
            if (i < nv && j < nb) {
                if (MODE == RL_C) B[(size_t)(v0 + i) + (size_t)(k0 + j) * ldb] = acc[a][c];
                else B[(size_t)(k0 + j) + (size_t)(v0 + i) * ldb] = acc[a][c];
            }
        }
}

template <int MODE>
int diag(hipStream_t s, int k0, int nb, int nvec, const zd* L, int ldl, zd* B, int ldb)
{
    if (nvec <= 0) return 0;
    hipLaunchKernelGGL((k_trsm_diag<MODE>), dim3((nvec + TB - 1) / TB), dim3(256), 0, s, k0, nb, nvec, L, ldl, B, ldb);
    return (int)hipGetLastError();
}

}  // namespace

// L X = B, L n x n lower, B n x nrhs (overwritten by X).
int trsm_left_lower(hipStream_t s, int n, int nrhs, const zd* L, int ldl, zd* B, int ldb, const GemmWs& gw)
{
    for (int k0 = 0; k0 < n; k0 += TB) {
        const int nb = std::min(TB, n - k0);
        int rc = diag<LL_N>(s, k0, nb, nrhs, L, ldl, B, ldb);
        if (rc != 0) return rc;
        const int rest = n - k0 - nb;
        if (rest > 0) {   // B(k0+nb:, :) -= L(k0+nb:, k0:k0+nb) X(k0:k0+nb, :)
            rc = launch_zgemm(s, OP_N, OP_N, rest, nrhs, nb, -1.0, L + (size_t)(k0 + nb) + (size_t)k0 * ldl, ldl,
                              B + k0, ldb, 1.0, B + k0 + nb, ldb, gw);
            if (rc != 0) return rc;
        }
    }
    return 0;
}

// L^H X = B, L n x n lower, B n x nrhs (overwritten by X).
int trsm_left_lower_h(hipStream_t s, int n, int nrhs, const zd* L, int ldl, zd* B, int ldb, const GemmWs& gw)
{
    const int nblk = (n + TB - 1) / TB;
    for (int kb = nblk - 1; kb >= 0; --kb) {
        const int k0 = kb * TB, nb = std::min(TB, n - k0);
        int rc = diag<LL_C>(s, k0, nb, nrhs, L, ldl, B, ldb);
        if (rc != 0) return rc;
        if (k0 > 0) {   // B(0:k0, :) -= L(k0:k0+nb, 0:k0)^H X(k0:k0+nb, :)
            rc = launch_zgemm(s, OP_C, OP_N, k0, nrhs, nb, -1.0, L + k0, ldl, B + k0, ldb, 1.0, B, ldb, gw);
            if (rc != 0) return rc;
        }
    }
    return 0;
}

// X L^H = B, L ncol x ncol lower, B nrow x ncol (overwritten by X).
int trsm_right_lower_h(hipStream_t s, int nrow, int ncol, const zd* L, int ldl, zd* B, int ldb, const GemmWs& gw)
{
    for (int k0 = 0; k0 < ncol; k0 += TB) {
        const int nb = std::min(TB, ncol - k0);
        int rc = diag<RL_C>(s, k0, nb, nrow, L, ldl, B, ldb);
        if (rc != 0) return rc;
        const int rest = ncol - k0 - nb;
        if (rest > 0) {   // B(:, k0+nb:) -= X(:, k0:k0+nb) L(k0+nb:, k0:k0+nb)^H
            rc = launch_zgemm(s, OP_N, OP_C, nrow, rest, nb, -1.0, B + (size_t)k0 * ldb, ldb,
                              L + (size_t)(k0 + nb) + (size_t)k0 * ldl, ldl, 1.0, B + (size_t)(k0 + nb) * ldb, ldb, gw);
            if (rc != 0) return rc;
        }
    }
    return 0;
}
