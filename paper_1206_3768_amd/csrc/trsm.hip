// Triangular solves with the Cholesky factor L (lower, n x n) of the reduction to standard form
// and of Cholesky QR: blocked substitution with 64 x 64 diagonal blocks solved in LDS and the
// off-diagonal updates on the MFMA complex GEMM of gemm.hip.
//   trsm_left_lower   L X = B          (H = L^{-1} A, first half of the reduction)
//   trsm_left_lower_h L^H X = B        (X = L^{-H} V, back-transform of the eigenvectors)
//   trsm_right_lower_h X L^H = B       (H = W L^{-H}, second half; Q = Y R^{-1} of Cholesky QR)
// Each solve runs over the 64-blocks of the triangular dimension in dependency order: the
// diagonal-block kernel solves one block row (or column) of B, then one GEMM subtracts its
// contribution from the rest.  Only the lower triangle of L is read.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

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
//   RL_C: vectors are rows r of B(:, k0:k0+nb):   x L_kk^H = b  (forward)
//   LL_N: vectors are columns c of B(k0:k0+nb, :): L_kk x = b    (forward)
//   LL_C: vectors are columns c of B(k0:k0+nb, :): L_kk^H x = b  (backward)
// nvec: number of vectors (rows of B for RL_C, columns for LL_*).  Four lanes per vector split
// each dot product and combine it with shuffles; one barrier per position.
template <int MODE>
__global__ __launch_bounds__(256) void k_trsm_diag(int k0, int nb, int nvec, const zd* __restrict__ L, int ldl,
                                                   zd* __restrict__ B, int ldb)
{
    __shared__ zd T[TB * TP];   // L_kk (lower), identity padding
    __shared__ zd X[TB * TP];   // X[u][v]: vector u, position v
    const int tid = threadIdx.x;
    const int v0 = blockIdx.x * TB;
    const int nv = min(TB, nvec - v0);
    for (int e = tid; e < TB * TB; e += 256) {
        const int i = e % TB, j = e / TB;
        zd t = make_double2(i == j ? 1.0 : 0.0, 0.0);
        if (i < nb && j < nb && i >= j) t = L[(size_t)(k0 + i) + (size_t)(k0 + j) * ldl];
        T[i * TP + j] = (i >= j || i >= nb || j >= nb) ? t : make_double2(0.0, 0.0);
        // vector u = i, position v = j
        zd b = make_double2(0.0, 0.0);
        if (i < nv && j < nb)
            b = (MODE == RL_C) ? B[(size_t)(v0 + i) + (size_t)(k0 + j) * ldb] : B[(size_t)(k0 + j) + (size_t)(v0 + i) * ldb];
        X[i * TP + j] = b;
    }
    __syncthreads();
    const int u = tid >> 2, t = tid & 3;
    for (int s = 0; s < nb; ++s) {
        const int v = (MODE == LL_C) ? nb - 1 - s : s;
        zd acc = make_double2(0.0, 0.0);
        if (MODE == LL_C) {
            for (int l = v + 1 + t; l < nb; l += 4) acc = zfma(acc, zc(T[l * TP + v]), X[u * TP + l], -1.0);
        } else {
            for (int l = t; l < v; l += 4) {
                const zd c = (MODE == RL_C) ? zc(T[v * TP + l]) : T[v * TP + l];
                acc = zfma(acc, c, X[u * TP + l], -1.0);
            }
        }
        acc.x += __shfl_xor(acc.x, 1);
        acc.y += __shfl_xor(acc.y, 1);
        acc.x += __shfl_xor(acc.x, 2);
        acc.y += __shfl_xor(acc.y, 2);
        if (t == 0) {
            const double d = 1.0 / T[v * TP + v].x;
            const zd b = X[u * TP + v];
            X[u * TP + v] = make_double2((b.x + acc.x) * d, (b.y + acc.y) * d);
        }
        __syncthreads();
    }
    for (int e = tid; e < nv * nb; e += 256) {
        const int i = e % nv, j = e / nv;
        if (MODE == RL_C) B[(size_t)(v0 + i) + (size_t)(k0 + j) * ldb] = X[i * TP + j];
        else B[(size_t)(k0 + j) + (size_t)(v0 + i) * ldb] = X[i * TP + j];
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
