// Cholesky factorisation S = L L^H (lower) of the reduction to standard form (Section 3.2), blocked
// right-looking with 64-column panels:
//   k_chol_panel  one workgroup per 64-row block of the panel: every workgroup factors the 64 x 64
//                 diagonal block in LDS (redundantly, which costs less than a second launch);
//                 workgroup 0 writes L11, workgroup b > 0 solves L21_b L11^H = A21_b by forward
//                 substitution in LDS.
//   trailing      A22 <- A22 - L21 L21^H with the MFMA complex GEMM of gemm.hip.
// A non-positive (or non-finite) pivot sets *info to its 1-based column, as LAPACK's potrf does;
// the factorisation then continues on meaningless numbers and the caller discards the result.
// Only the lower triangle of the input is read; the strict upper triangle of the result is left as
// the trailing updates made it (callers zero it).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace {

constexpr int CB = 64;          // panel width
constexpr int CP = CB + 1;      // LDS pitch

__device__ inline zd zsub_mul_conj(zd acc, zd a, zd b)   // acc - a conj(b)
{
    acc.x -= a.x * b.x + a.y * b.y;
    acc.y -= a.y * b.x - a.x * b.y;
    return acc;
}

__global__ __launch_bounds__(256) void k_chol_panel(int n, int k0, zd* __restrict__ A, int lda, int* __restrict__ info)
{
    __shared__ zd L[CB * CP];    // diagonal block, factored in place (lower)
    __shared__ zd X[CB * CP];    // the row block being solved
    __shared__ double piv;
    const int tid = threadIdx.x;
    const int nb = min(CB, n - k0);
    // diagonal block (lower triangle mirrored; identity padding beyond nb)
    for (int e = tid; e < CB * CB; e += 256) {
        const int i = e % CB, j = e / CB;
        zd v = make_double2(i == j ? 1.0 : 0.0, 0.0);
        if (i < nb && j < nb) {
            if (i >= j) v = A[(size_t)(k0 + i) + (size_t)(k0 + j) * lda];
            else {
                const zd u = A[(size_t)(k0 + j) + (size_t)(k0 + i) * lda];
                v = make_double2(u.x, -u.y);
            }
            if (i == j) v.y = 0.0;
        }
        L[i * CP + j] = v;
    }
    __syncthreads();
    // unblocked right-looking Cholesky of the 64 x 64 block
    for (int k = 0; k < CB; ++k) {
        if (tid == 0) {
            const double d = L[k * CP + k].x;
            piv = d;
            if (!(d > 0.0) && blockIdx.x == 0 && k < nb && info) atomicCAS(info, 0, k0 + k + 1);
            L[k * CP + k] = make_double2(sqrt(d > 0.0 ? d : 1.0), 0.0);
        }
        __syncthreads();
        const double inv = 1.0 / sqrt(piv > 0.0 ? piv : 1.0);
        for (int i = k + 1 + tid; i < CB; i += 256) {
            zd v = L[i * CP + k];
            L[i * CP + k] = make_double2(v.x * inv, v.y * inv);
        }
        __syncthreads();
        const int rem = CB - k - 1;
        for (int e = tid; e < rem * rem; e += 256) {
            const int i = k + 1 + e % rem, j = k + 1 + e / rem;
            if (i >= j) L[i * CP + j] = zsub_mul_conj(L[i * CP + j], L[i * CP + k], L[j * CP + k]);
        }
        __syncthreads();
    }
    if (blockIdx.x == 0) {
        for (int e = tid; e < nb * nb; e += 256) {
            const int i = e % nb, j = e / nb;
            if (i >= j) A[(size_t)(k0 + i) + (size_t)(k0 + j) * lda] = L[i * CP + j];
        }
        return;
    }
    const int r0 = k0 + blockIdx.x * CB;            // first row of this row block
    const int nr = min(CB, n - r0);
    // L21 rows by forward substitution, x L11^H = a for each row: x_j = (a_j - sum_{l < j} x_l
    // conj(L_jl)) / L_jj.  Four lanes per row (one wave holds 16 rows) split each sum and combine
    // it with shuffles; one barrier per column makes x_j visible to the next column.
    for (int e = tid; e < CB * CB; e += 256) {
        const int r = e % CB, l = e / CB;
        X[r * CP + l] = (r < nr && l < nb) ? A[(size_t)(r0 + r) + (size_t)(k0 + l) * lda] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int r = tid >> 2, t = tid & 3;
    for (int j = 0; j < nb; ++j) {
        zd acc = make_double2(0.0, 0.0);
        for (int l = t; l < j; l += 4) acc = zsub_mul_conj(acc, X[r * CP + l], L[j * CP + l]);
        acc.x += __shfl_xor(acc.x, 1);
        acc.y += __shfl_xor(acc.y, 1);
        acc.x += __shfl_xor(acc.x, 2);
        acc.y += __shfl_xor(acc.y, 2);
        if (t == 0) {
            const double d = 1.0 / L[j * CP + j].x;
            const zd a = X[r * CP + j];
            X[r * CP + j] = make_double2((a.x + acc.x) * d, (a.y + acc.y) * d);
        }
        __syncthreads();
    }
    for (int e = tid; e < nr * nb; e += 256) {
        const int rr = e % nr, l = e / nr;
        A[(size_t)(r0 + rr) + (size_t)(k0 + l) * lda] = X[rr * CP + l];
    }
}

}  // namespace

// L L^H = A (n x n, lower triangle of A read, L written in place).  *info (device, zeroed by the
// caller) receives the first non-positive pivot (1-based) or stays 0.  gw: workspace of the
// trailing GEMMs.  Returns hipError_t as int.
int chol_lower(hipStream_t s, int n, zd* A, int lda, int* info, const GemmWs& gw)
{
    for (int k0 = 0; k0 < n; k0 += CB) {
        const int nb = std::min(CB, n - k0);
        const int rows = n - k0;
        const int blocks = (rows + CB - 1) / CB;
        hipLaunchKernelGGL(k_chol_panel, dim3(blocks), dim3(256), 0, s, n, k0, A, lda, info);
        int rc = (int)hipGetLastError();
        if (rc != 0) return rc;
        const int m2 = rows - nb;
        if (m2 > 0) {
            zd* L21 = A + (size_t)(k0 + nb) + (size_t)k0 * lda;
            zd* A22 = A + (size_t)(k0 + nb) + (size_t)(k0 + nb) * lda;
            rc = launch_zgemm(s, OP_N, OP_C, m2, m2, nb, -1.0, L21, lda, L21, lda, 1.0, A22, lda, gw);
            if (rc != 0) return rc;
        }
    }
    return 0;
}
