// Cholesky factorisation S = L L^H (lower) of the reduction to standard form (Section 3.2), blocked
// right-looking with 64-column panels:
//   k_chol_panel  one workgroup per 64-row block of the panel: every workgroup factors the 64 x 64
//                 diagonal block in LDS (redundantly, which costs less than a second launch);
//                 workgroup 0 writes L11, workgroup b > 0 inverts L11 in LDS (tri64.h) and forms
//                 L21_b = A21_b L11^{-H} as a product.
//   trailing      A22 <- A22 - L21 L21^H with the MFMA complex GEMM of gemm.hip.
// A non-positive (or non-finite) pivot sets *info to its 1-based column, as LAPACK's potrf does;
// the factorisation then continues on meaningless numbers and the caller discards the result.
// Only the lower triangle of the input is read; the strict upper triangle of the result is left as
// the trailing updates made it (callers zero it).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "tri64.h"

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
    __shared__ zd X[CB * CP];    // L11^{-1}
    const int tid = threadIdx.x;
    const int nb = min(CB, n - k0);
    // diagonal block: lower triangle (the upper is never read), identity padding beyond nb
    #pragma unroll
    for (int e = tid; e < CB * CB; e += 256) {
        const int i = e % CB, j = e / CB;
        zd v = make_double2(i == j ? 1.0 : 0.0, 0.0);
        if (i < nb && j < nb && i >= j) {
            v = A[(size_t)(k0 + i) + (size_t)(k0 + j) * lda];
            if (i == j) v.y = 0.0;
        }
        L[i * CP + j] = v;
    }
    __syncthreads();
    // right-looking Cholesky of the 64 x 64 block, four columns at a time: wave 0 factors the
    // 64 x 4 column panel in registers (lane = row, diagonal entries shared by shuffles), then all
    // threads apply the rank-4 update to the trailing lower triangle
    const int lane = tid & 63;
    for (int k = 0; k < CB; k += 4) {
        if (tid < 64) {
            zd v[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = L[lane * CP + k + c];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int kc = k + c;
                const double d = __shfl(v[c].x, kc);
                if (lane == 0 && !(d > 0.0) && blockIdx.x == 0 && kc < nb && info) atomicCAS(info, 0, k0 + kc + 1);
                const double sd = sqrt(d > 0.0 ? d : 1.0), inv = 1.0 / sd;
                if (lane > kc) v[c] = make_double2(v[c].x * inv, v[c].y * inv);
                else if (lane == kc) v[c] = make_double2(sd, 0.0);
#pragma unroll
                for (int j = c + 1; j < 4; ++j) {   // columns k + j of the panel, rows >= k + j
                    const double lr = __shfl(v[c].x, k + j), li = __shfl(v[c].y, k + j);
                    if (lane >= k + j) v[j] = zsub_mul_conj(v[j], v[c], make_double2(lr, li));
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (lane >= k + c) L[lane * CP + k + c] = v[c];
        }
        __syncthreads();
        const int r0t = k + 4, rem = CB - r0t;
        for (int e = tid; e < rem * rem; e += 256) {
            const int i = r0t + e % rem, j = r0t + e / rem;
            if (i < j) continue;
            zd acc = L[i * CP + j];
#pragma unroll
            for (int c = 0; c < 4; ++c) acc = zsub_mul_conj(acc, L[i * CP + k + c], L[j * CP + k + c]);
            L[i * CP + j] = acc;
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
    // L21 = A21 L11^{-H}: row r, column v: sum_l A21(r, l) conj(X(v, l)), X = L11^{-1}; the
    // coefficient table conj(X(v, l)) goes to L (transposed, contiguous in v), the rows of A21 to X
    tri64::lower_inverse(L, X);
    #pragma unroll
    for (int e = tid; e < CB * CB; e += 256) {   // L[l][v] = conj(X[v][l]), contiguous in v
        const int v = e % CB, l = e / CB;
        const zd x = X[v * CP + l];
        L[l * CP + v] = make_double2(x.x, -x.y);
    }
    __syncthreads();
    #pragma unroll
    for (int e = tid; e < CB * CB; e += 256) {
        const int r = e % CB, l = e / CB;
        X[r * CP + l] = (r < nr && l < nb) ? A[(size_t)(r0 + r) + (size_t)(k0 + l) * lda] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int rg = (tid >> 4) * 4, vg = (tid & 15) * 4;
    zd acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = make_double2(0.0, 0.0);
    for (int l = 0; l < CB; ++l) {
        zd av[4], xv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = X[(rg + a) * CP + l];
#pragma unroll
        for (int c = 0; c < 4; ++c) xv[c] = L[l * CP + vg + c];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) {   // acc += a xv  (xv holds conj(X[v][l]))
                acc[a][c].x += av[a].x * xv[c].x - av[a].y * xv[c].y;
                acc[a][c].y += av[a].y * xv[c].x + av[a].x * xv[c].y;
            }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int r = rg + a, v = vg + c;
            if (r < nr && v < nb) A[(size_t)(r0 + r) + (size_t)(k0 + v) * lda] = acc[a][c];
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
