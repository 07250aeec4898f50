// Cholesky factorisation S = L L^H (lower) of the reduction to standard form (Section 3.2), blocked
// right-looking with 64-column panels:
//   k_chol_diag   one workgroup factors the 64 x 64 diagonal block in LDS, writes L11 and stores
//                 L11^{-1} (tri64.h) for this factorisation and the later triangular solves;
//   L21           L21 = A21 L11^{-H}, in place, as an MFMA product with the stored inverse (trsm.hip);
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

// value of v in lane `lane` (wave-uniform) of the wave
__device__ inline double readlane_d(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ inline zd zsub_mul_conj(zd acc, zd a, zd b)   // acc - a conj(b)
{
    acc.x -= a.x * b.x + a.y * b.y;
    acc.y -= a.y * b.x - a.x * b.y;
    return acc;
}

// Factors the nb x nb (nb <= 64) diagonal block at A in LDS (one workgroup), writes L11 to A and
// L11^{-1} (64 x 64, column-major, zero above the diagonal, identity beyond nb) to D.  col0: global
// index of the block's first column (for the pivot reported in *info).
__global__ __launch_bounds__(256) void k_chol_diag(int nb, int col0, zd* __restrict__ A, int lda,
                                                   int* __restrict__ info, zd* __restrict__ D)
{
    __shared__ zd L[CB * CP];    // diagonal block, factored in place (lower)
    __shared__ zd X[CB * CP];    // L11^{-1}
    const int tid = threadIdx.x;
    // lower triangle (the upper is never read), identity padding beyond nb: all 16 loads of a
    // thread are issued (clamped into the block) before any is used
    {
        zd v[CB * CB / 256];
#pragma unroll
        for (int p = 0; p < CB * CB / 256; ++p) {
            const int e = tid + 256 * p, i = e % CB, j = e / CB;
            v[p] = A[(size_t)min(i, nb - 1) + (size_t)min(j, nb - 1) * lda];
        }
#pragma unroll
        for (int p = 0; p < CB * CB / 256; ++p) {
            const int e = tid + 256 * p, i = e % CB, j = e / CB;
            zd w = make_double2(i == j ? 1.0 : 0.0, 0.0);
            if (i < nb && j < nb && i >= j) {
                w.x = v[p].x;
                w.y = i == j ? 0.0 : v[p].y;
            }
            L[i * CP + j] = w;
        }
    }
    __syncthreads();
    // right-looking Cholesky, four columns at a time: wave 0 factors the 64 x 4 column panel in
    // registers (lane = row; the diagonal and the panel rows are broadcast with v_readlane), then
    // all threads apply the rank-4 update to the trailing lower triangle (lane = row i, the waves
    // take every fourth column j; the entries of row j are broadcast reads)
    const int lane = tid & 63, wave = tid >> 6;
    for (int k = 0; k < CB; k += 4) {
        if (tid < 64) {
            zd v[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = L[lane * CP + k + c];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int kc = k + c;
                const double d = readlane_d(v[c].x, kc);
                if (lane == 0 && !(d > 0.0) && kc < nb && info) atomicCAS(info, 0, col0 + kc + 1);
                const double inv = rsqrt_nr(d > 0.0 ? d : 1.0), sd = (d > 0.0 ? d : 1.0) * inv;
                if (lane > kc) v[c] = make_double2(v[c].x * inv, v[c].y * inv);
                else if (lane == kc) v[c] = make_double2(sd, 0.0);
#pragma unroll
                for (int j = c + 1; j < 4; ++j) {   // columns k + j of the panel, rows >= k + j
                    const zd l = make_double2(readlane_d(v[c].x, k + j), readlane_d(v[c].y, k + j));
                    if (lane >= k + j) v[j] = zsub_mul_conj(v[j], v[c], l);
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (lane >= k + c) L[lane * CP + k + c] = v[c];
        }
        __syncthreads();
        const int r0t = k + 4;
        if (lane >= r0t) {
            zd a[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) a[c] = L[lane * CP + k + c];
            // columns j = r0t + wave + 4 t, j <= lane, four at a time so that their LDS reads overlap
            for (int j0 = r0t + wave; j0 <= lane; j0 += 16) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = j0 + 4 * u;
                    if (j <= lane) {
                        zd acc = L[lane * CP + j];
#pragma unroll
                        for (int c = 0; c < 4; ++c) acc = zsub_mul_conj(acc, a[c], L[j * CP + k + c]);
                        L[lane * CP + j] = acc;
                    }
                }
            }
        }
        __syncthreads();
    }
    #pragma unroll
    for (int e = tid; e < CB * CB; e += 256) {
        const int i = e % CB, j = e / CB;
        if (i < nb && j < nb && i >= j) A[(size_t)i + (size_t)j * lda] = L[i * CP + j];
    }
    tri64::lower_inverse(L, X);
    #pragma unroll
    for (int e = tid; e < CB * CB; e += 256) {
        const int i = e % CB, j = e / CB;
        D[i + (size_t)j * CB] = X[i * CP + j];
    }
}

}  // namespace

namespace {

// recursive on halves (split at a multiple of 64) above 1024: L11 = chol(A11), L21 = A21 L11^{-H}
// (a triangular solve with the inverses just stored), A22 -= L21 L21^H (one GEMM with K = n / 2),
// L22 = chol(A22); up to 1024, right-looking over 64-column panels (fewer launches)
int chol_rec(hipStream_t s, int k0, int n, zd* A, int lda, int* info, zd* dinv, const GemmWs& gw)
{
    if (n <= 1024) {
        for (int j0 = 0; j0 < n; j0 += CB) {
            const int nb = std::min(CB, n - j0);
            zd* Ajj = A + j0 + (size_t)j0 * lda;
            zd* D = dinv + (size_t)(j0 / CB) * CB * CB;
            hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, nb, k0 + j0, Ajj, lda, info, D);
            int rc = (int)hipGetLastError();
            if (rc != 0) return rc;
            const int m2 = n - j0 - nb;
            if (m2 > 0) {
                zd* L21 = Ajj + nb;
                rc = tri_apply(s, TA_RIGHT_C, nb, m2, D, L21, lda);   // L21 = A21 L11^{-H}
                if (rc != 0) return rc;
                rc = launch_zgemm(s, OP_N, OP_C, m2, m2, nb, -1.0, L21, lda, L21, lda, 1.0, Ajj + nb + (size_t)nb * lda,
                                  lda, gw);
                if (rc != 0) return rc;
            }
        }
        return 0;
    }
    const int h = CB * (((n + CB - 1) / CB + 1) / 2);
    int rc = chol_rec(s, k0, h, A, lda, info, dinv, gw);
    if (rc != 0) return rc;
    zd* L21 = A + h;
    rc = trsm_right_lower_h(s, n - h, h, A, lda, dinv, L21, lda, gw);
    if (rc != 0) return rc;
    rc = gemm_lower_nc(s, n - h, h, L21, lda, L21, lda, A + h + (size_t)h * lda, lda, gw);   // lower triangle only
    if (rc != 0) return rc;
    return chol_rec(s, k0 + h, n - h, A + h + (size_t)h * lda, lda, info, dinv + (size_t)(h / CB) * CB * CB, gw);
}

}  // namespace

// L L^H = A (n x n, lower triangle of A read, L written in place).  *info (device, zeroed by the
// caller) receives the first non-positive pivot (1-based) or stays 0.  dinv (device,
// tri_dinv_elems(n) elements) receives the inverses of the 64 x 64 diagonal blocks of L, which the
// triangular solves with this L take.  gw: workspace of the GEMMs.  Returns hipError_t as int.
int chol_lower(hipStream_t s, int n, zd* A, int lda, int* info, zd* dinv, const GemmWs& gw)
{
    if (n <= 0) return 0;
    return chol_rec(s, 0, n, A, lda, info, dinv, gw);
}
