// Cholesky factorisation S = L L^H (lower) of the reduction to standard form (Section 3.2), blocked
// right-looking with 64-column panels:
//   k_chol_diag   one workgroup factors the 64 x 64 diagonal block (register resident), writes L11
//                 and stores L11^{-1} (tri64.h) for this factorisation and the later triangular
//                 solves;
//   L21           L21 = A21 L11^{-H}, in place, as an MFMA product with the stored inverse (trsm.hip);
//   trailing      A22 <- A22 - L21 L21^H with the MFMA complex GEMM of gemm.hip.
// A non-positive (or non-finite) pivot sets *info to its 1-based column, as LAPACK's potrf does;
// the factorisation then continues on meaningless numbers and the caller discards the result.
// Only the lower triangle of the input is read; the strict upper triangle of the result is left as
// the trailing updates made it (callers zero it).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "gemm_tile.h"
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

// acc - a conj(b) with fused multiply-adds
__device__ inline zd zfms_conj(zd acc, zd a, zd b)
{
    acc.x = __builtin_fma(-a.x, b.x, acc.x);
    acc.x = __builtin_fma(-a.y, b.y, acc.x);
    acc.y = __builtin_fma(-a.y, b.x, acc.y);
    acc.y = __builtin_fma(a.x, b.y, acc.y);
    return acc;
}

// Factors the nb x nb (nb <= 64) diagonal block at A (one workgroup), writes L11 to A and L11^{-1}
// (64 x 64, column-major, zero above the diagonal, identity beyond nb) to D.  col0: global index of
// the block's first column (for the pivot reported in *info).
//
// Right-looking over 16 panels of 4 columns.  Lane = row: wave w keeps its row's entries of the
// column blocks q = w, w + 4, w + 8, w + 12 in registers, so that only the panels pass through LDS.
//   * Panel s is factored by the wave that holds it (pivots and panel rows broadcast with
//     v_readlane); each pivot is formed from the previous one's reciprocal,
//     d_{c+1} = a_{c+1,c+1} - |u|^2 / d_c with u the unscaled entry below the previous pivot, so
//     that the column updates stay off the chain of pivots.
//   * The holder of block s + 1 applies panel s to that block and factors it at once (look-ahead)
//     and applies panel s to its other blocks one step later; the others apply panel s to their
//     later blocks.  Panels live in a ring of four LDS buffers, so one barrier per panel suffices.
//   * Entries above the diagonal are updated like the others (no branches) and never read.
// The inverse follows from the factor in LDS (tri64.h) with the pivots' reciprocals.
__global__ __launch_bounds__(256) void k_chol_diag(int nb, int col0, zd* __restrict__ A, int lda,
                                                   int* __restrict__ info, zd* __restrict__ D)
{
    __shared__ zd L[CB * CP];     // the factor, row-major (pitch CP), zero above the diagonal
    __shared__ zd X[CB * CP];     // L^{-1}
    __shared__ zd Pn[4][4][CB];   // panel ring: Pn[s & 3][c][row]
    __shared__ double Rv[CB];     // 1 / L_kk
    __shared__ int fail_min;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int fail = CB;                // first non-positive pivot met by this wave (wave-uniform)
    if (tid == 0) fail_min = CB;
    // lower triangle (the upper is never read), identity padding beyond nb; all 16 loads of a lane
    // (clamped into the block) are issued before any is used
    zd r[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = 4 * (wave + 4 * t) + c;
            r[t][c] = A[(size_t)min(lane, nb - 1) + (size_t)min(j, nb - 1) * lda];
        }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = 4 * (wave + 4 * t) + c;
            zd w = make_double2(lane == j ? 1.0 : 0.0, 0.0);
            if (lane < nb && j < nb && lane >= j) {
                w.x = r[t][c].x;
                w.y = lane == j ? 0.0 : r[t][c].y;
            }
            r[t][c] = w;
        }
    auto factor = [&](int s, zd (&b)[4]) {
        double d = readlane_d(b[0].x, 4 * s);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int kc = 4 * s + c;
            fail = (!(d > 0.0) && kc < nb) ? min(fail, kc) : fail;
            const double dd = d > 0.0 ? d : 1.0;
            double un = 0.0, a1 = 0.0;
            if (c < 3) {
                const double ux = readlane_d(b[c].x, kc + 1), uy = readlane_d(b[c].y, kc + 1);
                un = ux * ux + uy * uy;
                a1 = readlane_d(b[c + 1].x, kc + 1);
            }
            const double inv = rsqrt_nr(dd), sd = dd * inv;
            if (c < 3) d = __builtin_fma(-un, inv * inv, a1);
            Rv[kc] = inv;   // the same value from every lane
            const bool diag = lane == kc;
            b[c].x = diag ? sd : b[c].x * inv;
            b[c].y = diag ? 0.0 : b[c].y * inv;
#pragma unroll
            for (int j = c + 1; j < 4; ++j) {
                const zd l = make_double2(readlane_d(b[c].x, 4 * s + j), readlane_d(b[c].y, 4 * s + j));
                b[j] = zfms_conj(b[j], b[c], l);
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) Pn[s & 3][c][lane] = b[c];
    };
    // block q (held in b) -= (this row's entries of panel s) (block q's rows of panel s)^H
    auto update = [&](int s, zd (&b)[4], int q) {
        zd p[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) p[c] = Pn[s & 3][c][lane];
#pragma unroll
        for (int c2 = 0; c2 < 4; ++c2) {
            const int j = 4 * q + c2;
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c2] = zfms_conj(b[c2], p[c], Pn[s & 3][c][j]);
        }
    };
    if (wave == 0) factor(0, r[0]);
    __syncthreads();
#pragma clang loop unroll(full)
    for (int s = 0; s < 15; ++s) {
        const int nxt = s + 1;
        if (wave == (nxt & 3)) {
            update(s, r[nxt >> 2], nxt);
            factor(nxt, r[nxt >> 2]);
        } else {
            if (s >= 1 && wave == (s & 3)) {   // deferred: panel s - 1 on this wave's blocks after s
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (wave + 4 * t > s) update(s - 1, r[t], wave + 4 * t);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (wave + 4 * t > nxt) update(s, r[t], wave + 4 * t);
        }
        __syncthreads();
    }
    if (fail < CB && lane == 0) atomicMin(&fail_min, fail);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = 4 * (wave + 4 * t) + c;
            L[lane * CP + j] = lane >= j ? r[t][c] : make_double2(0.0, 0.0);
            if (lane < nb && j < nb && lane >= j) A[(size_t)lane + (size_t)j * lda] = r[t][c];
        }
    __syncthreads();
    if (tid == 0 && fail_min < CB && info) atomicCAS(info, 0, col0 + fail_min + 1);
    tri64::lower_inverse(L, Rv, X);
#pragma unroll
    for (int e = tid; e < CB * CB; e += 256) {
        const int i = e % CB, j = e / CB;
        D[i + (size_t)j * CB] = i >= j ? X[i * CP + j] : make_double2(0.0, 0.0);
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
