// Triangular solves with the Cholesky factor L (lower, n x n) of the reduction to standard form
// and of Cholesky QR: blocked substitution with 64 x 64 diagonal blocks whose inverses the
// factorisation stored (chol.hip), so that every step is a product on the MFMA tile of
// gemm_tile.h:
//   trsm_left_lower    L X = B          (H = L^{-1} A, first half of the reduction)
//   trsm_left_lower_h  L^H X = B        (X = L^{-H} V, back-transform of the eigenvectors)
//   trsm_right_lower_h X L^H = B        (H = W L^{-H}, second half; Q = Y R^{-1} of Cholesky QR)
// A large solve recurses on halves of the triangular dimension (solve one half, subtract its
// contribution from the other with one GEMM, solve the other half); up to 1024 it runs over the
// 64-blocks, each one in-place product with its stored inverse followed by one GEMM for the rest.
// Only the lower triangle of L is read.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "gemm_tile.h"

namespace {

constexpr int TB = 64;   // diagonal block size

// In-place product with the inverse D of one diagonal block (64 x 64, column-major, ld 64):
//   TA_LEFT_N  : B(0:nb, 0:nvec) <- D B        one workgroup per BN columns, BM = 64 covers all rows
//   TA_LEFT_C  : B(0:nb, 0:nvec) <- D^H B
//   TA_RIGHT_C : B(0:nvec, 0:nb) <- B D^H      one workgroup per BM rows, BN = 64 covers all columns
// Every workgroup reads only the rows / columns of B it writes, and writes them after its last
// read of them, so the product can overwrite its operand.
template <int MODE, int BM, int BN>
__global__ __launch_bounds__(256) void k_tri_apply(int nb, int nvec, const zd* __restrict__ D, zd* B, int ldb)
{
    typedef chfsi_tile::TileShape<double, BM, BN> S;
    __shared__ zd As[2 * S::AS_ELEMS];
    __shared__ zd Bs[2 * S::BS_ELEMS];
    d4 accr[S::MI][S::NJ], acci[S::MI][S::NJ];
    int i0 = 0, j0 = 0, M, N;
    if (MODE == TA_RIGHT_C) {
        i0 = blockIdx.x * BM;
        M = nvec;
        N = nb;
        chfsi_tile::tile_mainloop<double, OP_N, OP_C, BM, BN>(B, ldb, M, D, TB, N, i0, 0, 0, nb, As, Bs, accr, acci);
    } else {
        j0 = blockIdx.x * BN;
        M = nb;
        N = nvec;
        chfsi_tile::tile_mainloop<double, MODE == TA_LEFT_N ? OP_N : OP_C, OP_N, BM, BN>(D, TB, M, B, ldb, N, 0, j0, 0,
                                                                                        nb, As, Bs, accr, acci);
    }
#pragma unroll
    for (int bi = 0; bi < S::MI; ++bi)
#pragma unroll
        for (int bj = 0; bj < S::NJ; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = chfsi_tile::tile_row<double, BM, BN>(i0, bi);
                const int j = chfsi_tile::tile_col<double, BM, BN>(j0, bj, r);
                if (i < M && j < N) B[(size_t)i + (size_t)j * ldb] = make_double2(accr[bi][bj][r], acci[bi][bj][r]);
            }
}

}  // namespace

size_t tri_dinv_elems(int n) { return (size_t)((n + TB - 1) / TB) * TB * TB; }

int tri_apply(hipStream_t s, int mode, int nb, int nvec, const zd* D, zd* B, int ldb)
{
    if (nvec <= 0 || nb <= 0) return 0;
    if (nb > TB) return (int)hipErrorInvalidValue;
    if (mode == TA_RIGHT_C)
        hipLaunchKernelGGL((k_tri_apply<TA_RIGHT_C, 32, 64>), dim3((nvec + 31) / 32), dim3(256), 0, s, nb, nvec, D, B,
                           ldb);
    else if (mode == TA_LEFT_N)
        hipLaunchKernelGGL((k_tri_apply<TA_LEFT_N, 64, 32>), dim3((nvec + 31) / 32), dim3(256), 0, s, nb, nvec, D, B,
                           ldb);
    else if (mode == TA_LEFT_C)
        hipLaunchKernelGGL((k_tri_apply<TA_LEFT_C, 64, 32>), dim3((nvec + 31) / 32), dim3(256), 0, s, nb, nvec, D, B,
                           ldb);
    else
        return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

namespace {

// first index of the second half of [0, n): a multiple of TB, so that every sub-block starts on a
// stored diagonal block
inline int split_point(int n) { return TB * (((n + TB - 1) / TB + 1) / 2); }

// The solves recurse on halves of the triangular dimension down to REC_MIN, so that most of the
// work of a large solve is in a few GEMMs with a long inner dimension; below REC_MIN they run over
// the 64-blocks (one in-place product with the stored inverse, then one GEMM with K = 64 for the
// rest), which takes fewer launches.  L, dinv and B point at the sub-problem's origin.
constexpr int REC_MIN = 1024;

int loop_left(hipStream_t s, int n, int nrhs, const zd* L, int ldl, const zd* dinv, zd* B, int ldb, const GemmWs& gw)
{
    for (int k0 = 0; k0 < n; k0 += TB) {
        const int nb = std::min(TB, n - k0);
        int rc = tri_apply(s, TA_LEFT_N, nb, nrhs, dinv + (size_t)(k0 / TB) * TB * TB, B + k0, ldb);
        if (rc != 0) return rc;
        if (n - k0 - nb > 0) {   // B(k0+nb:, :) -= L(k0+nb:, k0:k0+nb) X(k0:k0+nb, :)
            rc = launch_zgemm(s, OP_N, OP_N, n - k0 - nb, nrhs, nb, -1.0, L + (size_t)(k0 + nb) + (size_t)k0 * ldl, ldl,
                              B + k0, ldb, 1.0, B + k0 + nb, ldb, gw);
            if (rc != 0) return rc;
        }
    }
    return 0;
}

int loop_left_h(hipStream_t s, int n, int nrhs, const zd* L, int ldl, const zd* dinv, zd* B, int ldb,
                const GemmWs& gw)
{
    for (int kb = (n + TB - 1) / TB - 1; kb >= 0; --kb) {
        const int k0 = kb * TB, nb = std::min(TB, n - k0);
        int rc = tri_apply(s, TA_LEFT_C, nb, nrhs, dinv + (size_t)kb * TB * TB, B + k0, ldb);
        if (rc != 0) return rc;
        if (k0 > 0) {   // B(0:k0, :) -= L(k0:k0+nb, 0:k0)^H X(k0:k0+nb, :)
            rc = launch_zgemm(s, OP_C, OP_N, k0, nrhs, nb, -1.0, L + k0, ldl, B + k0, ldb, 1.0, B, ldb, gw);
            if (rc != 0) return rc;
        }
    }
    return 0;
}

int loop_right_h(hipStream_t s, int nrow, int n, const zd* L, int ldl, const zd* dinv, zd* B, int ldb,
                 const GemmWs& gw)
{
    for (int k0 = 0; k0 < n; k0 += TB) {
        const int nb = std::min(TB, n - k0);
        int rc = tri_apply(s, TA_RIGHT_C, nb, nrow, dinv + (size_t)(k0 / TB) * TB * TB, B + (size_t)k0 * ldb, ldb);
        if (rc != 0) return rc;
        if (n - k0 - nb > 0) {   // B(:, k0+nb:) -= X(:, k0:k0+nb) L(k0+nb:, k0:k0+nb)^H
            rc = launch_zgemm(s, OP_N, OP_C, nrow, n - k0 - nb, nb, -1.0, B + (size_t)k0 * ldb, ldb,
                              L + (size_t)(k0 + nb) + (size_t)k0 * ldl, ldl, 1.0, B + (size_t)(k0 + nb) * ldb, ldb, gw);
            if (rc != 0) return rc;
        }
    }
    return 0;
}

int rec_left(hipStream_t s, int n, int nrhs, const zd* L, int ldl, const zd* dinv, zd* B, int ldb, const GemmWs& gw)
{
    if (n <= REC_MIN) return loop_left(s, n, nrhs, L, ldl, dinv, B, ldb, gw);
    const int h = split_point(n);
    int rc = rec_left(s, h, nrhs, L, ldl, dinv, B, ldb, gw);
    if (rc != 0) return rc;
    // B2 -= L21 X1
    rc = launch_zgemm(s, OP_N, OP_N, n - h, nrhs, h, -1.0, L + h, ldl, B, ldb, 1.0, B + h, ldb, gw);
    if (rc != 0) return rc;
    return rec_left(s, n - h, nrhs, L + h + (size_t)h * ldl, ldl, dinv + (size_t)(h / TB) * TB * TB, B + h, ldb, gw);
}

int rec_left_h(hipStream_t s, int n, int nrhs, const zd* L, int ldl, const zd* dinv, zd* B, int ldb, const GemmWs& gw)
{
    if (n <= REC_MIN) return loop_left_h(s, n, nrhs, L, ldl, dinv, B, ldb, gw);
    const int h = split_point(n);
    int rc = rec_left_h(s, n - h, nrhs, L + h + (size_t)h * ldl, ldl, dinv + (size_t)(h / TB) * TB * TB, B + h, ldb, gw);
    if (rc != 0) return rc;
    // B1 -= L21^H X2
    rc = launch_zgemm(s, OP_C, OP_N, h, nrhs, n - h, -1.0, L + h, ldl, B + h, ldb, 1.0, B, ldb, gw);
    if (rc != 0) return rc;
    return rec_left_h(s, h, nrhs, L, ldl, dinv, B, ldb, gw);
}

int rec_right_h(hipStream_t s, int nrow, int n, const zd* L, int ldl, const zd* dinv, zd* B, int ldb, const GemmWs& gw)
{
    if (n <= REC_MIN) return loop_right_h(s, nrow, n, L, ldl, dinv, B, ldb, gw);
    const int h = split_point(n);
    int rc = rec_right_h(s, nrow, h, L, ldl, dinv, B, ldb, gw);
    if (rc != 0) return rc;
    // B2 -= X1 L21^H
    rc = launch_zgemm(s, OP_N, OP_C, nrow, n - h, h, -1.0, B, ldb, L + h, ldl, 1.0, B + (size_t)h * ldb, ldb, gw);
    if (rc != 0) return rc;
    return rec_right_h(s, nrow, n - h, L + h + (size_t)h * ldl, ldl, dinv + (size_t)(h / TB) * TB * TB,
                       B + (size_t)h * ldb, ldb, gw);
}

// lower triangle of X with X L^H = B (B n x n), over the 64-blocks: column block k0 needs rows >= k0
// only, and the update of the later columns only the square below-right of it
int loop_right_h_lower(hipStream_t s, int n, const zd* L, int ldl, const zd* dinv, zd* B, int ldb, const GemmWs& gw)
{
    for (int k0 = 0; k0 < n; k0 += TB) {
        const int nb = std::min(TB, n - k0);
        int rc = tri_apply(s, TA_RIGHT_C, nb, n - k0, dinv + (size_t)(k0 / TB) * TB * TB, B + k0 + (size_t)k0 * ldb,
                           ldb);
        if (rc != 0) return rc;
        const int rest = n - k0 - nb;
        if (rest > 0) {   // B(k0+nb:, k0+nb:) -= X(k0+nb:, k0:k0+nb) L(k0+nb:, k0:k0+nb)^H
            rc = launch_zgemm(s, OP_N, OP_C, rest, rest, nb, -1.0, B + (k0 + nb) + (size_t)k0 * ldb, ldb,
                              L + (k0 + nb) + (size_t)k0 * ldl, ldl, 1.0, B + (k0 + nb) + (size_t)(k0 + nb) * ldb, ldb,
                              gw);
            if (rc != 0) return rc;
        }
    }
    return 0;
}

// [X11; X21] L11^H = [B11; B21] gives the lower part of X11 (recursively) and X21 in full; then
// B22 -= X21 L21^H on its lower triangle, and the lower part of X22 recursively
int rec_right_h_lower(hipStream_t s, int n, const zd* L, int ldl, const zd* dinv, zd* B, int ldb, const GemmWs& gw)
{
    if (n <= REC_MIN) return loop_right_h_lower(s, n, L, ldl, dinv, B, ldb, gw);
    const int h = split_point(n);
    int rc = rec_right_h_lower(s, h, L, ldl, dinv, B, ldb, gw);
    if (rc != 0) return rc;
    rc = rec_right_h(s, n - h, h, L, ldl, dinv, B + h, ldb, gw);
    if (rc != 0) return rc;
    rc = gemm_lower_nc(s, n - h, h, B + h, ldb, L + h, ldl, B + h + (size_t)h * ldb, ldb, gw);
    if (rc != 0) return rc;
    return rec_right_h_lower(s, n - h, L + h + (size_t)h * ldl, ldl, dinv + (size_t)(h / TB) * TB * TB,
                             B + h + (size_t)h * ldb, ldb, gw);
}

}  // namespace

// lower triangle of C (n x n) -= A B^H (A, B n x K): the diagonal blocks up to 512 as full GEMMs,
// larger ones split in halves (the strictly upper quarter is never computed)
int gemm_lower_nc(hipStream_t s, int n, int K, const zd* A, int lda, const zd* B, int ldb, zd* C, int ldc,
                  const GemmWs& gw)
{
    if (n <= 512) return launch_zgemm(s, OP_N, OP_C, n, n, K, -1.0, A, lda, B, ldb, 1.0, C, ldc, gw);
    const int h = split_point(n);
    int rc = gemm_lower_nc(s, h, K, A, lda, B, ldb, C, ldc, gw);
    if (rc != 0) return rc;
    rc = launch_zgemm(s, OP_N, OP_C, n - h, h, K, -1.0, A + h, lda, B, ldb, 1.0, C + h, ldc, gw);
    if (rc != 0) return rc;
    return gemm_lower_nc(s, n - h, K, A + h, lda, B + h, ldb, C + h + (size_t)h * ldc, ldc, gw);
}

// lower triangle of X with X L^H = B, B n x n (the strictly upper part of B is left meaningless)
int trsm_right_lower_h_lowertri(hipStream_t s, int n, const zd* L, int ldl, const zd* dinv, zd* B, int ldb,
                                const GemmWs& gw)
{
    if (n <= 0) return 0;
    return rec_right_h_lower(s, n, L, ldl, dinv, B, ldb, gw);
}

// L X = B, L n x n lower, B n x nrhs (overwritten by X).
int trsm_left_lower(hipStream_t s, int n, int nrhs, const zd* L, int ldl, const zd* dinv, zd* B, int ldb,
                    const GemmWs& gw)
{
    if (n <= 0 || nrhs <= 0) return 0;
    return rec_left(s, n, nrhs, L, ldl, dinv, B, ldb, gw);
}

// L^H X = B, L n x n lower, B n x nrhs (overwritten by X).
int trsm_left_lower_h(hipStream_t s, int n, int nrhs, const zd* L, int ldl, const zd* dinv, zd* B, int ldb,
                      const GemmWs& gw)
{
    if (n <= 0 || nrhs <= 0) return 0;
    return rec_left_h(s, n, nrhs, L, ldl, dinv, B, ldb, gw);
}

// X L^H = B, L ncol x ncol lower, B nrow x ncol (overwritten by X).
int trsm_right_lower_h(hipStream_t s, int nrow, int ncol, const zd* L, int ldl, const zd* dinv, zd* B, int ldb,
                       const GemmWs& gw)
{
    if (nrow <= 0 || ncol <= 0) return 0;
    return rec_right_h(s, nrow, ncol, L, ldl, dinv, B, ldb, gw);
}
