// Reduction of the Hermitian-definite pencil (A, S = L L^H) to standard form H = L^{-1} A L^{-H}
// (Section 3.2: the generalized problem is reduced with the Cholesky factor of the overlap before
// the iterative solver runs), using the Hermitian structure of A and H throughout: only lower
// triangles are updated, which takes n^3/2 complex multiply-adds where two triangular solves with
// n right-hand sides take n^3.
//
// With L = [L11 0; L21 L22] and A = [A11 A21^H; A21 A22] (L11 a 64 x 64 block), H = L^{-1} A L^{-H}
// splits as
//   H11 = L11^{-1} A11 L11^{-H}
//   Y   = A21 L11^{-H} - 1/2 L21 H11
//   A22 <- A22 - (Y L21^H + L21 Y^H)           (= A22 - L21 H11 L21^H - W L21^H - L21 W^H)
//   W   = Y - 1/2 L21 H11                      (= A21 L11^{-H} - L21 H11)
//   H21 = L22^{-1} W,   H22 = L22^{-1} A22 L22^{-H}  (the same reduction of the trailing pencil)
// (the ordering of LAPACK's blocked xHEGST).  Phase 1 runs the panels left to right, each a few
// small products with the stored inverse D11 = L11^{-1}.  The trailing update of a panel is split:
// the columns of the rest of its group of four panels (GW = 256 columns) are updated at once (a
// rectangular product with K = 128), the lower triangle beyond the group only once per group, with
// the Y blocks of its four panels: one product [Y L21] [L21 Y]^H with K = 512 on the tiles on or
// below the diagonal.  The panels of a group read nothing beyond it, so the delayed update gives
// the same H; it streams the trailing matrix once per 256 columns instead of once per 64, with
// products four times as deep.  The solves H21 = L22^{-1} W of all panels are deferred: the block-strictly-lower
// part of H is L^{-1} W with W the block-strictly-lower matrix of the panels' W (column block c of W
// is zero in block rows <= c, and L^{-1} keeps that), which phase 2 solves recursively on halves in
// products with a long inner dimension.  The diagonal blocks H11 of every panel are final after
// phase 1; a last pass mirrors the lower triangle into the upper one.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace {

constexpr int TB = 64;   // panel width = the diagonal blocks whose inverses the Cholesky factor stores
constexpr int GW = 4 * TB;   // panels per delayed trailing update

// work (ldw x 192) <- [Y | L21 | Y] for the rank-2k update of a panel (rows rows, 64 columns each)
__global__ void k_pack_her2k(int rows, int nb, const zd* __restrict__ Y, int ldy, const zd* __restrict__ L21, int ldl,
                             zd* __restrict__ work, int ldw)
{
    const size_t total = (size_t)rows * nb;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % rows), j = (int)(e / rows);
        const zd y = Y[(size_t)i + (size_t)j * ldy];
        work[(size_t)i + (size_t)j * ldw] = y;
        work[(size_t)i + (size_t)(nb + j) * ldw] = L21[(size_t)i + (size_t)j * ldl];
        work[(size_t)i + (size_t)(2 * nb + j) * ldw] = y;
    }
}

inline int split_point(int n) { return TB * (((n + TB - 1) / TB + 1) / 2); }

// X = L^{-1} W for the block-strictly-lower W (64-blocks) held in the block-strictly-lower part of
// B (n x n); the other blocks of B are neither read nor written
int solve_block_lower(hipStream_t s, int n, const zd* L, int ldl, const zd* dinv, zd* B, int ldb, const GemmWs& gw)
{
    if (n <= TB) return 0;
    const int h = split_point(n);
    int rc = solve_block_lower(s, h, L, ldl, dinv, B, ldb, gw);                   // X11
    if (rc != 0) return rc;
    // W21 -= L21 X11: column block c of X11 is nonzero in rows >= 64 (c + 1) only
    rc = launch_zgemm_tri(s, TRI_B_BLOCK_LOWER, OP_N, OP_N, n - h, h, h, -1.0, L + h, ldl, B, ldb, 1.0, B + h, ldb);
    if (rc != 0) return rc;
    const zd* L22 = L + h + (size_t)h * ldl;
    const zd* D22 = dinv + (size_t)(h / TB) * TB * TB;
    rc = trsm_left_lower(s, n - h, h, L22, ldl, D22, B + h, ldb, gw);               // X21 = L22^{-1} W21
    if (rc != 0) return rc;
    return solve_block_lower(s, n - h, L22, ldl, D22, B + h + (size_t)h * ldb, ldb, gw);   // X22
}

// X (n x n) <- [D_1 0 ...; 0 D_2 ...; ...]: the stored inverses of L's 64 x 64 diagonal blocks on the
// block diagonal (the last block may be smaller: its inverse sits in the leading part of a
// 64 x 64 slot), zero elsewhere
__global__ __launch_bounds__(256) void k_blockdiag_init(int n, const zd* __restrict__ dinv, zd* __restrict__ X, int ldx)
{
    const size_t total = (size_t)n * n;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        const int bi = i / TB, bj = j / TB;
        zd v = make_double2(0.0, 0.0);
        if (bi == bj) v = dinv[(size_t)bi * TB * TB + (i - bi * TB) + (size_t)(j - bj * TB) * TB];
        X[(size_t)i + (size_t)j * ldx] = v;
    }
}

// Strictly lower blocks of X = L^{-1} on halves, X holding the diagonal-block inverses and zero
// below them: X11 = L11^{-1}, X21 = -L22^{-1} (L21 X11), X22 = L22^{-1}.  (The product with X11
// includes its diagonal blocks, unlike the deferred solves of the reduction above.)
int tri_inverse_rec(hipStream_t s, int n, const zd* L, int ldl, const zd* dinv, zd* X, int ldx, const GemmWs& gw)
{
    if (n <= TB) return 0;
    const int h = split_point(n);
    int rc = tri_inverse_rec(s, h, L, ldl, dinv, X, ldx, gw);
    if (rc == 0) rc = launch_zgemm(s, OP_N, OP_N, n - h, h, h, -1.0, L + h, ldl, X, ldx, 0.0, X + h, ldx, gw);
    const zd* L22 = L + h + (size_t)h * ldl;
    const zd* D22 = dinv + (size_t)(h / TB) * TB * TB;
    if (rc == 0) rc = trsm_left_lower(s, n - h, h, L22, ldl, D22, X + h, ldx, gw);
    if (rc == 0) rc = tri_inverse_rec(s, n - h, L22, ldl, D22, X + h + (size_t)h * ldx, ldx, gw);
    return rc;
}

}  // namespace

// X (n x n, leading dimension ldx) <- L^{-1} for the lower-triangular L whose diagonal-block
// inverses are dinv (chol_lower): X starts as the block diagonal of the inverses, zero elsewhere,
// and a recursion on halves fills the strictly lower blocks.
int tri_inverse_lower(hipStream_t s, int n, const zd* L, int ldl, const zd* dinv, zd* X, int ldx, const GemmWs& gw)
{
    if (n <= 0) return 0;
    const size_t blocks = std::min<size_t>(((size_t)n * n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_blockdiag_init, dim3((unsigned)blocks), dim3(256), 0, s, n, dinv, X, ldx);
    const int rc = (int)hipGetLastError();
    if (rc != 0) return rc;
    return tri_inverse_rec(s, n, L, ldl, dinv, X, ldx, gw);
}

// H (n x n, leading dimension n) <- Linv A Linv^H with the explicit inverse Linv = L^{-1} (n x n,
// lower triangular) and A (n x n Hermitian, full storage): T = Linv A (row tile i of T takes the
// first i + 1 column tiles of Linv), the tiles of H on or below the diagonal as T Linv^H (tile
// (i, j) takes the first j + 1 column tiles of T), then the upper triangle mirrored (exactly
// Hermitian, real diagonal).  About 16 n^3 / 3 real flops in three launches, against the panel
// algorithm's 4 n^3 in a few hundred small ones.  T: n x n elements.
int hegst_explicit(hipStream_t s, int n, const zd* A, int lda, const zd* Linv, zd* T, zd* H)
{
    if (n <= 0) return 0;
    int rc = launch_zgemm_tri(s, TRI_A_LOWER, OP_N, OP_N, n, n, n, 1.0, Linv, n, A, lda, 0.0, T, n);
    if (rc == 0)
        rc = launch_zgemm_tri(s, TRI_C_LOWER | TRI_B_UPPER, OP_N, OP_C, n, n, n, 1.0, T, n, Linv, n, 0.0, H, n);
    if (rc == 0) rc = launch_mirror_lower(s, n, H, n);
    return rc;
}

// work: [Y | L21 | Y] of one panel (n x 3 TB), the Y blocks of a group below it (n x GW), and
// [Yg | Lg | Yg] of the group's delayed update (n x 3 GW)
size_t hegst_work_elems(int n) { return (size_t)n * (3 * TB + GW + 3 * GW); }

// A (n x n, lower triangle read, Hermitian) <- H = L^{-1} A L^{-H} in full (exactly Hermitian, real
// diagonal); L lower with the inverses of its 64 x 64 diagonal blocks in dinv (chol_lower); work:
// hegst_work_elems(n) elements.  Returns hipError_t as int.
int hegst_lower(hipStream_t s, int n, zd* A, int lda, const zd* L, int ldl, const zd* dinv, zd* work,
                const GemmWs& gw)
{
    if (n <= 0) return 0;
    int rc = 0;
    zd* pw = work;                           // [Y | L21 | Y] of the current panel, leading dimension n
    zd* yg = work + (size_t)n * 3 * TB;      // Y of the group's panels below the group (n x GW)
    zd* gwk = yg + (size_t)n * GW;           // [Yg | Lg | Yg] of the group update (n x 3 GW)
    for (int g0 = 0; g0 < n && rc == 0; g0 += GW) {
        const int gend = std::min(n, g0 + GW);   // columns of this group: [g0, gend)
        const int below = n - gend;               // rows beyond the group
        for (int k0 = g0; k0 < gend && rc == 0; k0 += TB) {
            const int nb = std::min(TB, n - k0), rest = n - k0 - nb;
            zd* A11 = A + k0 + (size_t)k0 * lda;
            const zd* D = dinv + (size_t)(k0 / TB) * TB * TB;
            // H11 = D A11 D^H from the lower triangle of A11 (the updates leave its upper part stale)
            if ((rc = launch_mirror_lower(s, nb, A11, lda)) != 0) break;
            if ((rc = tri_apply(s, TA_LEFT_N, nb, nb, D, A11, lda)) != 0) break;
            if ((rc = tri_apply(s, TA_RIGHT_C, nb, nb, D, A11, lda)) != 0) break;
            if (rest == 0) break;
            zd* A21 = A11 + nb;
            zd* A22 = A21 + (size_t)nb * lda;
            const zd* L21 = L + (k0 + nb) + (size_t)k0 * ldl;
            if ((rc = tri_apply(s, TA_RIGHT_C, nb, rest, D, A21, lda)) != 0) break;                 // A21 L11^{-H}
            if ((rc = launch_zgemm(s, OP_N, OP_N, rest, nb, nb, -0.5, L21, ldl, A11, lda, 1.0, A21, lda, gw)) != 0)
                break;                                                                               // Y
            const int cr = gend - (k0 + nb);   // columns of the group after this panel
            if (cr > 0) {
                hipLaunchKernelGGL(k_pack_her2k, dim3((unsigned)std::min<size_t>(((size_t)rest * nb + 255) / 256, 2048)),
                                   dim3(256), 0, s, rest, nb, A21, lda, L21, ldl, pw, n);
                if ((rc = (int)hipGetLastError()) != 0) break;
                // A22[:, group columns] -= [Y L21] [L21 Y]_(group rows)^H  (rows below the diagonal of
                // the group's block are not read by the later panels: written, never used)
                if ((rc = launch_zgemm(s, OP_N, OP_C, rest, cr, 2 * nb, -1.0, pw, n, pw + (size_t)nb * n, n, 1.0, A22,
                                       lda, gw)) != 0)
                    break;
            }
            if (below > 0) {   // this panel's Y below the group, for the group's delayed update
                if ((rc = launch_zlacpy(s, below, nb, A21 + cr, lda, yg + (size_t)(k0 - g0) * n, n)) != 0) break;
            }
            if ((rc = launch_zgemm(s, OP_N, OP_N, rest, nb, nb, -0.5, L21, ldl, A11, lda, 1.0, A21, lda, gw)) != 0)
                break;                                                                               // W
        }
        if (rc != 0 || below <= 0) continue;
        // delayed update of the lower triangle beyond the group: A_bb -= [Yg Lg] [Lg Yg]^H, K = 2 GW
        const int gwid = gend - g0;
        const zd* Lg = L + gend + (size_t)g0 * ldl;
        hipLaunchKernelGGL(k_pack_her2k, dim3((unsigned)std::min<size_t>(((size_t)below * gwid + 255) / 256, 4096)),
                           dim3(256), 0, s, below, gwid, yg, n, Lg, ldl, gwk, n);
        if ((rc = (int)hipGetLastError()) != 0) break;
        zd* Abb = A + gend + (size_t)gend * lda;
        rc = launch_zgemm_tri(s, TRI_C_LOWER, OP_N, OP_C, below, below, 2 * gwid, -1.0, gwk, n, gwk + (size_t)gwid * n,
                              n, 1.0, Abb, lda);
    }
    if (rc != 0) return rc;
    if ((rc = solve_block_lower(s, n, L, ldl, dinv, A, lda, gw)) != 0) return rc;              // H21 of every panel
    return launch_mirror_lower(s, n, A, lda);
}
