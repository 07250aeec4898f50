// Block LOBPCG without preconditioner (Knyazev 2001), the second solver of Section 3.1, on the
// library's kernels: the dense products of the filter (MFMA GEMM), the block Jacobi eigensolver of
// the Rayleigh-Ritz step, the residual and column kernels.  Table 2 compares iterating on the
// pencil (A, S) directly ("GEN") with iterating on the reduced problem H = L^{-1} A L^{-H} of
// Section 3.2 ("STD"); both are here (chfsi_lobpcg_params::gen).
//
// Each iteration performs Rayleigh-Ritz on the trial basis Z = [X | W | P]: the current Ritz block
// X (bs columns), the residuals W of its unconverged columns and the previous search directions P.
// The basis is made B-orthonormal block by block (W against X, P against X and W, each projection
// twice), so the projected problem Z^H A Z is a standard Hermitian one.  A block is
// orthonormalised through the eigen-decomposition of its B-Gram matrix after scaling its columns
// to unit B-norm, dropping directions whose Gram eigenvalue is below 1e-8 of the largest (with an
// ill-conditioned B the Gram rounding grows with kappa(B)).  The image A Z is updated with the same
// linear combinations as Z (one product with A per new residual column); B Z is formed again with B
// after every change of a block, since an updated B-image drifts from B Z when B is ill-conditioned
// and the Rayleigh-Ritz step relies on Z^H B Z = I.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "chfsi.h"
#include "common.h"
#include "driver.h"
#include "state.h"

namespace {

#define TRY(x)                                 \
    do {                                       \
        int rc_ = (int)(x);                    \
        if (rc_ != 0) return CHFSI_ERR_DEVICE; \
    } while (0)
#define TRYS(x)                                \
    do {                                       \
        chfsi_status s_ = (x);                 \
        if (s_ != CHFSI_SUCCESS) return s_;    \
    } while (0)

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// The iteration's operators and buffers.  Z, AZ, BZ: n x 3bs (BZ == Z when B = I); Tp: n x 3bs
// (the new directions and their A-images); Tx: n x bs; G: (3bs)^2; C: (3bs)^2.
struct Lob {
    chfsi_handle h;
    hipStream_t st;
    int n, bs;
    const zd* A;
    int lda;
    const zd* B;    // nullptr: B = I
    int ldb;
    zd *Z, *AZ, *BZ, *Tp, *Tx, *G, *C;
    double *theta, *res, *g, *dots;   // device [3bs]
    int* idx;                          // device [3bs]
    void* eigw;
    std::vector<double> ehost;
    GemmWs gw;
    long long matvecs = 0, bmatvecs = 0;
    int dropped = 0, restarts = 0;

    int gemm(int opa, int opb, int m, int ncol, int k, double al, const zd* X, int ldx, const zd* Y, int ldy, double be,
             zd* Cc, int ldc)
    {
        return launch_zgemm(st, opa, opb, m, ncol, k, al, X, ldx, Y, ldy, be, Cc, ldc, gw);
    }

    // out = A Y (k columns), with the filter's tuned plan for that shape
    chfsi_status apply_a(int k, const zd* Y, zd* out)
    {
        if (k <= 0) return CHFSI_SUCCESS;
        GemmWs g2 = gw;
        apply_tuned_plan(h, CHFSI_FP64, n, k, g2);
        TRY(launch_zgemm(st, OP_N, OP_N, n, k, n, 1.0, A, lda, Y, n, 0.0, out, n, g2));
        matvecs += k;
        return CHFSI_SUCCESS;
    }

    // out = B Y, or nothing when B = I (the caller's BY is Y itself)
    chfsi_status apply_b(int k, const zd* Y, zd* out)
    {
        if (k <= 0 || !B) return CHFSI_SUCCESS;
        GemmWs g2 = gw;
        apply_tuned_plan(h, CHFSI_FP64, n, k, g2);
        TRY(launch_zgemm(st, OP_N, OP_N, n, k, n, 1.0, B, ldb, Y, n, 0.0, out, n, g2));
        bmatvecs += k;
        return CHFSI_SUCCESS;
    }

    // (Y, AY) <- (Y, AY) - (Q, AQ) c with c = BQ^H Y (q x k, in C); BY = B Y formed again
    chfsi_status project_out(int q, const zd* Q, const zd* AQ, const zd* BQ, int k, zd* Y, zd* AY, zd* BY)
    {
        if (q <= 0 || k <= 0) return CHFSI_SUCCESS;
        TRY(gemm(OP_C, OP_N, q, k, n, 1.0, BQ, n, Y, n, 0.0, C, q));
        TRY(gemm(OP_N, OP_N, n, k, q, -1.0, Q, n, C, q, 1.0, Y, n));
        if (AY) TRY(gemm(OP_N, OP_N, n, k, q, -1.0, AQ, n, C, q, 1.0, AY, n));
        return apply_b(k, Y, BY);
    }

    // Makes the k columns of (Y, AY) B-orthonormal (AY may be null; BY == Y when B = I) and forms
    // BY = B Y again; *kept receives the number of columns kept, which are the leading ones.
    // CHFSI_ERR_NO_CONVERGENCE when the eigensolver of the Gram matrix does not converge.
    chfsi_status b_orthonormalize(int k, zd* Y, zd* AY, zd* BY, int* kept)
    {
        *kept = 0;
        if (k <= 0) return CHFSI_SUCCESS;
        TRY(launch_pair_dots(st, n, k, Y, n, BY, n, dots));
        TRY(launch_scale_cols_rsqrt(st, n, k, Y, n, dots));
        if (AY) TRY(launch_scale_cols_rsqrt(st, n, k, AY, n, dots));
        if (B) TRY(launch_scale_cols_rsqrt(st, n, k, BY, n, dots));
        TRY(gemm(OP_C, OP_N, k, k, n, 1.0, Y, n, BY, n, 0.0, G, k));
        // a Gram matrix within 1e-8 of the identity (the second pass, as a rule) takes the
        // first-order factor instead: Y <- Y (I - F), F = strict upper part of G + diag(G - I) / 2,
        // B-orthonormal to second order; the eigensolver is not asked to split a cluster of k
        // eigenvalues all equal to 1
        double off = 0;
        TRY(launch_max_rowsum_off_identity(st, k, G, k, dots));
        TRY(hipMemcpyAsync(&off, dots, sizeof(double), hipMemcpyDeviceToHost, st));
        TRY(hipStreamSynchronize(st));
        if (!std::isfinite(off)) return CHFSI_ERR_NUMERIC;
        if (off <= 1e-8) {
            TRY(launch_first_order_factor(st, k, G, k));
            zd* mats[2] = {Y, AY};
            for (zd* M : mats) {
                if (!M) continue;
                TRY(launch_zlacpy(st, n, k, M, n, Tx, n));
                TRY(gemm(OP_N, OP_N, n, k, k, -1.0, M, n, G, k, 1.0, Tx, n));
                TRY(launch_zlacpy(st, n, k, Tx, n, M, n));
            }
            *kept = k;
            return apply_b(k, Y, BY);
        }
        // the columns have unit B-norm, so the Gram matrix has a unit diagonal: an off-diagonal
        // level of 1e-12 resolves every direction kept (eigenvalue above 1e-8 of the largest)
        int sweeps = 0;
        const int rc = eig_jacobi(st, k, G, k, g, eigw, ehost.data(), &sweeps, 1e-12);
        if (rc == -1) return CHFSI_ERR_NO_CONVERGENCE;   // the caller decides (P: restart without it)
        TRY(rc);
        std::vector<double> gh(k);
        TRY(hipMemcpyAsync(gh.data(), g, sizeof(double) * k, hipMemcpyDeviceToHost, st));
        TRY(hipStreamSynchronize(st));
        if (!std::isfinite(gh[k - 1])) return CHFSI_ERR_NUMERIC;
        int kk = 0;
        for (int c = k - 1; c >= 0 && gh[c] > 1e-8 * gh[k - 1]; --c) ++kk;
        dropped += k - kk;
        *kept = kk;
        if (kk == 0) return CHFSI_SUCCESS;
        TRY(launch_orth_factor(st, k, kk, G, k, g, C, k));
        zd* mats[2] = {Y, AY};
        for (zd* M : mats) {
            if (!M) continue;
            TRY(gemm(OP_N, OP_N, n, kk, k, 1.0, M, n, C, k, 0.0, Tx, n));
            TRY(launch_zlacpy(st, n, kk, Tx, n, M, n));
        }
        return apply_b(kk, Y, BY);
    }

    zd* bz(zd* z) const { return B ? BZ + (z - Z) : z; }

    // Rayleigh-Ritz of the leading k columns of Z: theta (device) <- the eigenvalues of Z^H A Z,
    // G <- its eigenvectors (k x k, ascending)
    chfsi_status rayleigh_ritz(int k)
    {
        TRY(gemm(OP_C, OP_N, k, k, n, 1.0, Z, n, AZ, n, 0.0, G, k));
        int sweeps = 0;
        const int rc = eig_jacobi(st, k, G, k, theta, eigw, ehost.data(), &sweeps);
        if (rc == -1) return CHFSI_ERR_NUMERIC;
        TRY(rc);
        return CHFSI_SUCCESS;
    }

    // X <- Z V(:, 0:bs) and A X alike (V = G, leading dimension k); B X formed again
    chfsi_status update_x(int k)
    {
        zd* mats[2] = {Z, AZ};
        for (zd* M : mats) {
            TRY(gemm(OP_N, OP_N, n, bs, k, 1.0, M, n, G, k, 0.0, Tx, n));
            TRY(launch_zlacpy(st, n, bs, Tx, n, M, n));
        }
        return apply_b(bs, Z, BZ);
    }
};

// The iteration on the operators of `L` from the block X (n x bs, already in Z).  thr: residual
// threshold on ||A x - theta B x||.  On return Z holds the Ritz vectors, theta_h / res_h the Ritz
// values and residual norms of the last check.  Returns SUCCESS, NO_CONVERGENCE or an error.
chfsi_status lobpcg_core(Lob& L, int nev, double thr, int maxiter, std::vector<double>& theta_h,
                         std::vector<double>& res_h, int* iters, int* nconv_out)
{
    const int n = L.n, bs = L.bs;
    const size_t nb = (size_t)n * bs;
    hipStream_t st = L.st;
    int kept = 0;
    // X B-orthonormal (two passes), then A X, then Rayleigh-Ritz on X alone
    TRYS(L.apply_b(bs, L.Z, L.BZ));
    for (int pass = 0; pass < 2; ++pass) {
        const chfsi_status s = L.b_orthonormalize(bs, L.Z, nullptr, L.bz(L.Z), &kept);
        if (s == CHFSI_ERR_NO_CONVERGENCE || (s == CHFSI_SUCCESS && kept < bs)) return CHFSI_ERR_NUMERIC;
        TRYS(s);
    }
    TRYS(L.apply_a(bs, L.Z, L.AZ));
    TRYS(L.rayleigh_ritz(bs));
    TRYS(L.update_x(bs));
    int np = 0;
    std::vector<int> act(bs);
    *iters = 0;
    *nconv_out = 0;
    for (int it = 1; it <= maxiter; ++it) {
        *iters = it;
        // residual norms of the block (theta: the first bs Ritz values of the last step)
        TRY(launch_residual_norms(st, n, bs, L.AZ, n, L.bz(L.Z), n, L.theta, L.res));
        TRY(hipMemcpyAsync(theta_h.data(), L.theta, sizeof(double) * bs, hipMemcpyDeviceToHost, st));
        TRY(hipMemcpyAsync(res_h.data(), L.res, sizeof(double) * bs, hipMemcpyDeviceToHost, st));
        TRY(hipStreamSynchronize(st));
        int na = 0, nconv = 0;
        bool prefix = true;
        for (int j = 0; j < bs; ++j) {
            if (!std::isfinite(res_h[j]) || !std::isfinite(theta_h[j])) return CHFSI_ERR_NUMERIC;
            if (res_h[j] <= thr) {
                if (prefix) ++nconv;
            } else {
                prefix = false;
                act[na++] = j;
            }
        }
        *nconv_out = nconv;
        if (nconv >= nev) return CHFSI_SUCCESS;
        const int nact = na;
        TRY(hipMemcpyAsync(L.idx, act.data(), sizeof(int) * nact, hipMemcpyHostToDevice, st));
        // W: the residuals of the active columns, B-orthogonal to X (twice), B-orthonormal
        zd* W = L.Z + nb;
        zd* AW = L.AZ + nb;
        TRY(launch_residual_gather(st, n, na, L.AZ, n, L.bz(L.Z), n, L.theta, L.idx, W, n));
        TRYS(L.apply_b(na, W, L.bz(W)));
        for (int pass = 0; pass < 2 && na > 0; ++pass) {
            TRYS(L.project_out(bs, L.Z, nullptr, L.bz(L.Z), na, W, nullptr, L.bz(W)));
            const chfsi_status s = L.b_orthonormalize(na, W, nullptr, L.bz(W), &na);
            if (s == CHFSI_ERR_NO_CONVERGENCE) return CHFSI_ERR_NUMERIC;
            TRYS(s);
        }
        TRYS(L.apply_a(na, W, AW));
        // P (the previous directions, kept in Tp) right after W, off X and W, B-orthonormal
        zd* P = W + (size_t)n * na;
        zd* AP = AW + (size_t)n * na;
        if (np > 0) {
            TRY(launch_zlacpy(st, n, np, L.Tp, n, P, n));
            TRY(launch_zlacpy(st, n, np, L.Tp + nb, n, AP, n));
            TRYS(L.apply_b(np, P, L.bz(P)));
            for (int pass = 0; pass < 2 && np > 0; ++pass) {
                TRYS(L.project_out(bs, L.Z, L.AZ, L.bz(L.Z), np, P, AP, L.bz(P)));
                TRYS(L.project_out(na, W, AW, L.bz(W), np, P, AP, L.bz(P)));
                const chfsi_status s = L.b_orthonormalize(np, P, AP, L.bz(P), &np);
                if (s == CHFSI_ERR_NO_CONVERGENCE) {   // restart: this step without the directions
                    np = 0;
                    ++L.restarts;
                    break;
                }
                TRYS(s);
            }
        }
        const int k = bs + na + np;
        TRYS(L.rayleigh_ritz(k));
        // new directions P = [W P] V(bs:k, act) and their A-images, before X is replaced
        const int nwp = na + np;
        if (nwp > 0 && nact > 0) {
            TRY(launch_permute_cols(st, nwp, nact, L.G + bs, k, L.C, nwp, L.idx));
            zd* mats[2] = {L.Z, L.AZ};
            for (int t = 0; t < 2; ++t)
                TRY(L.gemm(OP_N, OP_N, n, nact, nwp, 1.0, mats[t] + nb, n, L.C, nwp, 0.0, L.Tp + t * nb, n));
            np = nact;
        } else {
            np = 0;
        }
        TRYS(L.update_x(k));
    }
    return CHFSI_ERR_NO_CONVERGENCE;
}

}  // namespace

extern "C" void chfsi_lobpcg_default_params(chfsi_lobpcg_params* p)
{
    if (!p) return;
    p->nev = 32;
    p->bs = 0;
    p->maxiter = 1000;
    p->tol = 1e-10;
    p->gen = 0;
    p->seed = 0;
}

extern "C" chfsi_status chfsi_lobpcg(chfsi_handle h, int n, const void* Av, int lda, const void* Sv, int lds, void* Xv,
                                     int ldx, int x_is_guess, double* lambda, double* resid,
                                     const chfsi_lobpcg_params* p, chfsi_lobpcg_stats* stats)
{
    if (!h || !Av || !Xv || !lambda || !resid || !p || n <= 0 || lda < n || ldx < n || (Sv && lds < n)) return CHFSI_ERR_ARG;
    const int bs = p->bs > 0 ? p->bs : (int)std::ceil(1.05 * p->nev);
    if (p->nev <= 0 || bs < p->nev || bs > n || p->maxiter < 0 || !(p->tol > 0)) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    const double t0 = now_ms();
    chfsi_lobpcg_stats stt;
    std::memset(&stt, 0, sizeof(stt));
    const zd* A = (const zd*)Av;
    const zd* S = (const zd*)Sv;
    zd* X = (zd*)Xv;
    const bool reduce = S && !p->gen;
    const int m3 = 3 * bs;
    SolveBufs b;
    TRYS(prepare_bufs(h, h->ws, b, n, m3, 1, reduce, CHFSI_FP64, reduce));
    hipStream_t st = h->stream;
    // the blocks beyond the solver workspace
    const size_t nb = (size_t)n * bs;
    Arena& ar = h->lob;
    auto carve = [&](zd** tp, zd** tx) {
        *tp = ar.take<zd>(3 * nb);
        *tx = ar.take<zd>(nb);
    };
    zd *Tp = nullptr, *Tx = nullptr;
    ar.begin(true);
    carve(&Tp, &Tx);
    if (ar.off > ar.cap) {
        (void)hipStreamSynchronize(st);
        ar.grow(ar.off);
        if (ar.cap < ar.off) return CHFSI_ERR_ALLOC;
    }
    ar.begin(false);
    carve(&Tp, &Tx);

    // norms for the thresholds: ||A||_lo (largest column norm) and ||S||_inf
    double norms[2] = {0, 1};
    TRY(launch_max_colnorm(st, n, A, lda, b.dsc));
    TRY(hipMemcpyAsync(&norms[0], b.dsc, sizeof(double), hipMemcpyDeviceToHost, st));
    if (S) {
        TRY(launch_max_rowsum_abs(st, n, S, lds, b.dsc + n + 8));
        TRY(hipMemcpyAsync(&norms[1], b.dsc + n + 8, sizeof(double), hipMemcpyDeviceToHost, st));
    }
    TRY(hipStreamSynchronize(st));
    if (!std::isfinite(norms[0]) || !std::isfinite(norms[1]) || !(norms[0] > 0)) return CHFSI_ERR_NUMERIC;

    Lob L;
    L.h = h;
    L.st = st;
    L.n = n;
    L.bs = bs;
    L.Z = b.V;
    L.AZ = b.T;
    L.BZ = b.HY;
    L.Tp = Tp;
    L.Tx = Tx;
    L.G = b.G;
    L.C = b.Cm;
    L.theta = b.theta;
    L.res = b.r;
    L.g = b.lam;
    L.dots = b.E;
    L.idx = b.iperm;
    L.eigw = b.eigw;
    L.ehost.resize(eig_host_doubles(m3));
    L.gw = b.gw;
    double thr;
    const double tr0 = now_ms();
    if (reduce) {
        TRYS(step_reduce(h, n, A, lda, S, lds, b.H, b.L, b.dinvL, b.hwork, b.info, b.gw));
        L.A = b.H;
        L.lda = n;
        L.B = nullptr;
        thr = p->tol * norms[0] / std::sqrt(norms[1]);
    } else {
        L.A = A;
        L.lda = lda;
        L.B = S;
        L.ldb = lds;
        thr = p->tol * norms[0];
    }
    stt.t_reduce = now_ms() - tr0;
    // the start block in the iteration's coordinates: Y0 = L^H X0 on the reduced problem
    if (!x_is_guess) TRY(launch_philox_block(st, p->seed, 1, n, bs, L.Z, n));
    else if (reduce) TRY(launch_zgemm(st, OP_C, OP_N, n, bs, n, 1.0, b.L, n, X, ldx, 0.0, L.Z, n, b.gw));
    else TRY(launch_zlacpy(st, n, bs, X, ldx, L.Z, n));
    std::vector<double> th(bs), rs(bs);
    const double ti0 = now_ms();
    int iters = 0, nconv = 0;
    chfsi_status status = lobpcg_core(L, p->nev, thr, p->maxiter, th, rs, &iters, &nconv);
    stt.t_iterate = now_ms() - ti0;
    stt.iters = iters;
    stt.nconv = nconv;
    stt.matvecs = L.matvecs;
    stt.bmatvecs = L.bmatvecs;
    stt.dropped = L.dropped;
    stt.restarts = L.restarts;
    if (status != CHFSI_SUCCESS && status != CHFSI_ERR_NO_CONVERGENCE) {
        stt.t_total = now_ms() - t0;
        if (stats) *stats = stt;
        return status;
    }
    // back to generalized coordinates, unit S-norm columns from fresh products, verification:
    // resid = ||A x - lambda S x|| / ||A||_lo
    TRY(launch_zlacpy(st, n, bs, L.Z, n, X, ldx));
    if (reduce) TRY(trsm_left_lower_h(st, n, bs, b.L, n, b.dinvL, X, ldx, b.gw));
    zd* SX = Tx;
    if (S) TRY(launch_zgemm(st, OP_N, OP_N, n, bs, n, 1.0, S, lds, X, ldx, 0.0, SX, n, b.gw));
    else TRY(launch_zlacpy(st, n, bs, X, ldx, SX, n));
    TRY(launch_pair_dots(st, n, bs, X, ldx, SX, n, L.dots));
    TRY(launch_scale_cols_rsqrt(st, n, bs, X, ldx, L.dots));
    TRY(launch_scale_cols_rsqrt(st, n, bs, SX, n, L.dots));
    zd* AX = L.AZ;
    TRY(launch_zgemm(st, OP_N, OP_N, n, bs, n, 1.0, A, lda, X, ldx, 0.0, AX, n, b.gw));
    TRY(hipMemcpyAsync(L.theta, th.data(), sizeof(double) * bs, hipMemcpyHostToDevice, st));
    TRY(launch_residual_norms(st, n, bs, AX, n, SX, n, L.theta, L.res));
    TRY(hipMemcpyAsync(rs.data(), L.res, sizeof(double) * bs, hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    for (int j = 0; j < bs; ++j) {
        lambda[j] = th[j];
        resid[j] = rs[j] / norms[0];
    }
    stt.t_total = now_ms() - t0;
    if (stats) *stats = stt;
    return status;
}
