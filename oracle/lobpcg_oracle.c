/*
 * CPU reference ("oracle") for block LOBPCG without preconditioner (Knyazev 2001), the second
 * solver of Section 3.1 of Di Napoli & Berljafa, applied to a Hermitian pencil either directly
 * ("GEN": A x = lambda S x) or after the reduction to standard form of Section 3.2 ("STD":
 * H y = lambda y, the comparison of Table 2).
 *
 * TEST INFRASTRUCTURE ONLY, like chfsi_oracle.c (whose Cholesky, triangular solves, reduction,
 * dense product, Jacobi eigensolver and random block it uses).  FP64, plain loops.
 *
 * The method, as the paper describes it: each iteration performs the Rayleigh-Ritz procedure for
 * the pencil on the trial subspace spanned by the current block X of Ritz vectors, the residuals W
 * of the vectors that have not converged, and the block P of the previous search directions (the
 * part of the last update that did not come from X), keeping the bs lowest Ritz pairs.
 * Readings where the paper is silent:
 *  - the trial basis is made B-orthonormal block by block before the Rayleigh-Ritz step (W against
 *    X, then P against X and W, each projection done twice), so the projected problem is a
 *    standard Hermitian one; a block is orthonormalised through the eigen-decomposition of its
 *    B-Gram matrix after scaling its columns to unit B-norm, and directions whose Gram eigenvalue
 *    is below 1e-8 of the largest are dropped (a nearly dependent residual or direction: with an
 *    ill-conditioned B the rounding of the Gram matrix grows with kappa(B), and the direction of a
 *    smaller eigenvalue would come out of the scaling far from B-orthonormal);
 *  - A-images are updated with the same linear combinations as the blocks (one product with A per
 *    new residual), B-images are formed again with B after every change of a block: with an
 *    ill-conditioned B an updated image drifts from B Y, the basis stops being B-orthonormal and
 *    the Rayleigh-Ritz step returns spurious Ritz values;
 *  - soft locking: a column whose residual meets the threshold leaves W and P but stays in X;
 *  - the iteration stops when the nev lowest Ritz pairs (a leading prefix) all meet the threshold,
 *    or after maxiter iterations;
 *  - the threshold is the one of the ChFSI oracle: ||A x - lambda S x|| <= tol ||A||_lo (GEN) and
 *    ||H y - lambda y|| <= tol ||A||_lo / sqrt(||S||_inf) (STD), with ||A||_lo the largest column
 *    norm of A; every returned pair is verified on the pencil afterwards;
 *  - block size bs = ceil(1.05 nev) (Table 3), random start from the Philox block of stream 1.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zc;
#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* from chfsi_oracle.c */
void orc_zgemm(char ta, char tb, int m, int n, int k, zc alpha, const zc* A, int lda, const zc* B, int ldb,
               zc beta, zc* C, int ldc);
int orc_cholesky(int n, const zc* S, int lds, zc* L, int ldl);
void orc_trsm_lower_h(int n, int nrhs, const zc* L, int ldl, zc* B, int ldb);
void orc_reduce(int n, const zc* A, int lda, const zc* L, int ldl, zc* H, int ldh);
int orc_jacobi(int m, const zc* Gin, int ldg, double* w, zc* V, int ldv);
void orc_random_block(uint64_t seed, uint64_t stream, int n, int m, zc* Y, int ldy);

typedef struct {
    int nev, bs, maxiter, gen;
    double tol;
    uint64_t seed;
} orc_lobpcg_params;

typedef struct {
    int iters, nconv;
    long long matvecs;     /* columns multiplied by the operator A (or H) */
    long long bmatvecs;    /* columns multiplied by S (GEN only) */
    int dropped;           /* basis directions dropped as dependent */
} orc_lobpcg_stats;

/* The operator pair of the iteration: op(X) = Aop X and, when Bop != NULL, B X. */
typedef struct {
    int n;
    const zc* Aop;
    int lda;
    const zc* Bop;   /* NULL: B = I */
    int ldb;
} pencil_t;

static void apply(const pencil_t* P, const zc* M, int ld, int nrhs, const zc* X, int ldx, zc* Y, int ldy)
{
    orc_zgemm('N', 'N', P->n, nrhs, P->n, 1.0, M, ld, X, ldx, 0.0, Y, ldy);
}

/* BY = B Y (or a copy of Y when B = I) */
static void apply_b(const pencil_t* P, int k, const zc* Y, zc* BY, long long* bmv)
{
    if (P->Bop) {
        apply(P, P->Bop, P->ldb, k, Y, P->n, BY, P->n);
        *bmv += k;
    } else {
        memcpy(BY, Y, sizeof(zc) * (size_t)P->n * k);
    }
}

/* Y <- Y - Q (BQ^H Y): the B-projection of Y off span(Q), applied alike to A Y; B Y is formed
 * again from the new Y (an image updated by the same combination drifts from B Y when B is
 * ill-conditioned, and the Rayleigh-Ritz step relies on Z^H B Z = I). */
static void project_out(const pencil_t* P, int q, const zc* Q, const zc* AQ, const zc* BQ, int k, zc* Y, zc* AY,
                        zc* BY, long long* bmv)
{
    const int n = P->n;
    if (q == 0 || k == 0) return;
    zc* c = (zc*)malloc(sizeof(zc) * (size_t)q * k);
    orc_zgemm('C', 'N', q, k, n, 1.0, BQ, n, Y, n, 0.0, c, q);
    orc_zgemm('N', 'N', n, k, q, -1.0, Q, n, c, q, 1.0, Y, n);
    if (AY) orc_zgemm('N', 'N', n, k, q, -1.0, AQ, n, c, q, 1.0, AY, n);
    apply_b(P, k, Y, BY, bmv);
    free(c);
}

/* Makes the k columns of (Y, AY, BY) B-orthonormal: columns scaled to unit B-norm, then
 * Y <- Y U diag(g)^{-1/2} over the eigenpairs (g, U) of the B-Gram matrix Y^H B Y whose g exceeds
 * 1e-8 max(g), and BY = B Y again.  Returns the number of columns kept (the leading ones). */
static int b_orthonormalize(const pencil_t* P, int k, zc* Y, zc* AY, zc* BY, int* dropped, long long* bmv)
{
    const int n = P->n;
    if (k == 0) return 0;
    for (int j = 0; j < k; ++j) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += creal(conj(Y[IDX(i, j, n)]) * BY[IDX(i, j, n)]);
        const double d = s > 0 ? 1.0 / sqrt(s) : 0.0;
        for (int i = 0; i < n; ++i) {
            Y[IDX(i, j, n)] *= d;
            if (AY) AY[IDX(i, j, n)] *= d;
            BY[IDX(i, j, n)] *= d;
        }
    }
    zc* G = (zc*)malloc(sizeof(zc) * (size_t)k * k);
    zc* U = (zc*)malloc(sizeof(zc) * (size_t)k * k);
    double* g = (double*)malloc(sizeof(double) * (size_t)k);
    orc_zgemm('C', 'N', k, k, n, 1.0, Y, n, BY, n, 0.0, G, k);
    orc_jacobi(k, G, k, g, U, k);
    const double gmax = g[k - 1];
    int kept = 0;
    /* keep the largest eigenvalues; T = U(:, keep) diag(g)^{-1/2}, in descending order of g */
    zc* T = (zc*)calloc((size_t)k * k, sizeof(zc));
    for (int c = k - 1; c >= 0; --c) {
        if (!(g[c] > 1e-8 * gmax)) break;
        const double s = 1.0 / sqrt(g[c]);
        for (int i = 0; i < k; ++i) T[IDX(i, kept, k)] = U[IDX(i, c, k)] * s;
        ++kept;
    }
    *dropped += k - kept;
    zc* tmp = (zc*)malloc(sizeof(zc) * (size_t)n * (kept > 0 ? kept : 1));
    zc* mats[2] = {Y, AY};
    for (int t = 0; t < 2; ++t) {
        if (!mats[t] || kept == 0) continue;
        orc_zgemm('N', 'N', n, kept, k, 1.0, mats[t], n, T, k, 0.0, tmp, n);
        memcpy(mats[t], tmp, sizeof(zc) * (size_t)n * kept);
    }
    apply_b(P, kept, Y, BY, bmv);   /* B Y of the new block, formed again */
    free(G); free(U); free(g); free(T); free(tmp);
    return kept;
}

/* The iteration itself on the pencil P, block X (n x bs, overwritten by the Ritz vectors),
 * threshold thr on ||A x - theta B x||.  theta[bs], res[bs] receive the Ritz values and residual
 * norms of the last iteration.  Returns 0 (converged), 3 (maxiter), 4 (breakdown). */
static int lobpcg_core(const pencil_t* P, int bs, int nev, double thr, int maxiter, zc* X, int ldx, double* theta,
                       double* res, orc_lobpcg_stats* st)
{
    const int n = P->n;
    const size_t nb = (size_t)n * bs;
    /* Z = [X | W | P] and its images under A and B, each n x 3 bs */
    zc* Z = (zc*)calloc(3 * nb, sizeof(zc));
    zc* AZ = (zc*)calloc(3 * nb, sizeof(zc));
    zc* BZ = (zc*)calloc(3 * nb, sizeof(zc));
    zc* T = (zc*)malloc(sizeof(zc) * 3 * nb);
    zc* G = (zc*)malloc(sizeof(zc) * 9 * (size_t)bs * bs);
    zc* V = (zc*)malloc(sizeof(zc) * 9 * (size_t)bs * bs);
    zc* C = (zc*)malloc(sizeof(zc) * 9 * (size_t)bs * bs);
    double* w = (double*)malloc(sizeof(double) * 3 * (size_t)bs);
    int* act = (int*)malloc(sizeof(int) * (size_t)bs);
    int status = 3, np = 0;

    for (int j = 0; j < bs; ++j) memcpy(Z + IDX(0, j, n), X + IDX(0, j, ldx), sizeof(zc) * n);
    /* X B-orthonormal (two passes), then A X */
    for (int pass = 0; pass < 2; ++pass) {
        apply_b(P, bs, Z, BZ, &st->bmatvecs);
        if (b_orthonormalize(P, bs, Z, NULL, BZ, &st->dropped, &st->bmatvecs) < bs) { status = 4; goto done; }
    }
    apply(P, P->Aop, P->lda, bs, Z, n, AZ, n);
    st->matvecs += bs;
    /* first Rayleigh-Ritz on X alone */
    orc_zgemm('C', 'N', bs, bs, n, 1.0, Z, n, AZ, n, 0.0, G, bs);
    orc_jacobi(bs, G, bs, w, V, bs);
    {
        zc* mats[2] = {Z, AZ};
        for (int t = 0; t < 2; ++t) {
            orc_zgemm('N', 'N', n, bs, bs, 1.0, mats[t], n, V, bs, 0.0, T, n);
            memcpy(mats[t], T, sizeof(zc) * nb);
        }
        apply_b(P, bs, Z, BZ, &st->bmatvecs);
    }
    for (int j = 0; j < bs; ++j) theta[j] = w[j];

    for (int it = 1; it <= maxiter; ++it) {
        st->iters = it;
        /* residuals R = A X - B X diag(theta), written into the W slot */
        zc* W = Z + nb;
        zc* AW = AZ + nb;
        zc* BW = BZ + nb;
        int na = 0, nconv = 0, prefix = 1;
        for (int j = 0; j < bs; ++j) {
            double s = 0;
            for (int i = 0; i < n; ++i) {
                const zc r = AZ[IDX(i, j, n)] - theta[j] * BZ[IDX(i, j, n)];
                s += creal(r) * creal(r) + cimag(r) * cimag(r);
            }
            res[j] = sqrt(s);
            if (res[j] <= thr) {
                if (prefix) ++nconv;
            } else {
                prefix = 0;
                act[na++] = j;
            }
        }
        st->nconv = nconv;
        if (nconv >= nev) { status = 0; goto done; }
        for (int c = 0; c < na; ++c) {
            const int j = act[c];
            for (int i = 0; i < n; ++i) W[IDX(i, c, n)] = AZ[IDX(i, j, n)] - theta[j] * BZ[IDX(i, j, n)];
        }
        /* W: B-orthogonal to X (twice), B-orthonormal; then its images */
        apply_b(P, na, W, BW, &st->bmatvecs);
        for (int pass = 0; pass < 2; ++pass) {
            project_out(P, bs, Z, NULL, BZ, na, W, NULL, BW, &st->bmatvecs);
            na = b_orthonormalize(P, na, W, NULL, BW, &st->dropped, &st->bmatvecs);
        }
        apply(P, P->Aop, P->lda, na, W, n, AW, n);
        st->matvecs += na;
        /* P (kept in the third slot, its images updated alike): off X and W, B-orthonormal */
        zc* Pp = Z + 2 * nb;
        zc* AP = AZ + 2 * nb;
        zc* BP = BZ + 2 * nb;
        if (np > 0) {
            for (int pass = 0; pass < 2; ++pass) {
                project_out(P, bs, Z, AZ, BZ, np, Pp, AP, BP, &st->bmatvecs);
                project_out(P, na, W, AW, BW, np, Pp, AP, BP, &st->bmatvecs);
                np = b_orthonormalize(P, np, Pp, AP, BP, &st->dropped, &st->bmatvecs);
            }
        }
        /* compact basis [X | W(:, 0:na) | P(:, 0:np)]: move P right after W */
        const int k = bs + na + np;
        if (np > 0 && na < bs) {
            memmove(Z + IDX(0, bs + na, n), Pp, sizeof(zc) * (size_t)n * np);
            memmove(AZ + IDX(0, bs + na, n), AP, sizeof(zc) * (size_t)n * np);
            memmove(BZ + IDX(0, bs + na, n), BP, sizeof(zc) * (size_t)n * np);
        }
        /* Rayleigh-Ritz on the trial subspace: G = Z^H A Z, the bs lowest eigenpairs */
        orc_zgemm('C', 'N', k, k, n, 1.0, Z, n, AZ, n, 0.0, G, k);
        orc_jacobi(k, G, k, w, V, k);
        for (int j = 0; j < bs; ++j) theta[j] = w[j];
        /* new directions P = [W P] C(bs:k, act) for the columns that were active in this iteration
         * (computed before X is overwritten), new X = Z C(:, 0:bs) */
        int nact = 0;
        for (int j = 0; j < bs; ++j)
            if (res[j] > thr) act[nact++] = j;
        if (na + np > 0) {
            for (int c = 0; c < nact; ++c)
                for (int i = 0; i < na + np; ++i) C[IDX(i, c, na + np)] = V[IDX(bs + i, act[c], k)];
            zc* mats[2] = {Z, AZ};
            for (int t = 0; t < 2; ++t)
                orc_zgemm('N', 'N', n, nact, na + np, 1.0, mats[t] + IDX(0, bs, n), n, C, na + np, 0.0,
                          T + IDX(0, t * bs, n), n);
        }
        {
            zc* mats[2] = {Z, AZ};
            zc* Xn = (zc*)malloc(sizeof(zc) * nb);
            for (int t = 0; t < 2; ++t) {
                orc_zgemm('N', 'N', n, bs, k, 1.0, mats[t], n, V, k, 0.0, Xn, n);
                memcpy(mats[t], Xn, sizeof(zc) * nb);
            }
            free(Xn);
            apply_b(P, bs, Z, BZ, &st->bmatvecs);
        }
        np = (na + np > 0) ? nact : 0;
        for (int t = 0; t < 2 && np > 0; ++t) {
            zc* dst = (t == 0 ? Z : AZ) + 2 * nb;
            memcpy(dst, T + IDX(0, t * bs, n), sizeof(zc) * (size_t)n * np);
        }
        if (np > 0) apply_b(P, np, Z + 2 * nb, BZ + 2 * nb, &st->bmatvecs);
    }
done:
    for (int j = 0; j < bs; ++j) memcpy(X + IDX(0, j, ldx), Z + IDX(0, j, n), sizeof(zc) * n);
    free(Z); free(AZ); free(BZ); free(T); free(G); free(V); free(C); free(w); free(act);
    return status;
}

static double max_colnorm(int n, const zc* A, int lda)
{
    double best = 0;
    for (int j = 0; j < n; ++j) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += creal(A[IDX(i, j, lda)]) * creal(A[IDX(i, j, lda)]) +
                                         cimag(A[IDX(i, j, lda)]) * cimag(A[IDX(i, j, lda)]);
        if (s > best) best = s;
    }
    return sqrt(best);
}

static double inf_norm(int n, const zc* S, int lds)
{
    double best = 0;
    for (int j = 0; j < n; ++j) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += cabs(S[IDX(i, j, lds)]);
        if (s > best) best = s;
    }
    return best;
}

/* LOBPCG for A x = lambda S x (S = NULL: standard).  X (n x bs): in = start block if x_is_guess,
 * out = Ritz vectors (S-orthonormal), ascending; lambda[bs], resid[bs] (||A x - lambda S x|| /
 * ||A||_lo of the returned vectors).  p->gen = 1 iterates on the pencil, 0 on H = L^{-1} A L^{-H}.
 * Returns 0 (converged), 2 (S not HPD), 3 (maxiter), 4 (breakdown). */
int orc_lobpcg(int n, const zc* A, int lda, const zc* S, int lds, zc* X, int ldx, int x_is_guess, double* lambda,
               double* resid, const orc_lobpcg_params* p, orc_lobpcg_stats* st)
{
    memset(st, 0, sizeof(*st));
    const int bs = p->bs;
    if (bs <= 0 || bs > n || p->nev <= 0 || p->nev > bs) return 1;
    const double norm_a = max_colnorm(n, A, lda);
    if (!x_is_guess) orc_random_block(p->seed, 1, n, bs, X, ldx);
    int status;
    zc* L = NULL;
    zc* H = NULL;
    if (S && !p->gen) {
        /* STD: reduce, iterate on H with Y0 = L^H X0, back-transform */
        L = (zc*)malloc(sizeof(zc) * (size_t)n * n);
        if (orc_cholesky(n, S, lds, L, n)) { free(L); return 2; }
        H = (zc*)malloc(sizeof(zc) * (size_t)n * n);
        orc_reduce(n, A, lda, L, n, H, n);
        if (x_is_guess) {   /* Y0 = L^H X0 */
            zc* Y = (zc*)malloc(sizeof(zc) * (size_t)n * bs);
            orc_zgemm('C', 'N', n, bs, n, 1.0, L, n, X, ldx, 0.0, Y, n);
            for (int j = 0; j < bs; ++j) memcpy(X + IDX(0, j, ldx), Y + IDX(0, j, n), sizeof(zc) * n);
            free(Y);
        }
        pencil_t P = {n, H, n, NULL, 0};
        const double thr = p->tol * norm_a / sqrt(inf_norm(n, S, lds));
        status = lobpcg_core(&P, bs, p->nev, thr, p->maxiter, X, ldx, lambda, resid, st);
        orc_trsm_lower_h(n, bs, L, n, X, ldx);
    } else {
        pencil_t P = {n, A, lda, S, lds};
        status = lobpcg_core(&P, bs, p->nev, p->tol * norm_a, p->maxiter, X, ldx, lambda, resid, st);
    }
    /* the implicitly updated images drift from S X over many iterations: scale each returned
     * vector to unit S-norm with a fresh product, then verify on the pencil:
     * resid = ||A x - lambda S x|| / ||A||_lo */
    zc* AX = (zc*)malloc(sizeof(zc) * (size_t)n * bs);
    zc* SX = (zc*)malloc(sizeof(zc) * (size_t)n * bs);
    if (S) orc_zgemm('N', 'N', n, bs, n, 1.0, S, lds, X, ldx, 0.0, SX, n);
    for (int j = 0; j < bs; ++j) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += creal(conj(X[IDX(i, j, ldx)]) * (S ? SX[IDX(i, j, n)] : X[IDX(i, j, ldx)]));
        const double d = s > 0 ? 1.0 / sqrt(s) : 1.0;
        for (int i = 0; i < n; ++i) {
            X[IDX(i, j, ldx)] *= d;
            if (S) SX[IDX(i, j, n)] *= d;
        }
    }
    orc_zgemm('N', 'N', n, bs, n, 1.0, A, lda, X, ldx, 0.0, AX, n);
    for (int j = 0; j < bs; ++j) {
        double s = 0;
        for (int i = 0; i < n; ++i) {
            const zc sx = S ? SX[IDX(i, j, n)] : X[IDX(i, j, ldx)];
            const zc r = AX[IDX(i, j, n)] - lambda[j] * sx;
            s += creal(r) * creal(r) + cimag(r) * cimag(r);
        }
        resid[j] = sqrt(s) / norm_a;
    }
    free(AX); free(SX); free(L); free(H);
    return status;
}
