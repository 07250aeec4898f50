/*
 * CPU reference ("oracle") for Chebyshev-filtered subspace iteration with locking
 * (Di Napoli & Berljafa, "Block iterative eigensolvers for sequences of correlated eigenvalue
 * problems", Section 3.1, Algorithm 1).
 *
 * TEST INFRASTRUCTURE ONLY.  It is called by the tests, by the smoke check and by the benchmark's
 * CPU-baseline leg, never by the product path.  It is plain, slow and meant to be checked by eye
 * against the paper: FP64 throughout, column-major complex double (C99 `double complex`), no
 * blocking or fusion beyond what each definition states.  It shares no source with the GPU library.
 *
 * Where the paper is silent, the readings used here are:
 *  - the filter is the scaled three-term Chebyshev recurrence on [a, b] normalised at mu1
 *    (the paper names a degree-deg Chebyshev filter without printing it);
 *  - Cholesky / reduction use L^H where the paper writes L^T (complex data; it uses the dagger in
 *    the Rayleigh quotient of Algorithm 1);
 *  - the loop repeats *while* fewer than nev pairs are locked, and "converged" counts locked pairs;
 *  - re-orthonormalisation is classical Gram-Schmidt twice against the locked vectors followed by
 *    Householder QR with a real non-negative diagonal of R;
 *  - the reduced problem is solved by cyclic Jacobi; eigenvalues ascending, each eigenvector's
 *    largest-magnitude entry made real positive;
 *  - Lanczos runs k steps with full reorthogonalisation from a counter-based random unit vector;
 *    b = theta_max + beta_k, mu1 = theta_min, and on a cold start a is the smallest Ritz value whose
 *    cumulative weight |z_1j|^2 reaches m/n;
 *  - a pair is locked when ||H y - theta y|| <= tol * ||A||_lo / sqrt(||S||_inf), which makes the
 *    final check ||A x - lambda S x|| / ||A||_lo <= tol hold, with ||A||_lo the largest column norm
 *    of A (a lower bound of ||A||_2);
 *  - random vectors (cold start block, Lanczos start) come from Philox4x64-10 (Salmon et al., SC'11)
 *    with uniform real and imaginary parts in [-1, 1).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef double complex zc;

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* ------------------------------------------------------------------------------------------------
 * Optional library primitives.  The dense product, the triangular solve and the Cholesky factor
 * below are written out as plain loops; a caller may route them to library routines of the same
 * definition instead (BLAS/LAPACK on the host), which the order-8192 problems need: the plain loops
 * stream the whole matrix once per column.  Every step of the method above these primitives stays
 * as written here.  NULL (the default) selects the plain loops.
 * ---------------------------------------------------------------------------------------------- */
typedef void (*orc_gemm_hook)(char ta, char tb, int m, int n, int k, double alpha_re, double alpha_im,
                              const zc* A, int lda, const zc* B, int ldb, double beta_re, double beta_im,
                              zc* C, int ldc);
typedef void (*orc_trsm_hook)(int conj_trans, int n, int nrhs, const zc* L, int ldl, zc* B, int ldb);
typedef int (*orc_chol_hook)(int n, const zc* S, int lds, zc* L, int ldl);
static orc_gemm_hook g_gemm_hook = 0;
static orc_trsm_hook g_trsm_hook = 0;
static orc_chol_hook g_chol_hook = 0;

void orc_set_library_hooks(orc_gemm_hook g, orc_trsm_hook t, orc_chol_hook c)
{
    g_gemm_hook = g;
    g_trsm_hook = t;
    g_chol_hook = c;
}

/* ------------------------------------------------------------------------------------------------
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11):
 * ten rounds of two 64x64->128-bit multiplies with the published multipliers and Weyl key bumps.
 * ---------------------------------------------------------------------------------------------- */
void orc_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static double u53(uint64_t v) { return (double)(v >> 11) * 0x1.0p-53; }

/* Element e of random stream `stream`: counter (e/2, stream, 0, 0), key (seed, 0); the four words
 * give two complex numbers, element parity picks one; parts are uniform in [-1, 1). */
zc orc_random_element(uint64_t seed, uint64_t stream, uint64_t e)
{
    uint64_t ctr[4] = {e >> 1, stream, 0, 0}, key[2] = {seed, 0}, o[4];
    orc_philox4x64(ctr, key, o);
    int w = (int)(e & 1) * 2;
    return (2.0 * u53(o[w]) - 1.0) + I * (2.0 * u53(o[w + 1]) - 1.0);
}

void orc_random_block(uint64_t seed, uint64_t stream, int n, int m, zc* Y, int ldy)
{
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < n; ++i)
            Y[IDX(i, j, ldy)] = orc_random_element(seed, stream, (uint64_t)i + (uint64_t)j * (uint64_t)n);
}

/* ------------------------------------------------------------------------------------------------
 * Dense products.  C = alpha op(A) op(B) + beta C, op = identity ('N') or conjugate transpose ('C').
 * op(A) is m x k, op(B) is k x n.  beta == 0 ignores C's previous contents.
 * ---------------------------------------------------------------------------------------------- */
static inline zc opB(char tb, const zc* B, int ldb, int p, int j)
{
    return tb == 'N' ? B[IDX(p, j, ldb)] : conj(B[IDX(j, p, ldb)]);
}

void orc_zgemm(char ta, char tb, int m, int n, int k, zc alpha, const zc* A, int lda,
               const zc* B, int ldb, zc beta, zc* C, int ldc)
{
    if (g_gemm_hook) {
        if (m > 0 && n > 0)
            g_gemm_hook(ta, tb, m, n, k, creal(alpha), cimag(alpha), A, lda, B, ldb, creal(beta), cimag(beta), C, ldc);
        return;
    }
    const int RB = 256;
    const int nrb = (m + RB - 1) / RB;
    #pragma omp parallel for collapse(2) schedule(dynamic)
    for (int j = 0; j < n; ++j) {
        for (int rb = 0; rb < nrb; ++rb) {
            int i0 = rb * RB, i1 = i0 + RB < m ? i0 + RB : m;
            zc acc[256];
            for (int i = i0; i < i1; ++i) acc[i - i0] = 0;
            if (ta == 'N') {
                for (int p = 0; p < k; ++p) {
                    zc bpj = opB(tb, B, ldb, p, j);
                    const zc* ap = A + IDX(0, p, lda);
                    for (int i = i0; i < i1; ++i) acc[i - i0] += ap[i] * bpj;
                }
            } else {
                for (int i = i0; i < i1; ++i) {
                    const zc* ai = A + IDX(0, i, lda);
                    zc s = 0;
                    for (int p = 0; p < k; ++p) s += conj(ai[p]) * opB(tb, B, ldb, p, j);
                    acc[i - i0] = s;
                }
            }
            for (int i = i0; i < i1; ++i) {
                zc v = alpha * acc[i - i0];
                C[IDX(i, j, ldc)] = (beta == 0) ? v : v + beta * C[IDX(i, j, ldc)];
            }
        }
    }
}

static double znrm2(int n, const zc* x)
{
    double s = 0;
    for (int i = 0; i < n; ++i) s += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
    return sqrt(s);
}

/* ------------------------------------------------------------------------------------------------
 * Cholesky S = L L^H (Section 3.2, reduction to standard form), column by column.
 * L is lower triangular with a real positive diagonal; its strict upper part is set to zero.
 * Returns 0, or 1 when a pivot is not positive (S not positive definite).
 * ---------------------------------------------------------------------------------------------- */
int orc_cholesky(int n, const zc* S, int lds, zc* L, int ldl)
{
    if (g_chol_hook) return g_chol_hook(n, S, lds, L, ldl);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) L[IDX(i, j, ldl)] = 0;
    zc* v = (zc*)malloc(sizeof(zc) * (size_t)n);
    int status = 0;
    for (int j = 0; j < n && !status; ++j) {
        /* v = S(j:n, j) - L(j:n, 0:j) L(j, 0:j)^H */
        #pragma omp parallel for schedule(static)
        for (int i = j; i < n; ++i) v[i] = S[IDX(i, j, lds)];
        const int CH = 512;
        #pragma omp parallel for schedule(static)
        for (int i0 = j; i0 < n; i0 += CH) {
            int i1 = i0 + CH < n ? i0 + CH : n;
            for (int p = 0; p < j; ++p) {
                zc ljp = conj(L[IDX(j, p, ldl)]);
                const zc* lp = L + IDX(0, p, ldl);
                for (int i = i0; i < i1; ++i) v[i] -= lp[i] * ljp;
            }
        }
        double d = creal(v[j]);
        if (!(d > 0.0) || !isfinite(d)) { status = 1; break; }
        double ljj = sqrt(d);
        L[IDX(j, j, ldl)] = ljj;
        for (int i = j + 1; i < n; ++i) L[IDX(i, j, ldl)] = v[i] / ljj;
    }
    free(v);
    return status;
}

/* Solve L X = B in place (L lower triangular, B n x nrhs), forward substitution per column. */
void orc_trsm_lower(int n, int nrhs, const zc* L, int ldl, zc* B, int ldb)
{
    if (g_trsm_hook) { g_trsm_hook(0, n, nrhs, L, ldl, B, ldb); return; }
    #pragma omp parallel for schedule(dynamic)
    for (int j = 0; j < nrhs; ++j) {
        zc* x = B + IDX(0, j, ldb);
        for (int p = 0; p < n; ++p) {
            x[p] /= L[IDX(p, p, ldl)];
            zc xp = x[p];
            const zc* lp = L + IDX(0, p, ldl);
            for (int i = p + 1; i < n; ++i) x[i] -= lp[i] * xp;
        }
    }
}

/* Solve L^H X = B in place, back substitution per column. */
void orc_trsm_lower_h(int n, int nrhs, const zc* L, int ldl, zc* B, int ldb)
{
    if (g_trsm_hook) { g_trsm_hook(1, n, nrhs, L, ldl, B, ldb); return; }
    #pragma omp parallel for schedule(dynamic)
    for (int j = 0; j < nrhs; ++j) {
        zc* x = B + IDX(0, j, ldb);
        for (int p = n - 1; p >= 0; --p) {
            const zc* lp = L + IDX(0, p, ldl);
            zc s = x[p];
            for (int q = p + 1; q < n; ++q) s -= conj(lp[q]) * x[q];
            x[p] = s / conj(lp[p]);
        }
    }
}

/* H = L^{-1} A L^{-H}, then H <- (H + H^H)/2 (Section 3.2).  W = L^{-1} A; H = L^{-1} W^H. */
void orc_reduce(int n, const zc* A, int lda, const zc* L, int ldl, zc* H, int ldh)
{
    zc* W = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) W[IDX(i, j, n)] = A[IDX(i, j, lda)];
    orc_trsm_lower(n, n, L, ldl, W, n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) H[IDX(i, j, ldh)] = conj(W[IDX(j, i, n)]);
    orc_trsm_lower(n, n, L, ldl, H, ldh);
    for (int j = 0; j < n; ++j)
        for (int i = j; i < n; ++i) {
            zc v = 0.5 * (H[IDX(i, j, ldh)] + conj(H[IDX(j, i, ldh)]));
            H[IDX(i, j, ldh)] = v;
            H[IDX(j, i, ldh)] = conj(v);
        }
    free(W);
}

/* ------------------------------------------------------------------------------------------------
 * Householder QR of Y (n x m, n >= m): Y <- Q, R (m x m) upper triangular with real non-negative
 * diagonal.  Returns 1 if a column is exactly dependent on the previous ones (R_jj == 0).
 * ---------------------------------------------------------------------------------------------- */
int orc_qr(int n, int m, zc* Y, int ldy, zc* R, int ldr)
{
    zc* W = (zc*)malloc(sizeof(zc) * (size_t)n * m);
    zc* V = (zc*)calloc((size_t)n * m, sizeof(zc));   /* reflector j lives in V(j:n, j) */
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < n; ++i) W[IDX(i, j, n)] = Y[IDX(i, j, ldy)];
    int status = 0;
    for (int j = 0; j < m; ++j) {
        zc* x = W + IDX(j, j, n);
        int len = n - j;
        double xn = znrm2(len, x);
        if (xn == 0.0) { status = 1; continue; }
        zc ph = cabs(x[0]) > 0 ? x[0] / cabs(x[0]) : 1.0;
        zc beta = -ph * xn;
        zc* v = V + IDX(j, j, n);
        for (int i = 0; i < len; ++i) v[i] = x[i];
        v[0] -= beta;
        double vn = znrm2(len, v);
        for (int i = 0; i < len; ++i) v[i] /= vn;
        /* W(j:n, j:m) <- (I - 2 v v^H) W(j:n, j:m) */
        #pragma omp parallel for schedule(static)
        for (int c = j; c < m; ++c) {
            zc* w = W + IDX(j, c, n);
            zc s = 0;
            for (int i = 0; i < len; ++i) s += conj(v[i]) * w[i];
            for (int i = 0; i < len; ++i) w[i] -= 2.0 * v[i] * s;
        }
    }
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) R[IDX(i, j, ldr)] = i <= j ? W[IDX(i, j, n)] : 0;
    /* Q = H_0 H_1 ... H_{m-1} [I; 0]: apply the reflectors in reverse order */
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < n; ++i) Y[IDX(i, j, ldy)] = (i == j) ? 1.0 : 0.0;
    for (int j = m - 1; j >= 0; --j) {
        const zc* v = V + IDX(j, j, n);
        int len = n - j;
        #pragma omp parallel for schedule(static)
        for (int c = 0; c < m; ++c) {
            zc* q = Y + IDX(j, c, ldy);
            zc s = 0;
            for (int i = 0; i < len; ++i) s += conj(v[i]) * q[i];
            for (int i = 0; i < len; ++i) q[i] -= 2.0 * v[i] * s;
        }
    }
    /* make R's diagonal real non-negative: R(j,:) *= conj(ph_j), Q(:,j) *= ph_j */
    for (int j = 0; j < m; ++j) {
        zc d = R[IDX(j, j, ldr)];
        double ad = cabs(d);
        if (ad == 0.0) continue;
        zc ph = d / ad;
        for (int c = j; c < m; ++c) R[IDX(j, c, ldr)] *= conj(ph);
        R[IDX(j, j, ldr)] = ad;
        for (int i = 0; i < n; ++i) Y[IDX(i, j, ldy)] *= ph;
    }
    free(W);
    free(V);
    return status;
}

/* ------------------------------------------------------------------------------------------------
 * Cyclic Jacobi for a Hermitian matrix G (m x m): G = V diag(w) V^H.
 * Each rotation zeroes G(p,q): the phase of G(p,q) is removed with diag(1, e^{-i phi}) and the real
 * symmetric 2x2 remainder is diagonalised by the classical rotation with t = tan(angle) the smaller
 * root of t^2 + 2 theta t - 1 = 0, theta = (G_qq - G_pp) / (2 |G_pq|).
 * Sweeps repeat until no off-diagonal entry exceeds 1e-16 ||G||_F.  Eigenvalues are returned in
 * ascending order (ties keep index order); each eigenvector's largest-magnitude entry (first on
 * ties) is made real positive.
 * ---------------------------------------------------------------------------------------------- */
int orc_jacobi(int m, const zc* Gin, int ldg, double* w, zc* V, int ldv)
{
    zc* G = (zc*)malloc(sizeof(zc) * (size_t)m * m);
    double fro = 0;
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
            zc g = 0.5 * (Gin[IDX(i, j, ldg)] + conj(Gin[IDX(j, i, ldg)]));
            G[IDX(i, j, m)] = g;
            fro += creal(g) * creal(g) + cimag(g) * cimag(g);
        }
    fro = sqrt(fro);
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) V[IDX(i, j, ldv)] = (i == j) ? 1.0 : 0.0;
    const double thr = 1e-16 * fro;
    int sweeps = 0;
    for (; sweeps < 100; ++sweeps) {
        int rotated = 0;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                zc g = G[IDX(p, q, m)];
                double ag = cabs(g);
                if (!(ag > thr)) continue;
                double a = creal(G[IDX(p, p, m)]), b = creal(G[IDX(q, q, m)]);
                double theta = (b - a) / (2.0 * ag);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                zc e = conj(g) / ag;                       /* e^{-i phi} */
                /* columns: [G_p, G_q] <- [G_p, G_q] J,  J = [[c, s], [-s e, c e]] */
                for (int i = 0; i < m; ++i) {
                    zc gp = G[IDX(i, p, m)], gq = G[IDX(i, q, m)];
                    G[IDX(i, p, m)] = c * gp - s * e * gq;
                    G[IDX(i, q, m)] = s * gp + c * e * gq;
                    zc vp = V[IDX(i, p, ldv)], vq = V[IDX(i, q, ldv)];
                    V[IDX(i, p, ldv)] = c * vp - s * e * vq;
                    V[IDX(i, q, ldv)] = s * vp + c * e * vq;
                }
                /* rows: [G_p; G_q] <- J^H [G_p; G_q] */
                for (int k = 0; k < m; ++k) {
                    zc gp = G[IDX(p, k, m)], gq = G[IDX(q, k, m)];
                    G[IDX(p, k, m)] = c * gp - s * conj(e) * gq;
                    G[IDX(q, k, m)] = s * gp + c * conj(e) * gq;
                }
                G[IDX(p, q, m)] = 0;
                G[IDX(q, p, m)] = 0;
                G[IDX(p, p, m)] = a - t * ag;
                G[IDX(q, q, m)] = b + t * ag;
                rotated = 1;
            }
        if (!rotated) break;
    }
    /* ascending order, stable on ties (insertion sort on (value, index)) */
    int* ord = (int*)malloc(sizeof(int) * (size_t)m);
    double* d = (double*)malloc(sizeof(double) * (size_t)m);
    for (int i = 0; i < m; ++i) { ord[i] = i; d[i] = creal(G[IDX(i, i, m)]); }
    for (int i = 1; i < m; ++i) {
        int o = ord[i], j = i - 1;
        while (j >= 0 && d[ord[j]] > d[o]) { ord[j + 1] = ord[j]; --j; }
        ord[j + 1] = o;
    }
    zc* Vs = (zc*)malloc(sizeof(zc) * (size_t)m * m);
    for (int j = 0; j < m; ++j) {
        w[j] = d[ord[j]];
        for (int i = 0; i < m; ++i) Vs[IDX(i, j, m)] = V[IDX(i, ord[j], ldv)];
    }
    for (int j = 0; j < m; ++j) {
        int imax = 0;
        double vmax = -1;
        for (int i = 0; i < m; ++i) {
            double av = cabs(Vs[IDX(i, j, m)]);
            if (av > vmax) { vmax = av; imax = i; }
        }
        zc ph = vmax > 0 ? Vs[IDX(imax, j, m)] / vmax : 1.0;
        for (int i = 0; i < m; ++i) V[IDX(i, j, ldv)] = Vs[IDX(i, j, m)] * conj(ph);
        V[IDX(imax, j, ldv)] = vmax;
    }
    free(Vs); free(d); free(ord); free(G);
    return sweeps;
}

/* ------------------------------------------------------------------------------------------------
 * Lanczos with full reorthogonalisation (Algorithm 1, spectral upper bound): k steps from the
 * Philox unit vector of stream 2.  Returns the Ritz values of T_k (ascending), the squared first
 * components |z_1j|^2 of its eigenvectors, beta_k, and the number of steps actually taken (fewer
 * if an invariant subspace is found).
 * ---------------------------------------------------------------------------------------------- */
int orc_lanczos(int n, const zc* H, int ldh, int k, uint64_t seed, double* theta, double* zw,
                double* beta_k)
{
    zc* V = (zc*)malloc(sizeof(zc) * (size_t)n * (k + 1));
    zc* w = (zc*)malloc(sizeof(zc) * (size_t)n);
    zc* cc = (zc*)malloc(sizeof(zc) * (size_t)(k + 1));
    double* al = (double*)calloc((size_t)k + 1, sizeof(double));
    double* be = (double*)calloc((size_t)k + 1, sizeof(double));
    for (int i = 0; i < n; ++i) V[i] = orc_random_element(seed, 2, (uint64_t)i);
    double vn = znrm2(n, V);
    for (int i = 0; i < n; ++i) V[i] /= vn;
    int kk = 0;
    for (int j = 0; j < k; ++j) {
        zc* vj = V + IDX(0, j, n);
        orc_zgemm('N', 'N', n, 1, n, 1.0, H, ldh, vj, n, 0.0, w, n);
        zc s = 0;
        for (int i = 0; i < n; ++i) s += conj(vj[i]) * w[i];
        al[j] = creal(s);
        for (int i = 0; i < n; ++i) w[i] -= al[j] * vj[i];
        if (j > 0)
            for (int i = 0; i < n; ++i) w[i] -= be[j - 1] * V[IDX(i, j - 1, n)];
        for (int pass = 0; pass < 2; ++pass) {          /* classical Gram-Schmidt, twice */
            orc_zgemm('C', 'N', j + 1, 1, n, 1.0, V, n, w, n, 0.0, cc, k + 1);
            orc_zgemm('N', 'N', n, 1, j + 1, -1.0, V, n, cc, k + 1, 1.0, w, n);
        }
        be[j] = znrm2(n, w);
        kk = j + 1;
        if (!(be[j] > 1e-300)) break;
        for (int i = 0; i < n; ++i) V[IDX(i, j + 1, n)] = w[i] / be[j];
    }
    zc* T = (zc*)calloc((size_t)kk * kk, sizeof(zc));
    zc* Z = (zc*)malloc(sizeof(zc) * (size_t)kk * kk);
    for (int j = 0; j < kk; ++j) {
        T[IDX(j, j, kk)] = al[j];
        if (j + 1 < kk) { T[IDX(j + 1, j, kk)] = be[j]; T[IDX(j, j + 1, kk)] = be[j]; }
    }
    orc_jacobi(kk, T, kk, theta, Z, kk);
    for (int j = 0; j < kk; ++j) zw[j] = creal(Z[IDX(0, j, kk)]) * creal(Z[IDX(0, j, kk)]) +
                                      cimag(Z[IDX(0, j, kk)]) * cimag(Z[IDX(0, j, kk)]);
    *beta_k = be[kk - 1];
    free(T); free(Z); free(V); free(w); free(cc); free(al); free(be);
    return kk;
}

/* Bounds from the Lanczos output: b = theta_max + beta_k, mu1 = theta_min, and the cold-start
 * a = smallest theta_j with sum_{i<=j} |z_1i|^2 >= m/n (kept strictly inside (mu1, b)). */
void orc_bounds(int kk, const double* theta, const double* zw, double beta_k, int m, int n,
                double* mu1, double* a, double* b)
{
    *b = theta[kk - 1] + beta_k;
    *mu1 = theta[0];
    double frac = (double)m / (double)n, cum = 0;
    double aa = theta[kk - 1];
    for (int j = 0; j < kk; ++j) {
        cum += zw[j];
        if (cum >= frac) { aa = theta[j]; break; }
    }
    if (!(aa > *mu1) || !(aa < *b)) aa = 0.5 * (*mu1 + *b);
    *a = aa;
}

/* ------------------------------------------------------------------------------------------------
 * Chebyshev filter (Algorithm 1, filtering step), scaled three-term recurrence on [a, b]:
 *   c = (a+b)/2, e = (b-a)/2, sigma_1 = e / (mu1 - c),
 *   Y_1 = (sigma_1 / e) (H - cI) Y_0,
 *   sigma_{k+1} = 1 / (2/sigma_1 - sigma_k),
 *   Y_{k+1} = (2 sigma_{k+1} / e) (H - cI) Y_k - sigma_k sigma_{k+1} Y_{k-1},
 * so that Y_d = T_d((H - cI)/e) Y_0 / T_d((mu1 - c)/e).  Column i stops after deg[i] steps
 * (deg == NULL: every column takes deg_uniform steps); the sigma sequence is shared.  Each step is
 * one product of H with the block of the columns still filtering.
 * ---------------------------------------------------------------------------------------------- */
void orc_filter(int n, const zc* H, int ldh, int m, zc* Y, int ldy, const int* deg, int deg_uniform,
                double a, double b, double mu1)
{
    const double c = 0.5 * (a + b), e = 0.5 * (b - a);
    const double sigma1 = e / (mu1 - c);
    int dmax = 0;
    for (int j = 0; j < m; ++j) {
        int d = deg ? deg[j] : deg_uniform;
        if (d > dmax) dmax = d;
    }
    if (dmax <= 0 || n <= 0) return;
    const size_t nm = (size_t)n * m;
    zc* prev = (zc*)malloc(sizeof(zc) * nm);   /* Y_{k-2} */
    zc* cur = (zc*)malloc(sizeof(zc) * nm);    /* Y_{k-1} */
    zc* nxt = (zc*)malloc(sizeof(zc) * nm);    /* Y_k */
    zc* G = (zc*)malloc(sizeof(zc) * nm);      /* the active columns of Y_{k-1} */
    zc* Z = (zc*)malloc(sizeof(zc) * nm);      /* H times them */
    int* act = (int*)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < n; ++i) cur[IDX(i, j, n)] = Y[IDX(i, j, ldy)];
    double sigma = sigma1;
    for (int k = 1; k <= dmax; ++k) {
        /* step k advances the columns whose degree is at least k */
        int w = 0;
        for (int j = 0; j < m; ++j)
            if ((deg ? deg[j] : deg_uniform) >= k) act[w++] = j;
        for (int q = 0; q < w; ++q)
            memcpy(G + IDX(0, q, n), cur + IDX(0, act[q], n), sizeof(zc) * (size_t)n);
        orc_zgemm('N', 'N', n, w, n, 1.0, H, ldh, G, n, 0.0, Z, n);   /* Z = H Y_{k-1} */
        double alpha, beta, sigma_new;
        if (k == 1) {            /* Y_1 = (sigma_1 / e) (H - cI) Y_0 */
            sigma_new = sigma1;
            alpha = sigma1 / e;
            beta = 0.0;
        } else {                 /* Y_k = (2 sigma_k / e)(H - cI) Y_{k-1} - sigma_{k-1} sigma_k Y_{k-2} */
            sigma_new = 1.0 / (2.0 / sigma1 - sigma);
            alpha = 2.0 * sigma_new / e;
            beta = -sigma * sigma_new;
        }
        #pragma omp parallel for schedule(static)
        for (int q = 0; q < w; ++q) {
            const int j = act[q];
            for (int i = 0; i < n; ++i) {
                zc v = alpha * (Z[IDX(i, q, n)] - c * cur[IDX(i, j, n)]);
                if (k > 1) v += beta * prev[IDX(i, j, n)];
                nxt[IDX(i, j, n)] = v;
            }
            if ((deg ? deg[j] : deg_uniform) == k)   /* the column's last step: Y_d */
                for (int i = 0; i < n; ++i) Y[IDX(i, j, ldy)] = nxt[IDX(i, j, n)];
        }
        sigma = sigma_new;
        zc* t = prev; prev = cur; cur = nxt; nxt = t;
    }
    free(prev); free(cur); free(nxt); free(G); free(Z); free(act);
}

/* Residual norms r_i = || (HY)_i - theta_i Y_i ||_2. */
void orc_residuals(int n, int m, const zc* HY, int ldhy, const zc* Y, int ldy, const double* theta,
                   double* r)
{
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < m; ++j) {
        double s = 0;
        for (int i = 0; i < n; ++i) {
            zc d = HY[IDX(i, j, ldhy)] - theta[j] * Y[IDX(i, j, ldy)];
            s += creal(d) * creal(d) + cimag(d) * cimag(d);
        }
        r[j] = sqrt(s);
    }
}

/* Per-column degree from the textbook growth of T_d outside [-1, 1]:
 * t = (theta - c)/e, rho = |t| + sqrt(t^2 - 1), d = ceil(ln(r / thr) / ln rho) clamped to
 * [dmin, dmax]; columns inside the damped interval or with non-finite data take dmax, columns
 * already below thr take dmin. */
int orc_analytic_degree(double theta, double r, double a, double b, double thr, int dmin, int dmax)
{
    double c = 0.5 * (a + b), e = 0.5 * (b - a);
    double t = (theta - c) / e;
    if (!(fabs(t) > 1.0) || !isfinite(r)) return dmax;
    if (!(r > thr)) return dmin;
    double rho = fabs(t) + sqrt(t * t - 1.0);
    double d = ceil(log(r / thr) / log(rho));
    if (d < dmin) d = dmin;
    if (d > dmax) d = dmax;
    return (int)d;
}

/* ------------------------------------------------------------------------------------------------
 * The whole solver (Algorithm 1 with the reduction of Section 3.2 around it).
 * ---------------------------------------------------------------------------------------------- */
typedef struct {
    int nev, nex, deg;
    double tol;
    int max_loops, lanczos_steps;
    int degree_policy;          /* 0 fixed, 1 analytic */
    int deg_min, deg_max;
    uint64_t seed;
    int have_bounds;
    double mu1, a;
} orc_params;

typedef struct {
    int status, loops, nlocked, lanczos_steps;
    long long filtered_vectors, matvecs;
    double mu1, a, b, norm_a, lock_threshold;
} orc_stats;

enum { ORC_OK = 0, ORC_ERR_ARG = 1, ORC_ERR_NOT_HPD = 2, ORC_ERR_NO_CONVERGENCE = 3, ORC_ERR_NUMERIC = 4 };

int orc_solve(int n, const zc* A, int lda, const zc* S, int lds, zc* X, int ldx, int x_is_guess,
              double* lambda, double* resid, const orc_params* p, orc_stats* st)
{
    const int nev = p->nev, m = p->nev + p->nex;
    memset(st, 0, sizeof(*st));
    if (n <= 0 || nev <= 0 || p->nex < 0 || m > n || p->deg < 0) { st->status = ORC_ERR_ARG; return ORC_ERR_ARG; }
    const size_t nn = (size_t)n * n;

    /* reduction to standard form */
    zc* L = NULL;
    zc* H = (zc*)malloc(sizeof(zc) * nn);
    if (S) {
        L = (zc*)malloc(sizeof(zc) * nn);
        if (orc_cholesky(n, S, lds, L, n)) { free(L); free(H); st->status = ORC_ERR_NOT_HPD; return ORC_ERR_NOT_HPD; }
        orc_reduce(n, A, lda, L, n, H, n);
    } else {
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) H[IDX(i, j, n)] = A[IDX(i, j, lda)];
    }
    double norm_a = 0, s_inf = 1.0;
    for (int j = 0; j < n; ++j) norm_a = fmax(norm_a, znrm2(n, A + IDX(0, j, lda)));
    if (S) {
        s_inf = 0;
        for (int i = 0; i < n; ++i) {
            double rs = 0;
            for (int j = 0; j < n; ++j) rs += cabs(S[IDX(i, j, lds)]);
            s_inf = fmax(s_inf, rs);
        }
    }
    const double thr = p->tol * norm_a / sqrt(s_inf);
    st->norm_a = norm_a;
    st->lock_threshold = thr;

    /* starting block in standard-form coordinates */
    zc* Y = (zc*)malloc(sizeof(zc) * (size_t)n * m);
    if (x_is_guess) {
        if (S) orc_zgemm('C', 'N', n, m, n, 1.0, L, n, X, ldx, 0.0, Y, n);   /* Y0 = L^H X */
        else
            for (int j = 0; j < m; ++j)
                for (int i = 0; i < n; ++i) Y[IDX(i, j, n)] = X[IDX(i, j, ldx)];
    } else {
        orc_random_block(p->seed, 1, n, m, Y, n);
    }

    /* Lanczos bounds */
    int k = p->lanczos_steps;
    if (k < 10) k = 10;
    if (k > 3 * m) k = 3 * m;
    if (k > n) k = n;
    double* theta_t = (double*)malloc(sizeof(double) * (size_t)k);
    double* zw = (double*)malloc(sizeof(double) * (size_t)k);
    double beta_k;
    int kk = orc_lanczos(n, H, n, k, p->seed, theta_t, zw, &beta_k);
    double mu1, a, b;
    orc_bounds(kk, theta_t, zw, beta_k, m, n, &mu1, &a, &b);
    if (p->have_bounds) {
        mu1 = p->mu1;
        a = p->a;
        if (!(a > mu1) || !(a < b)) a = 0.5 * (mu1 + b);
    }
    st->lanczos_steps = kk;
    free(theta_t); free(zw);

    int* degs = (int*)malloc(sizeof(int) * (size_t)m);
    for (int i = 0; i < m; ++i) degs[i] = p->deg;
    zc* HY = (zc*)malloc(sizeof(zc) * (size_t)n * m);
    zc* G = (zc*)malloc(sizeof(zc) * (size_t)m * m);
    zc* Wv = (zc*)malloc(sizeof(zc) * (size_t)m * m);
    zc* R = (zc*)malloc(sizeof(zc) * (size_t)m * m);
    zc* T = (zc*)malloc(sizeof(zc) * (size_t)n * m);
    zc* C = (zc*)malloc(sizeof(zc) * (size_t)m * m);
    zc* AX = (zc*)malloc(sizeof(zc) * (size_t)n * m);
    zc* SX = (zc*)malloc(sizeof(zc) * (size_t)n * m);
    double* theta = (double*)malloc(sizeof(double) * (size_t)m);
    double* r = (double*)malloc(sizeof(double) * (size_t)m);
    int nlocked = 0, status = ORC_ERR_NO_CONVERGENCE, loops = 0;

    for (int it = 0; it < p->max_loops; ++it) {
        const int ma = m - nlocked;
        zc* Ya = Y + IDX(0, nlocked, n);
        loops = it + 1;

        /* 1. filter */
        orc_filter(n, H, n, ma, Ya, n, degs + nlocked, 0, a, b, mu1);
        st->filtered_vectors += ma;
        for (int i = nlocked; i < m; ++i) st->matvecs += degs[i];

        /* 2. re-orthonormalise: CGS twice against the locked vectors, then Householder QR */
        if (nlocked > 0)
            for (int pass = 0; pass < 2; ++pass) {
                orc_zgemm('C', 'N', nlocked, ma, n, 1.0, Y, n, Ya, n, 0.0, C, m);
                orc_zgemm('N', 'N', n, ma, nlocked, -1.0, Y, n, C, m, 1.0, Ya, n);
            }
        if (orc_qr(n, ma, Ya, n, R, m)) { status = ORC_ERR_NUMERIC; break; }

        /* 3. Rayleigh-Ritz: G = Ya^H H Ya, G = W diag(theta) W^H, Ya <- Ya W */
        orc_zgemm('N', 'N', n, ma, n, 1.0, H, n, Ya, n, 0.0, HY, n);
        orc_zgemm('C', 'N', ma, ma, n, 1.0, Ya, n, HY, n, 0.0, G, m);
        orc_jacobi(ma, G, m, theta, Wv, m);
        orc_zgemm('N', 'N', n, ma, ma, 1.0, Ya, n, Wv, m, 0.0, T, n);
        for (int j = 0; j < ma; ++j) memcpy(Ya + IDX(0, j, n), T + IDX(0, j, n), sizeof(zc) * (size_t)n);
        orc_zgemm('N', 'N', n, ma, ma, 1.0, HY, n, Wv, m, 0.0, T, n);
        memcpy(HY, T, sizeof(zc) * (size_t)n * ma);

        /* 4. residuals and locking of the converged prefix */
        orc_residuals(n, ma, HY, n, Ya, n, theta, r);
        int nonfinite = 0;
        for (int j = 0; j < ma; ++j) if (!isfinite(r[j]) || !isfinite(theta[j])) nonfinite = 1;
        if (nonfinite) { status = ORC_ERR_NUMERIC; break; }
        int cnt = 0;
        while (cnt < nev - nlocked && r[cnt] <= thr) ++cnt;
        for (int j = 0; j < ma; ++j) { lambda[nlocked + j] = theta[j]; resid[nlocked + j] = r[j]; }
        nlocked += cnt;

        /* 5. bounds for the next filter, per-column degrees */
        a = theta[ma - 1];
        if (theta[0] < mu1) mu1 = theta[0];
        if (!(a > mu1)) a = 0.5 * (mu1 + b);
        if (p->degree_policy == 1)
            for (int j = cnt; j < ma; ++j)
                degs[nlocked + j - cnt] = orc_analytic_degree(theta[j], r[j], a, b, thr, p->deg_min, p->deg_max);

        if (nlocked >= nev) {
            /* back-transform X = L^{-H} Y and check ||A x - lambda S x|| / ||A||_lo */
            for (int j = 0; j < m; ++j)
                for (int i = 0; i < n; ++i) X[IDX(i, j, ldx)] = Y[IDX(i, j, n)];
            if (S) orc_trsm_lower_h(n, m, L, n, X, ldx);
            orc_zgemm('N', 'N', n, m, n, 1.0, A, lda, X, ldx, 0.0, AX, n);
            if (S) orc_zgemm('N', 'N', n, m, n, 1.0, S, lds, X, ldx, 0.0, SX, n);
            else
                for (int j = 0; j < m; ++j)
                    for (int i = 0; i < n; ++i) SX[IDX(i, j, n)] = X[IDX(i, j, ldx)];
            for (int j = 0; j < m; ++j) {
                double s = 0;
                for (int i = 0; i < n; ++i) {
                    zc d = AX[IDX(i, j, n)] - lambda[j] * SX[IDX(i, j, n)];
                    s += creal(d) * creal(d) + cimag(d) * cimag(d);
                }
                resid[j] = sqrt(s) / norm_a;
            }
            int bad = -1;
            for (int j = 0; j < nev; ++j) if (!(resid[j] <= p->tol)) { bad = j; break; }
            if (bad < 0) { status = ORC_OK; break; }
            nlocked = bad;      /* unlock the failing pair and everything locked after it */
            for (int i = bad; i < m; ++i) degs[i] = p->deg;
        }
    }
    if (status == ORC_ERR_NO_CONVERGENCE) {
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < n; ++i) X[IDX(i, j, ldx)] = Y[IDX(i, j, n)];
        if (S) orc_trsm_lower_h(n, m, L, n, X, ldx);
    }
    st->status = status;
    st->loops = loops;
    st->nlocked = nlocked;
    st->mu1 = mu1; st->a = a; st->b = b;
    free(degs); free(HY); free(G); free(Wv); free(R); free(T); free(C); free(AX); free(SX);
    free(theta); free(r); free(Y); free(H); free(L);
    return status;
}

int orc_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------------------------------
 * Correlation of two successive problems of a sequence (Section 2.2: scalar products between the
 * eigenvectors of neighbouring problems, and the deviation angle of each eigenvector from its
 * counterpart, Fig. 1).  Xp, Xc: n x m, S-orthonormal columns (S = NULL: the identity).
 *   O = Xp^H S Xc                                   (m x m, the matrix of scalar products)
 *   sin_pair[i] = || xc_i - xp_i O_ii ||_S / || xc_i ||_S      (sine of the angle of pair i)
 *   sin_sub[k]  = sqrt of the eigenvalues, ascending, of R^H S R with R = Xc - Xp O
 *                 (sines of the principal angles between the two spans)
 * The sines come from differences of vectors, never from 1 - |O|^2, so angles of 1e-8 keep their
 * digits.
 * ---------------------------------------------------------------------------------------------- */
static double s_norm2(int n, const zc* S, int lds, const zc* x)
{
    double s = 0;
    if (!S) {
        for (int i = 0; i < n; ++i) s += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
        return s;
    }
    zc* t = (zc*)malloc(sizeof(zc) * (size_t)n);
    orc_zgemm('N', 'N', n, 1, n, 1.0, S, lds, x, n, 0.0, t, n);
    zc d = 0;
    for (int i = 0; i < n; ++i) d += conj(x[i]) * t[i];
    free(t);
    return creal(d);
}

void orc_correlation(int n, int m, const zc* S, int lds, const zc* Xp, int ldxp, const zc* Xc, int ldxc, zc* O,
                     int ldo, double* sin_pair, double* sin_sub)
{
    zc* SX = (zc*)malloc(sizeof(zc) * (size_t)n * m);
    zc* r = (zc*)malloc(sizeof(zc) * (size_t)n);
    zc* R = (zc*)malloc(sizeof(zc) * (size_t)n * m);
    zc* SR = (zc*)malloc(sizeof(zc) * (size_t)n * m);
    zc* G = (zc*)malloc(sizeof(zc) * (size_t)m * m);
    zc* V = (zc*)malloc(sizeof(zc) * (size_t)m * m);
    double* w = (double*)malloc(sizeof(double) * (size_t)m);
    /* O = Xp^H (S Xc) */
    if (S) orc_zgemm('N', 'N', n, m, n, 1.0, S, lds, Xc, ldxc, 0.0, SX, n);
    else
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < n; ++i) SX[IDX(i, j, n)] = Xc[IDX(i, j, ldxc)];
    orc_zgemm('C', 'N', m, m, n, 1.0, Xp, ldxp, SX, n, 0.0, O, ldo);
    /* angle of each pair (xp_i, xc_i) */
    for (int i = 0; i < m; ++i) {
        const zc oii = O[IDX(i, i, ldo)];
        for (int k = 0; k < n; ++k) r[k] = Xc[IDX(k, i, ldxc)] - Xp[IDX(k, i, ldxp)] * oii;
        sin_pair[i] = sqrt(fmax(s_norm2(n, S, lds, r), 0.0) / s_norm2(n, S, lds, Xc + IDX(0, i, ldxc)));
    }
    /* principal angles: R = Xc - Xp O, eigenvalues of R^H S R */
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < n; ++i) R[IDX(i, j, n)] = Xc[IDX(i, j, ldxc)];
    orc_zgemm('N', 'N', n, m, m, -1.0, Xp, ldxp, O, ldo, 1.0, R, n);
    if (S) orc_zgemm('N', 'N', n, m, n, 1.0, S, lds, R, n, 0.0, SR, n);
    else memcpy(SR, R, sizeof(zc) * (size_t)n * m);
    orc_zgemm('C', 'N', m, m, n, 1.0, R, n, SR, n, 0.0, G, m);
    orc_jacobi(m, G, m, w, V, m);
    for (int k = 0; k < m; ++k) sin_sub[k] = sqrt(fmax(w[k], 0.0));
    free(SX); free(r); free(R); free(SR); free(G); free(V); free(w);
}
