// Internal declarations of the gfx950 ChFSI library: complex types, device helpers and the
// launchers each translation unit exports to the host driver.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double2 zd;   // complex double, interleaved (re, im)
typedef float2 zf;    // complex float
typedef double __attribute__((ext_vector_type(4))) d4;
typedef float __attribute__((ext_vector_type(4))) f4;

#define CHK_HIP(x)                                                   \
    do {                                                             \
        hipError_t e_ = (x);                                         \
        if (e_ != hipSuccess) return chfsi_internal_hip_error(e_);   \
    } while (0)

int chfsi_internal_hip_error(hipError_t e);

__host__ __device__ inline zd zmul(zd a, zd b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__host__ __device__ inline zd zcmul(zd a, zd b) { return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }  // conj(a) b
__host__ __device__ inline double zabs2(zd a) { return a.x * a.x + a.y * a.y; }

// 1 / sqrt(x), x > 0 normal: the hardware estimate (v_rsq_f64) refined by two Newton steps, each of
// which roughly squares the relative error, so any estimate good to 2^-14 ends at double precision
__device__ inline double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * (1.5 - hx * y * y);
    y = y * (1.5 - hx * y * y);
    return y;
}

// ---- GEMM (gemm.hip) --------------------------------------------------------------------------
// C = alpha op(A) op(B) + beta C, complex, op = N or C, all device pointers, real scalars.
// `ws`/`ws_bytes` is scratch for split-K partials (may be null: no split).
enum { OP_N = 0, OP_C = 1 };
enum { PREC_F64 = 0, PREC_F32 = 1 };

// Scratch of the GEMM launches: split-K partials plus one arrival counter per output tile.  The
// counters must be zero before a launch; each launch leaves them zero again.
struct GemmWs {
    void* ws = nullptr;
    size_t bytes = 0;
    int* cnt = nullptr;
    int ncnt = 0;
    // forced tile plan (plan_bm == 0: choose automatically): output tile plan_bm x plan_bn
    // (32 or 64 each), K split plan_ksplit, split mode 1 (partials + reduce kernel) or 2 (fused)
    int plan_bm = 0, plan_bn = 0, plan_ksplit = 0, plan_mode = 1;
    // launch timing of a filter step (all three set, or none): ev_start takes the start of the
    // step's first kernel, ev_main the end of its main kernel and ev_end the end of its last kernel,
    // each from the dispatch's own timestamps (no marker between the kernels)
    hipEvent_t ev_start = nullptr, ev_main = nullptr, ev_end = nullptr;
    int* plan_used = nullptr;       // when set, receives bm, bn, ksplit, mode of the launch
};

// Launches kernel<<<grid, block, 0, s>>>(args...); `start` / `stop` (either may be null) are set
// to the kernel's own start and end times.
template <typename F, typename... Args>
inline void launch_timed(F kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t start, hipEvent_t stop,
                         Args... args)
{
    if (start || stop) hipExtLaunchKernelGGL(kernel, grid, block, 0, s, start, stop, 0, args...);
    else hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

struct FilterStep {
    // out = alpha * (H Yk - shift Yk) + beta * Yprev, columns [0, ncols)
    double alpha, beta, shift;
};

// Restricted products of launch_zgemm_tri (gemm.hip)
enum { TRI_C_LOWER = 1, TRI_B_BLOCK_LOWER = 2, TRI_A_LOWER = 4, TRI_B_UPPER = 8 };
int launch_zgemm_tri(hipStream_t s, int tri, int opa, int opb, int M, int N, int K, double alpha, const zd* A,
                     int lda, const zd* B, int ldb, double beta, zd* C, int ldc);

// FP64 complex GEMM on MFMA.  Returns hipError_t as int.
int launch_zgemm(hipStream_t s, int opa, int opb, int M, int N, int K, double alpha, const zd* A, int lda,
                 const zd* B, int ldb, double beta, zd* C, int ldc, const GemmWs& gw);
// One filter step, FP64: Yout = alpha (H Yk - shift Yk) + beta Yprev (Yout may alias Yprev).
int launch_filter_step_f64(hipStream_t s, int n, int ncols, const zd* H, int ldh, const zd* Yk, int ldyk,
                           const zd* Yprev, int ldyp, zd* Yout, int ldyo, FilterStep fs, const GemmWs& gw);
// One filter step, FP32 complex (complex64 storage, FP32 MFMA and accumulation).
int launch_filter_step_f32(hipStream_t s, int n, int ncols, const zf* H, int ldh, const zf* Yk, int ldyk,
                           const zf* Yprev, int ldyp, zf* Yout, int ldyo, FilterStep fs, const GemmWs& gw);
size_t zgemm_ws_bytes(int M, int N, int K, int elem_bytes);

// ---- BF16-split filter (gemm_bf16.hip) ---------------------------------------------------------
// H planes: for each of the `nterms` split terms, separate re and im planes of bf16, column-major
// with leading dimension ldh (elements).  Yk is complex64.
int launch_split_h_bf16(hipStream_t s, int n, const zd* H, int ldh, uint16_t* planes, int ldp, int nterms);
int launch_filter_step_bf16(hipStream_t s, int n, int ncols, const uint16_t* Hplanes, int ldp, int nterms,
                            const zf* Yk, int ldyk, const zf* Yprev, int ldyp, zf* Yout, int ldyo,
                            FilterStep fs, uint16_t* ysplit, const GemmWs& gw);
size_t bf16_ysplit_bytes(int n, int ncols, int nterms);
size_t bf16_hplanes_elems(int n, int nterms);

// ---- level-1/2 and small kernels (blas1.hip) ----------------------------------------------------
int launch_zlacpy(hipStream_t s, int M, int N, const zd* A, int lda, zd* B, int ldb);
int launch_z2c(hipStream_t s, int M, int N, const zd* A, int lda, zf* B, int ldb);   // complex128 -> complex64
int launch_c2z(hipStream_t s, int M, int N, const zf* A, int lda, zd* B, int ldb);   // complex64 -> complex128
// upper triangle <- conjugate transpose of the lower triangle, diagonal made real
int launch_mirror_lower(hipStream_t s, int n, zd* H, int ldh);
int launch_philox_block(hipStream_t s, unsigned long long seed, unsigned long long stream, int n, int m, zd* Y,
                        int ldy);
// y[j] = conj(V[:, j]) . x  for j < ncols (column dot products; for Hermitian V this is V x)
int launch_coldots(hipStream_t s, int n, int ncols, const zd* V, int ldv, const zd* x, zd* y);
// x += alpha * V c   (c length ncols, device; alpha real)
int launch_gemv_n(hipStream_t s, int n, int ncols, const zd* V, int ldv, const zd* c, double alpha, zd* x);
// residual norms r[j] = || HY[:, j] - theta[j] Y[:, j] ||  (theta, r device)
int launch_residual_norms(hipStream_t s, int n, int m, const zd* HY, int ldhy, const zd* Y, int ldy,
                          const double* theta, double* r);
int launch_colnorms(hipStream_t s, int n, int m, const zd* Y, int ldy, double* r);
// d[j] = Re(A[:, j]^H B[:, j])  (d device, m doubles)
int launch_pair_dots(hipStream_t s, int n, int m, const zd* A, int lda, const zd* B, int ldb, double* d);
// *flag |= 1 (device) when A and B (n x n) differ in any bit; flag is not cleared
int launch_any_diff(hipStream_t s, int n, const zd* A, int lda, const zd* B, int ldb, int* flag);
// Y[:, j] *= 1/sqrt(d[j]) (0 when d[j] <= 0), d device
int launch_scale_cols_rsqrt(hipStream_t s, int n, int m, zd* Y, int ldy, const double* d);
// W[:, c] = AX[:, idx[c]] - theta[idx[c]] BX[:, idx[c]] for c < na (theta, idx device)
int launch_residual_gather(hipStream_t s, int n, int na, const zd* AX, int lda, const zd* BX, int ldb,
                           const double* theta, const int* idx, zd* W, int ldw);
// T[:, c] = U[:, k-1-c] / sqrt(g[k-1-c]) for c < kept (g ascending, device)
int launch_orth_factor(hipStream_t s, int k, int kept, const zd* U, int ldu, const double* g, zd* T, int ldt);
// D[:, j] = Xc[:, j] - O_jj Xp[:, j]
int launch_sub_diag_scaled(hipStream_t s, int n, int m, const zd* Xc, int ldc, const zd* Xp, int ldp, const zd* O,
                           int ldo, zd* D, int ldd);
int launch_scale_cols_inv(hipStream_t s, int n, int m, zd* Y, int ldy, const double* nrm);   // Y[:, j] /= nrm[j]
int launch_max_colnorm(hipStream_t s, int n, const zd* A, int lda, double* out);            // max_j ||A[:, j]||
int launch_max_rowsum_abs(hipStream_t s, int n, const zd* A, int lda, double* out);         // ||A||_inf
// out[0] = max_i sum_j |A_ij - delta_ij| (A Hermitian n x n; out: n + 1 doubles)
int launch_max_rowsum_off_identity(hipStream_t s, int n, const zd* A, int lda, double* out);
// G <- F = strict upper triangle of G + diag((G_jj - 1) / 2): the first-order factor of G = I + E
int launch_first_order_factor(hipStream_t s, int m, zd* G, int ldg);
int launch_add_diag(hipStream_t s, int m, zd* G, int ldg, const double* shift_dev, double factor);
int launch_fro2(hipStream_t s, int n, int m, const zd* Y, int ldy, double* out);            // ||Y||_F^2
// Lanczos helpers
// alpha = Re(v^H w) written to *alpha_out (device), w -= alpha v + beta_prev v_prev; dot: device
// scratch for the complex product
int launch_lanczos_alpha(hipStream_t s, int n, const zd* v, zd* w, const zd* vprev, double* alpha_out,
                         const double* beta_prev, zd* dot);
int launch_lanczos_normalize(hipStream_t s, int n, const zd* w, zd* vnext, double* beta_out);
// phase-normalize eigenvector columns: largest-magnitude entry (first on ties) real positive
int launch_phase_normalize(hipStream_t s, int m, int ncols, zd* W, int ldw);
int launch_any_nonfinite(hipStream_t s, int n, const double* v, int* flag);
// gather/scatter columns: dst[:, j] = src[:, perm[j]]
int launch_permute_cols(hipStream_t s, int n, int m, const zd* src, int lds, zd* dst, int ldd, const int* perm);
int launch_copy_cols_flag(hipStream_t s, int n, int m, const zd* src, int lds, zd* dst, int ldd, const int* flag);
int launch_copy_cols_flag_c(hipStream_t s, int n, int m, const zf* src, int lds, zf* dst, int ldd, const int* flag);

// ---- Cholesky factorisation (chol.hip) -----------------------------------------------------------
// A = L L^H in place (lower triangle read and written), blocked with 64-column panels; *info
// (device, zero on entry) receives the first non-positive pivot, 1-based; dinv (device,
// tri_dinv_elems(n) elements) receives the inverses of L's 64 x 64 diagonal blocks (block kb at
// dinv + 4096 kb, column-major, ld 64), which the triangular solves below take with L.
int chol_lower(hipStream_t s, int n, zd* A, int lda, int* info, zd* dinv, const GemmWs& gw);

// ---- triangular solves with a lower Cholesky factor L (trsm.hip) ---------------------------------
size_t tri_dinv_elems(int n);
enum { TA_LEFT_N = 0, TA_LEFT_C = 1, TA_RIGHT_C = 2 };
// in place: TA_LEFT_N B <- D B (B nb x nvec), TA_LEFT_C B <- D^H B, TA_RIGHT_C B <- B D^H (B nvec x nb);
// D: 64 x 64 column-major, nb <= 64
int tri_apply(hipStream_t s, int mode, int nb, int nvec, const zd* D, zd* B, int ldb);
int trsm_left_lower(hipStream_t s, int n, int nrhs, const zd* L, int ldl, const zd* dinv, zd* B, int ldb,
                    const GemmWs& gw);   // L X = B
int trsm_left_lower_h(hipStream_t s, int n, int nrhs, const zd* L, int ldl, const zd* dinv, zd* B, int ldb,
                      const GemmWs& gw);   // L^H X = B
int trsm_right_lower_h(hipStream_t s, int nrow, int ncol, const zd* L, int ldl, const zd* dinv, zd* B, int ldb,
                       const GemmWs& gw);   // X L^H = B
// lower triangle of X with X L^H = B (B n x n; what H = W L^{-H} needs when H is Hermitian)
int trsm_right_lower_h_lowertri(hipStream_t s, int n, const zd* L, int ldl, const zd* dinv, zd* B, int ldb,
                                const GemmWs& gw);
// lower triangle of C (n x n) -= A B^H, A and B n x K
int gemm_lower_nc(hipStream_t s, int n, int K, const zd* A, int lda, const zd* B, int ldb, zd* C, int ldc,
                  const GemmWs& gw);

// ---- reduction to standard form (hegst.hip) -------------------------------------------------------
size_t hegst_work_elems(int n);
// A (lower triangle read) <- H = L^{-1} A L^{-H} in full, L lower with its stored diagonal-block
// inverses dinv; work: hegst_work_elems(n) elements
int hegst_lower(hipStream_t s, int n, zd* A, int lda, const zd* L, int ldl, const zd* dinv, zd* work,
                const GemmWs& gw);
// Y1 = alpha (HY - shift Y0) on columns [0, w) (HY complex128; Y0, Y1 complex128 or complex64): the
// first filter step of a block whose image HY = H Y0 is known
int launch_first_step(hipStream_t s, int n, int w, double alpha, double shift, const zd* HY, int ldhy, const zd* Y0,
                      int ldy0, zd* Y1, int ldy1);
int launch_first_step(hipStream_t s, int n, int w, double alpha, double shift, const zd* HY, int ldhy, const zf* Y0,
                      int ldy0, zf* Y1, int ldy1);
// X <- L^{-1} (n x n, zero above the diagonal) from L and its diagonal-block inverses dinv
int tri_inverse_lower(hipStream_t s, int n, const zd* L, int ldl, const zd* dinv, zd* X, int ldx, const GemmWs& gw);
// H (ld n) <- Linv A Linv^H (exactly Hermitian) from the explicit inverse Linv = L^{-1} (ld n) and the
// full Hermitian A; T: n x n elements of scratch
int hegst_explicit(hipStream_t s, int n, const zd* A, int lda, const zd* Linv, zd* T, zd* H);

// ---- Hermitian eigensolver of the Rayleigh quotient (eig.hip) -----------------------------------
int eig_padded_order(int m);
size_t eig_work_bytes(int m);
size_t eig_host_doubles(int m);
// G (m x m, device) <- W with G = W diag(theta) W^H, theta ascending (device).  host: at least
// eig_host_doubles(m) doubles.  Returns hipError_t as int, -1 when the sweeps did not converge.
// stop_abs: off-diagonal level (absolute) that is accurate enough for the caller; the sweeps stop at
// max(5e-14 scale, stop_abs) (0: at 5e-14 of the matrix scale)
int eig_jacobi(hipStream_t s, int m, zd* G, int ldg, double* theta, void* work, double* host, int* sweeps,
               double stop_abs = 0.0);

// ---- degree network (mlp.hip) -------------------------------------------------------------------
#define MLP_NF 5
#define MLP_NH 64
#define MLP_NPARAM (MLP_NH * MLP_NF + MLP_NH + 2 * (MLP_NH * MLP_NH + MLP_NH) + MLP_NH + 1)
int launch_mlp_forward(hipStream_t s, const float* P, int N, const float* X, float dmin, float dmax, float* out);
int launch_mlp_loss_grad(hipStream_t s, const float* P, int N, const float* X, const float* y, float dmin,
                         float dmax, float* grad, float* loss_dev, float* scratch);
size_t mlp_scratch_floats(int N);
int launch_mlp_adam(hipStream_t s, int np, float* P, const float* g, float* m, float* v, int t, float lr,
                    float b1, float b2, float eps);
int launch_gather_rows5(hipStream_t s, int nb, const float* X, const float* y, const int* idx, float* Xb, float* yb);
// features for the degree network from per-column (theta, r) and the filter bounds
int launch_degree_features_ext(hipStream_t s, int m, const double* theta, const double* r, double a, double b,
                               double mu1, double thr, const int* dprev, const float* norm, float* feat);
