/*
 * chfsi.h -- C ABI of the MI355X (gfx950) Chebyshev-filtered subspace iteration library.
 *
 * The method is Algorithm 1 of Di Napoli & Berljafa, "Block iterative eigensolvers for sequences
 * of correlated eigenvalue problems" (ChFSI with deflation and locking), wrapped by the reduction
 * of a generalized Hermitian pencil A x = lambda S x to standard form (Section 3.2) and the
 * back-transformation of the eigenvectors.
 *
 * Conventions for every entry point
 *  - Matrices are column-major complex double (interleaved re, im; layout-compatible with
 *    C99 `double _Complex` and std::complex<double>), leading dimension >= rows.
 *  - Matrix arguments are DEVICE pointers on the handle's device; `lambda`, `resid`, `deg`,
 *    `theta` and other small vectors are HOST pointers unless stated otherwise.
 *  - The caller owns every pointer it passes; the library never frees or keeps them past the
 *    return.  The library owns its workspace, grows it on demand and frees it in chfsi_destroy.
 *  - Every call enqueues its work on the handle's stream and is synchronous on return.
 *  - A status code is returned; no C++ exception crosses this interface.  Outputs are undefined
 *    on any status other than CHFSI_SUCCESS, except as stated for CHFSI_ERR_NO_CONVERGENCE.
 *  - One handle per host thread.
 */
#ifndef CHFSI_H
#define CHFSI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chfsi_handle_s* chfsi_handle;

typedef enum {
    CHFSI_SUCCESS = 0,
    CHFSI_ERR_ARG = 1,            /* invalid size, pointer or parameter                         */
    CHFSI_ERR_NOT_HPD = 2,        /* a Cholesky pivot of S was not positive                     */
    CHFSI_ERR_NO_CONVERGENCE = 3, /* max_loops reached; the locked prefix is valid              */
    CHFSI_ERR_NUMERIC = 4,        /* NaN/Inf in inputs or iterates, or a breakdown in QR        */
    CHFSI_ERR_DEVICE = 5,         /* a HIP runtime call failed                                  */
    CHFSI_ERR_ALLOC = 6,          /* device or host allocation failed                           */
    CHFSI_ERR_TOO_LARGE = 7       /* input larger than the fixed scratch of chfsi_filter_noalloc */
} chfsi_status;

/* Arithmetic of the Chebyshev filter.  Every other step (reduction, Lanczos, QR, Rayleigh-Ritz,
 * residuals, locking) is FP64 regardless of this setting. */
typedef enum {
    CHFSI_FP64 = 0,               /* complex128 on FP64 MFMA                                    */
    CHFSI_FP32 = 1,               /* complex64 on FP32 MFMA, FP32 accumulation                  */
    CHFSI_BF16X3 = 2,             /* FP32 operands split into 2 BF16 terms, 3 products, FP32 acc */
    CHFSI_BF16X6 = 3              /* FP32 operands split into 3 BF16 terms, 6 products, FP32 acc */
} chfsi_precision;

/* Per-vector filter degree (Algorithm 1 uses one fixed degree). */
typedef enum {
    CHFSI_DEG_FIXED = 0,          /* every vector gets `deg`                                    */
    CHFSI_DEG_ANALYTIC = 1,       /* from the Chebyshev growth rate at its Ritz value           */
    CHFSI_DEG_LEARNED = 2,        /* from the degree network set by chfsi_set_degree_model      */
    CHFSI_DEG_RANDOM = 3          /* uniform in [deg_min, deg_max] (Philox stream 4): traces    */
} chfsi_degree_policy;

typedef struct {
    int nev;                      /* wanted eigenpairs (lowest part of the spectrum)            */
    int nex;                      /* extra vectors: block size m = nev + nex (paper: nev + 40)  */
    int deg;                      /* filter degree; initial degree for adaptive policies (25)   */
    double tol;                   /* target for ||A x - lambda S x|| / ||A||  (1e-10)           */
    int max_loops;                /* inner-loop limit (50)                                      */
    int lanczos_steps;            /* clamped to [10, 3 m] and to n (25)                         */
    int filter_precision;         /* chfsi_precision (CHFSI_FP64)                               */
    int degree_policy;            /* chfsi_degree_policy (CHFSI_DEG_FIXED)                      */
    int deg_min, deg_max;         /* degree clamp for adaptive policies ([4, 30])               */
    unsigned long long seed;      /* random start block and Lanczos start vector (0)            */
    int have_bounds;              /* 1: use mu1 and a below (warm start of a sequence)          */
    double mu1;                   /* lower spectral estimate (previous lambda_1)                */
    double a;                     /* lower end of the damped interval (previous largest Ritz)   */
    int trace;                    /* 1: record per-vector (features, residual history) rows     */
    double switch_residual;       /* mixed precision: a vector whose residual falls below
                                     switch_residual * ||A||_lo is filtered in FP64 from then on
                                     (0 = precision-dependent default)                          */
    int deg_margin;               /* added to every degree of the ANALYTIC and LEARNED policies
                                     (before the clamp to deg_max): a safety margin against an
                                     extra loop caused by an underestimated degree (0)           */
} chfsi_params;

typedef struct {
    int loops;                    /* inner loops of Algorithm 1                                 */
    int nlocked;                  /* locked (converged) pairs                                   */
    long long filtered_vectors;   /* sum over loops of the active block width                   */
    long long matvecs;            /* sum over loops and vectors of the filter degree            */
    double filter_flops;          /* 8 n^2 per product the filter performed (complex GEMM
                                     count): the first step of a loop after the first is formed
                                     from the Rayleigh-Ritz step's H Y without a product, so this
                                     is 8 n^2 (matvecs - vectors filtered in those loops)      */
    double t_reduce, t_lanczos, t_filter, t_qr, t_rr, t_resid, t_lock, t_back, t_total; /* ms */
    double mu1, a, b;             /* final filter bounds                                        */
    double norm_a;                /* largest column 2-norm of A (lower bound of ||A||_2)        */
    int lanczos_steps;            /* Lanczos steps taken                                        */
    int precision_switches;       /* vectors moved from low precision to FP64                   */
    int filter_launches;          /* filter steps                                               */
    double t_filter_kernels;      /* ms: hipEvent-timed main filter kernel launches (summed)    */
    double t_filter_steps;        /* ms: the same launches plus their split-K reduce kernels    */
    int status;                   /* chfsi_status of this solve                                 */
    int factor_reused;            /* 1: S equal to the last factored overlap, its factor reused  */
} chfsi_stats;

/* One problem of a batch (chfsi_solve_batched); same meaning as chfsi_solve's arguments. */
typedef struct {
    int n, nev, nex;
    const void* A; int lda;
    const void* S; int lds;       /* NULL = standard problem                                    */
    void* X; int ldx;
    int x_is_guess;
    double* lambda;               /* host [nev + nex]                                           */
    double* resid;                /* host [nev + nex]                                           */
} chfsi_problem;

/* Tile plan of the filter-step kernel: a bm x bn complex output tile per workgroup (32 or 64
 * each) and the K dimension cut into ksplit slices (1 = none) whose partial tiles are summed in
 * slice order either by a second kernel (fused = 0) or by the last slice to finish (fused = 1). */
typedef struct { int bm, bn, ksplit, fused; } chfsi_tile_plan;

/* Fills *p with the defaults listed above (Table 3 of the paper: degree 25, TOL 1e-10). */
void chfsi_default_params(chfsi_params* p);

/* Creates a handle on `device` that enqueues on `hip_stream` (NULL = the null stream).
 * Errors: CHFSI_ERR_ARG (h NULL), CHFSI_ERR_DEVICE, CHFSI_ERR_ALLOC. */
chfsi_status chfsi_create(chfsi_handle* h, int device, void* hip_stream);
chfsi_status chfsi_destroy(chfsi_handle h);

/* Solves A x = lambda S x for the nev lowest eigenpairs with Algorithm 1 (Section 3.1), after
 * reducing to H = L^{-1} A L^{-H}, S = L L^H (Section 3.2; L^T in the paper read as L^H).
 *   A, lda   n x n Hermitian, full storage, not modified.
 *   S, lds   n x n Hermitian positive definite, not modified; NULL = standard problem (S = I).
 *   X, ldx   n x m, m = nev + nex.  In: warm-start block in generalized coordinates when
 *            x_is_guess != 0 (ignored otherwise: a Philox4x64-10 uniform block of stream 1 keyed
 *            by p->seed is used).  Out: Ritz vectors, S-orthonormal; the first nev converged.
 *   lambda   host [m]: ascending Ritz values; the first nev converged.
 *   resid    host [m]: ||A x_i - lambda_i S x_i||_2 / ||A||_lo.
 *   p        parameters (NULL = defaults); stats (nullable) receives counters and phase times.
 * The handle keeps the Cholesky factor of the last overlap it factored, with a copy of that S
 * (2 n^2 complex elements of device memory): a solve whose S equals it bit for bit (the overlap of
 * a sequence whose basis does not change) reuses the factor and only forms H; any other S is
 * factored again (stats->factor_reused says which).
 * Returns CHFSI_ERR_NOT_HPD if S is not positive definite, CHFSI_ERR_NO_CONVERGENCE when
 * max_loops is reached (stats->nlocked pairs at the front of X, lambda, resid are valid),
 * CHFSI_ERR_NUMERIC on NaN/Inf or QR breakdown. */
chfsi_status chfsi_solve(chfsi_handle h, int n, const void* A, int lda, const void* S, int lds,
                         void* X, int ldx, int x_is_guess, double* lambda, double* resid,
                         const chfsi_params* p, chfsi_stats* stats);

/* Solves `count` independent problems (the k-points of one self-consistent cycle, Section 2.1:
 * one generalized eigenproblem per k-point) with shared parameters p (p->nev and p->nex are
 * ignored: each problem carries its own; p->filter_precision must be CHFSI_FP64; p->trace has
 * no effect).  All unconverged problems advance through Algorithm 1 in lockstep loops: each
 * filter step of all of them is one persistent launch over a work list of output tiles of every
 * problem (tile plan from chfsi_autotune_batched / chfsi_set_batched_plan), the steps of a loop
 * replayed as one captured HIP graph; QR, Rayleigh-Ritz, locking and verification run per problem,
 * spread over the handle's lanes (streams, chfsi_set_batched_plan; three by default), one host
 * thread per lane during those steps, since they wait on the host; the reduction of a problem
 * completes before more work is enqueued.  The call is not reentrant on one handle.  Per problem
 * the results match chfsi_solve with the same parameters up to rounding.  Up to 64 problems share a launch; larger batches run in chunks of 64.
 * stats: [count], nullable; t_total of every entry is the wall time of the whole call, phase
 * times are not recorded (chfsi_batched_info has the filter time).  Returns the first
 * non-success status of any problem; the others are still solved. */
chfsi_status chfsi_solve_batched(chfsi_handle h, int count, const chfsi_problem* probs,
                                 const chfsi_params* p, chfsi_stats* stats);

/* Tile plan of the persistent multi-problem filter kernel of chfsi_solve_batched (bm, bn in
 * {32, 64}; ksplit and fused are ignored; plan NULL keeps the current one), whether each loop's
 * filter steps replay a captured HIP graph (use_graph != 0, the default) or are launched one by
 * one, and over how many streams (lanes, 1 .. 8; 0 keeps the current value, default 3) the
 * per-problem dense steps are spread (with more than one, each lane's dense steps run on a host
 * thread of their own). */
chfsi_status chfsi_set_batched_plan(chfsi_handle h, const chfsi_tile_plan* plan, int use_graph, int lanes);

/* Project autotuner of the persistent multi-problem filter kernel: times one filter step over all
 * `count` (<= 64) problems for every candidate tile (64x64, 64x32, 32x64, 32x32) with hipEvents,
 * reading A as the matrix and X as the block (neither is modified; outputs go to scratch it
 * allocates and frees), keeps the fastest for later chfsi_solve_batched calls and returns it with
 * its time per step in ms (both nullable). */
chfsi_status chfsi_autotune_batched(chfsi_handle h, int count, const chfsi_problem* probs,
                                    chfsi_tile_plan* best, double* best_ms);

/* Project autotuner of a tile per problem (a tile per order n and block width m = nev + nex), timed
 * on one filter step of the whole batch of `count` (<= 64) problems: first every one-tile kernel
 * (64x64, 64x32, 32x64, 32x32), then the persistent kernel that takes a tile per problem, starting
 * from the best one tile, the problems ordered by n in four groups, each group trying every shape
 * with the others fixed.  The faster of the two kernels serves later chfsi_solve_batched calls; its
 * tile per problem is kept per (n, m) and returned in tiles[count] (nullable; ksplit 1, fused 0),
 * the step time in *batch_ms (nullable).  A, X read as in chfsi_autotune_batched. */
chfsi_status chfsi_autotune_batched_tiles(chfsi_handle h, int count, const chfsi_problem* probs,
                                          chfsi_tile_plan* tiles, double* batch_ms);
/* Sets the tile of each problem's (n, nev + nex) by hand (bm, bn in {32, 64}; only n, nev, nex of
 * probs are read) and selects the kernel with a tile per problem; tiles == NULL clears the table and
 * returns to the one tile of chfsi_set_batched_plan, which (with a plan) also selects that kernel. */
chfsi_status chfsi_set_batched_tiles(chfsi_handle h, int count, const chfsi_problem* probs,
                                     const chfsi_tile_plan* tiles);

/* Counters of the last chfsi_solve_batched (host pointers, each nullable): filter time in ms
 * (hipEvents around each loop's filter launches, summed), filter flops (8 n^2 per column and
 * step), graph replays and persistent kernel launches. */
chfsi_status chfsi_batched_info(chfsi_handle h, double* filter_ms, double* filter_flops,
                                int* graph_launches, int* kernel_launches);

/* Applies the Chebyshev filter of Algorithm 1 in place to Y (n x m):
 *   Y <- T_d((H - cI)/e) Y / T_d((mu1 - c)/e),  c = (a+b)/2, e = (b-a)/2,
 * by the scaled three-term recurrence, column i taking deg[i] steps (deg == NULL: deg_uniform).
 * H (n x n Hermitian) is not modified.  prec selects the arithmetic (chfsi_precision).
 * Requires mu1 < a < b.  This is the hot path exposed for tests and benchmarks. */
chfsi_status chfsi_filter(chfsi_handle h, int n, const void* H, int ldh, void* Y, int ldy, int m,
                          const int* deg, int deg_uniform, double a, double b, double mu1, int prec);

/* Allocation-free variant of chfsi_filter, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  FP64 filter with
 * one degree `deg` for every column, otherwise the operation of chfsi_filter:
 *   Y <- T_deg((H - cI)/e) Y / T_deg((mu1 - c)/e),  c = (a+b)/2, e = (b-a)/2,  mu1 < a < b.
 * H (n x n Hermitian, leading dimension ldh >= n) and Y (n x m, ldy >= n) are device pointers on
 * the current device; Y is filtered in place.  No handle: the work is enqueued on `hip_stream`
 * (NULL = the null stream) and the call returns without waiting for it; the caller synchronises.
 * The recurrence's second n x m block and the split-K partial tiles live in one fixed device array
 * of CHFSI_NOALLOC_SCRATCH_BYTES per device, owned by the library and held until the process ends;
 * the call makes no allocation of any kind.  The first call on a device looks up that array's
 * address (a caller that captures a graph makes one call before capturing, m = 0 will do).
 * Calls that overlap on one device share the array and race: serialise them (one stream).
 * Errors: CHFSI_ERR_ARG for invalid sizes, pointers or bounds; CHFSI_ERR_TOO_LARGE when
 * 16 n m > CHFSI_NOALLOC_SCRATCH_BYTES (nothing is enqueued); CHFSI_ERR_DEVICE if a launch fails. */
#define CHFSI_NOALLOC_SCRATCH_BYTES (64ull << 20)
chfsi_status chfsi_filter_noalloc(void* hip_stream, int n, const void* H, int ldh, void* Y, int ldy, int m,
                                  int deg, double a, double b, double mu1);

/* Event timing of the filter-step launches of the last chfsi_solve / chfsi_filter on this handle:
 * *total_ms = sum over launches of the time between hipEvents recorded on the handle's stream just
 * before and just after each main filter kernel (split-K reduce kernels excluded), *launches =
 * their number (host pointers). */
chfsi_status chfsi_filter_kernel_time(chfsi_handle h, double* total_ms, int* launches);

/* Per-launch log of the filter steps of the last chfsi_solve / chfsi_filter: row r is
 * rows[9 r .. 9 r + 8] = n, block width, precision, bm, bn, ksplit, split mode (0 none, 1 reduce
 * kernel, 2 fused), main kernel ms, ms including the reduce kernel.  cap = rows the host buffer
 * holds; *count = rows available (rows == NULL: only *count is set). */
chfsi_status chfsi_filter_launch_log(chfsi_handle h, double* rows, int cap, int* count);


/* Project autotuner of the filter-step kernel: times every candidate plan for the n x m filter
 * step in precision prec on scratch buffers with hipEvents, stores the fastest in the handle's
 * plan table (used by every later filter step of that precision and n whose width is at most m
 * and above the next smaller tuned width) and returns it with its time per step in ms (both
 * outputs nullable).  Allocates and frees its own scratch.  CHFSI_FP64 / CHFSI_FP32: tiles
 * bm, bn in {32, 64}, K split 1..16, either summation.  CHFSI_BF16X3 / CHFSI_BF16X6: square tiles
 * of 64, or 128 for CHFSI_BF16X3, K split 1..16, always summed in the kernel (fused = 1 for a split). */
chfsi_status chfsi_autotune_filter(chfsi_handle h, int n, int m, int prec, chfsi_tile_plan* best, double* best_ms);
/* Sets (plan != NULL) or removes (plan == NULL) the table entry for (n, m, prec) by hand; a plan
 * outside the candidates listed above is rejected with CHFSI_ERR_ARG. */
chfsi_status chfsi_set_filter_plan(chfsi_handle h, int n, int m, int prec, const chfsi_tile_plan* plan);

/* Step-level entry points (the pieces chfsi_solve is made of), for parity tests.
 *  chfsi_reduce:  L L^H = S, H = L^{-1} A L^{-H} (exactly Hermitian: the upper triangle is the
 *                 conjugate of the lower one).  H, L: n x n device outputs
 *                 (leading dimension n).  CHFSI_ERR_NOT_HPD on a non-positive pivot.
 *  chfsi_reduce_explicit: the same outputs, H formed from the explicit inverse L^{-1} (two
 *                 products that skip its zero triangle), the form chfsi_solve takes for n <= 3072;
 *                 any n.  Allocates and frees 2 n^2 complex elements of device scratch.
 *  chfsi_lanczos: k-step Lanczos with full reorthogonalisation from the stream-2 Philox vector;
 *                 theta[k] ascending Ritz values of T_k, zw[k] = |z_1j|^2, *beta_k, *k_used (host).
 *  chfsi_orthonormalize: Y (n x m) <- Q with Y = Q R, R upper triangular with real positive
 *                 diagonal, after removing components along the nl columns of YL (may be 0).
 *  chfsi_rayleigh_ritz: Y (n x m, orthonormal columns) <- Y W where Y^H H Y = W diag(theta) W^H,
 *                 theta ascending (host [m]); resid (host [m]) = ||H y_i - theta_i y_i||_2. */
chfsi_status chfsi_reduce(chfsi_handle h, int n, const void* A, int lda, const void* S, int lds,
                          void* H, void* L);
chfsi_status chfsi_reduce_explicit(chfsi_handle h, int n, const void* A, int lda, const void* S,
                                   int lds, void* H, void* L);
chfsi_status chfsi_lanczos(chfsi_handle h, int n, const void* H, int ldh, int k,
                           unsigned long long seed, double* theta, double* zw, double* beta_k,
                           int* k_used);
chfsi_status chfsi_orthonormalize(chfsi_handle h, int n, int m, void* Y, int ldy, int nl,
                                  const void* YL, int ldyl);
chfsi_status chfsi_rayleigh_ritz(chfsi_handle h, int n, const void* H, int ldh, int m, void* Y,
                                 int ldy, double* theta, double* resid);

/* Correlation of the eigenvectors of two neighbouring problems of a sequence (Section 2.2: the
 * scalar products between eigenvectors of successive problems and the angle each one turns by,
 * Fig. 1).  Xp, Xc: n x m device blocks, each S-orthonormal (S = NULL: orthonormal, standard
 * problems); S: n x n HPD device matrix or NULL.  Outputs:
 *   O (device, m x m, leading dimension ldo >= m) = Xp^H S Xc;
 *   sin_pair (host [m]): sin_pair[i] = ||xc_i - O_ii xp_i||_S / ||xc_i||_S, the sine of the angle
 *                        between xp_i and xc_i;
 *   sin_sub (host [m]): the sines of the principal angles between span(Xp) and span(Xc),
 *                       ascending: square roots of the eigenvalues of R^H S R, R = Xc - Xp O.
 * Synchronous on return.  CHFSI_ERR_NUMERIC for non-finite values or a zero column of Xc. */
chfsi_status chfsi_correlation(chfsi_handle h, int n, int m, const void* S, int lds, const void* Xp, int ldxp,
                               const void* Xc, int ldxc, void* O, int ldo, double* sin_pair, double* sin_sub);

/* Block LOBPCG without preconditioner (Knyazev 2001), the paper's second solver (Section 3.1),
 * on the library's kernels.  gen = 1 iterates on the pencil A x = lambda S x directly; gen = 0
 * first reduces it to H = L^{-1} A L^{-H} (Section 3.2) and iterates on H (Table 2 compares the
 * two).  Each iteration is a Rayleigh-Ritz step on [X, W, P] (Ritz block, residuals of its
 * unconverged columns, previous directions), the basis made S-orthonormal block by block; soft
 * locking; the iteration stops when the nev lowest pairs all meet ||A x - lambda S x|| <=
 * tol ||A||_lo (on H: ||H y - lambda y|| <= tol ||A||_lo / sqrt(||S||_inf)), ||A||_lo the largest
 * column norm of A.  Block size bs (0: ceil(1.05 nev), Table 3), at most maxiter iterations
 * (Table 3: 1000).  Random start: the library's Philox block, stream 1 (in the coordinates the
 * iteration runs in). */
typedef struct {
    int nev;                      /* wanted eigenpairs (lowest)                                  */
    int bs;                       /* block size, nev <= bs <= n; 0 = ceil(1.05 nev)              */
    int maxiter;                  /* iteration limit                                             */
    double tol;                   /* target of ||A x - lambda S x|| / ||A||_lo                    */
    int gen;                      /* 1: iterate on (A, S); 0: reduce to standard form first       */
    unsigned long long seed;      /* random start block                                          */
} chfsi_lobpcg_params;

typedef struct {
    int iters, nconv;             /* iterations taken; leading pairs converged at the end        */
    long long matvecs, bmatvecs;  /* columns multiplied by A (or H) and by S                     */
    int dropped;                  /* basis directions dropped as dependent                       */
    double t_reduce, t_iterate, t_total;   /* ms: reduction, iteration, whole call             */
    int restarts;                 /* steps taken without the previous directions P, because the  */
                                  /* eigensolver of their Gram matrix did not converge          */
} chfsi_lobpcg_stats;

/* Defaults: nev 32, bs 0, maxiter 1000, tol 1e-10, gen 0, seed 0. */
void chfsi_lobpcg_default_params(chfsi_lobpcg_params* p);

/* A (n x n Hermitian), S (n x n HPD, or NULL for a standard problem; gen is then ignored), X
 * (n x bs, ldx >= n): in = start block when x_is_guess (generalized coordinates), out = Ritz
 * vectors with unit S-norm, ascending.  lambda, resid: host [bs], Ritz values and
 * ||A x - lambda S x|| / ||A||_lo of the returned vectors.  CHFSI_ERR_NO_CONVERGENCE after maxiter
 * iterations (outputs valid, stats->nconv pairs converged); CHFSI_ERR_NOT_HPD, CHFSI_ERR_NUMERIC
 * (non-finite values, or the start block is rank deficient) as for chfsi_solve.  Synchronous. */
chfsi_status chfsi_lobpcg(chfsi_handle h, int n, const void* A, int lda, const void* S, int lds, void* X, int ldx,
                          int x_is_guess, double* lambda, double* resid, const chfsi_lobpcg_params* p,
                          chfsi_lobpcg_stats* stats);

/* Fills Y (n x m, device) with the library's random block: element e = i + j n of stream `stream`
 * is Philox4x64-10 (Salmon et al., SC'11) of counter (e/2, stream, 0, 0) and key (seed, 0); the
 * parity of e selects words (0,1) or (2,3); each word w gives a part 2 (w >> 11) 2^-53 - 1 in
 * [-1, 1).  Stream 1 is the cold-start block of chfsi_solve, stream 2 the Lanczos start vector. */
chfsi_status chfsi_random_block(chfsi_handle h, unsigned long long seed, unsigned long long stream, int n, int m,
                                void* Y, int ldy);

/* Dense complex product C = alpha op(A) op(B) + beta C (op: 'N' or 'C' = conjugate transpose),
 * op(A) m x k, op(B) k x n, real alpha and beta, device pointers.  The MFMA kernel the filter and
 * the Rayleigh-Ritz step use. */
chfsi_status chfsi_zgemm(chfsi_handle h, char transa, char transb, int m, int n, int k,
                         double alpha, const void* A, int lda, const void* B, int ldb,
                         double beta, void* C, int ldc);

/* Degree network (learned per-vector degree).  A blob is the float32 parameter vector of the
 * 5 -> 64 -> 64 -> 64 -> 1 network (8769 values, layout W1[64][5] b1 W2[64][64] b2 W3[64][64] b3
 * W4[1][64] b4) followed by 10 float32 feature normalisation constants (mean[5], std[5]).
 * NULL clears the model; CHFSI_ERR_ARG if nbytes does not match. */
chfsi_status chfsi_set_degree_model(chfsi_handle h, const void* blob, size_t nbytes);

/* Copies the trace recorded by the last solve with p->trace = 1 into host_buf.  One row per active
 * column and loop, CHFSI_TRACE_COLS doubles: loop, column position, t = (theta - c)/e, log10 r
 * (residual after this loop), (a - mu1)/(b - mu1), (b - mu1)/(|mu1| + |b|) (with the bounds of the
 * next filter), degree used in this loop, degree assigned for the next loop, r_after (the residual
 * at the same position after the next loop; -1 if none), lock threshold.  These are the network's
 * features (t, log10 r / threshold, the two bound ratios, previous degree) and its label data.
 * With host_buf NULL only *nbytes is set. */
#define CHFSI_TRACE_COLS 10
chfsi_status chfsi_get_trace(chfsi_handle h, void* host_buf, size_t* nbytes);

/* Degree-network kernels (FP32, device pointers), used by training and by the gradient checks.
 *  forward:   out[N] = dmin + (dmax - dmin) sigmoid(net(X[N][5]))
 *  loss_grad: grad[8769] and *loss (host) of mean((out - y)^2)
 *  adam:      one bias-corrected Adam step on P with moments m, v (all [8769]), step t >= 1
 *  train:     epochs of shuffled minibatch Adam on (X, y); the shuffle uses Philox keyed by seed;
 *             loss_hist (host, nullable) receives the mean loss of each epoch. */
chfsi_status chfsi_mlp_forward(chfsi_handle h, const float* P, int N, const float* X, float dmin,
                               float dmax, float* out);
chfsi_status chfsi_mlp_loss_grad(chfsi_handle h, const float* P, int N, const float* X,
                                 const float* y, float dmin, float dmax, float* grad, float* loss);
chfsi_status chfsi_mlp_adam(chfsi_handle h, float* P, const float* grad, float* m, float* v, int t,
                            float lr, float beta1, float beta2, float eps);
chfsi_status chfsi_mlp_train(chfsi_handle h, float* P, int N, const float* X, const float* y,
                             float dmin, float dmax, int epochs, int batch, float lr,
                             unsigned long long seed, float* loss_hist);

/* Human-readable name of a status code (static storage). */
const char* chfsi_status_string(chfsi_status s);

#ifdef __cplusplus
}
#endif
#endif /* CHFSI_H */
