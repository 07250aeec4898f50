// Per-problem state of one solve of Algorithm 1, split into phases that first enqueue device work
// and then complete on the host after one stream synchronisation.  A single solve runs the phases
// back to back on the handle's stream; the batched solver interleaves them over many problems
// (each bound to one of several streams) and filters all problems together.
#pragma once
#include <chrono>
#include <vector>

#include "chfsi.h"
#include "common.h"
#include "driver.h"

struct SolveBufs {
    zd *H = nullptr, *L = nullptr;     // n x n (H aliases A for a standard FP64 problem)
    zf* Hf = nullptr;                  // n x n complex64 copy of H (low-precision filter)
    uint16_t* Hb = nullptr;            // BF16 planes of H
    zd *V = nullptr, *T = nullptr, *HY = nullptr;   // n x m
    zf *Vf = nullptr, *Tf = nullptr;   // n x m complex64
    uint16_t* ysplit = nullptr;        // BF16 split of Y_k
    zd *G = nullptr, *Cm = nullptr;    // m x m
    zd *dinvL = nullptr, *dinvG = nullptr;   // inverted 64 x 64 diagonal blocks of L (n) and of the Gram factor (m)
    zd* hwork = nullptr;               // panel operands of the reduction to standard form (n x 192)
    double *theta = nullptr, *r = nullptr, *E = nullptr, *lam = nullptr, *dsc = nullptr;
    int* info = nullptr;
    int* flag = nullptr;
    int* iperm = nullptr;
    zd *LV = nullptr, *lw = nullptr, *lc = nullptr;
    double* lcoef = nullptr;
    float* feat = nullptr;
    float* dpred = nullptr;
    void* eigw = nullptr;              // workspace of the Rayleigh-quotient eigensolver
    GemmWs gw;                         // split-K partials + the handle's tile counters
};

// device buffers of a solve of order n, block m, k Lanczos steps, carved from `ar` (grown when
// needed); the arena of the handle for single solves, one arena per problem for batched solves
// (reduce_ws: the panel operands of the reduction, which generalized problems always get)
chfsi_status prepare_bufs(chfsi_handle h, Arena& ar, SolveBufs& b, int n, int m, int k, bool gen, int prec,
                          bool reduce_ws = false);

struct TraceRow { int loop, col; double t, lr, a, b; int d_prev, d; double r_after, thr; };

struct SolveState {
    // problem and parameters
    int n = 0, nev = 0, m = 0, k = 0, prec = 0;
    const zd* A = nullptr;
    int lda = 0;
    const zd* S = nullptr;
    int lds = 0;
    zd* X = nullptr;
    int ldx = 0, x_is_guess = 0;
    double* lambda = nullptr;          // caller's host arrays [m]
    double* resid = nullptr;
    chfsi_params p;
    // resources
    SolveBufs b;
    PhaseTimer* tm = nullptr;          // phase events (single solves)
    double* hd = nullptr;              // pinned host doubles, see the accessors below
    int* hi = nullptr;                 // pinned host ints, see h_perm / h_flags
    bool permuted = false;             // the active columns are in the filter's degree order
    bool fc_store = false;             // the factor of this solve's S goes to the handle's cache
    bool fc_reused = false;            // the cached factor was reused
    // algorithm state
    const zd* H = nullptr;
    int ldh = 0;
    double norm_a = 0, thr = 0, bb = 0, mu1 = 0, a = 0, sw_thr = 0;
    std::vector<int> deg, lowp, deg_used, last_row;
    std::vector<double> rprev;
    std::vector<TraceRow> trace;
    int nlocked = 0, loops = 0, switches = 0;
    int hy_off = -1;                   // b.HY columns hy_off.. = H times the active block, or -1
    long long matvecs = 0, filtered = 0;
    double flops = 0;
    chfsi_status status = CHFSI_ERR_NO_CONVERGENCE;
    bool done = false, finalized = false, want_final = false;
    std::chrono::steady_clock::time_point t0;

    double* h_theta() { return hd; }               // [m]
    double* h_r() { return hd + m; }               // [m]
    double* h_norms() { return hd + 2 * m; }       // [2]: ||A||_lo estimate, ||S||_inf
    double* h_al() { return hd + 2 * m + 2; }      // [k]
    double* h_be() { return hd + 2 * m + 2 + k; }  // [k]
    double* h_lam() { return hd + 2 * m + 2 + 2 * k; }       // [m]
    double* h_res() { return hd + 3 * m + 2 + 2 * k; }       // [m]
    double* h_eig() { return hd + 4 * m + 2 + 2 * k; }       // [eig_host_doubles(m)]
    static size_t pinned_doubles(int m, int k) { return 4 * (size_t)m + 2 + 2 * (size_t)k + eig_host_doubles(m); }
    // pinned ints: info words [0, 16); the filter's column order and its inverse [32, 32 + 2 m);
    // the odd-degree flags of the batched filter [32 + 2 m, 32 + 3 m).  The two staging regions are
    // disjoint: the host writes the flags of a loop while the copy of that loop's column order may
    // still be pending on another stream.
    int* h_perm() { return hi + 32; }
    int* h_flags() { return hi + 32 + 2 * (size_t)m; }
    static size_t pinned_ints(int m) { return 32 + 3 * (size_t)m; }
    int ma() const { return m - nlocked; }
    zd* Ya() { return b.V + (size_t)nlocked * n; }
};

// Validates the arguments and fills s (no device work).
chfsi_status st_define(SolveState& s, int n, const zd* A, int lda, const zd* S, int lds, zd* X, int ldx,
                       int x_is_guess, double* lambda, double* resid, const chfsi_params& p);
// Device buffers (arena `ar`) and pinned staging (`pin`).
chfsi_status st_setup(chfsi_handle h, SolveState& s, Arena& ar, PinBuf& pin);
// Reduction to standard form, norms, starting block, Lanczos.
chfsi_status st_init_enqueue(chfsi_handle h, SolveState& s);
// Cholesky check, Lanczos bounds, the per-column degree and precision vectors.
chfsi_status st_init_complete(chfsi_handle h, SolveState& s);
// Filter of the active block (single-problem path, any precision).
chfsi_status st_filter(chfsi_handle h, SolveState& s);
// Orthonormalisation and Rayleigh-Ritz of the active block; Ritz values, residuals and info words
// are copied to pinned memory.
chfsi_status st_loop_enqueue(chfsi_handle h, SolveState& s);
// Locking, bounds and degrees for the next loop; sets want_final once nev pairs are locked.
chfsi_status st_loop_complete(chfsi_handle h, SolveState& s);
// Back-transform and residual verification of all m pairs.
chfsi_status st_final_enqueue(chfsi_handle h, SolveState& s);
// Convergence decision of the verification: done, or the failing suffix is unlocked again.
chfsi_status st_final_complete(chfsi_handle h, SolveState& s);
// Finalises an unconverged solve and fills the counters of stt (phase times excluded).
void st_finish(chfsi_handle h, SolveState& s, chfsi_stats& stt);
// Reorders the active columns by non-increasing degree (FP64 filter, batched path); dsorted
// receives the reordered degrees.
chfsi_status st_order_columns(chfsi_handle h, SolveState& s, std::vector<int>& dsorted);

// the whole solve on the handle's stream
chfsi_status solve_impl(chfsi_handle h, int n, const zd* A, int lda, const zd* S, int lds, zd* X, int ldx,
                        int x_is_guess, double* lambda, double* resid, const chfsi_params& p, chfsi_stats& stt);
