// Host driver of the ChFSI library: the C ABI of include/chfsi.h.
//
// The solver follows Algorithm 1 (Chebyshev filtered subspace iteration with locking) inside the
// reduction of Section 3.2:
//   reduction      S = L L^H, H = L^{-1} A L^{-H}          (own blocked Cholesky, Hermitian two-sided solve)
//   Lanczos        k steps, full reorthogonalisation      (own kernels; k x k eig on the host)
//   loop           filter -> orthonormalise -> Rayleigh-Ritz -> residuals -> lock prefix
//   back-transform X = L^{-H} Y and ||A x - lambda S x|| / ||A||_lo verification
// Every matrix operation runs on the handle's stream; the host synchronises once per loop to read
// the m_a Ritz values and residual norms it needs for the locking decision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "chfsi.h"
#include "driver.h"

int chfsi_internal_hip_error(hipError_t e) { return (int)e; }

// ---------------------------------------------------------------------------------------------
// handle, workspace and timers
// ---------------------------------------------------------------------------------------------

void Arena::grow(size_t bytes)
{
    if (bytes <= cap) return;
    if (base) (void)hipFree(base);
    base = nullptr;
    cap = 0;
    if (hipMalloc((void**)&base, bytes) != hipSuccess) { base = nullptr; return; }
    cap = bytes;
}

bool PinBuf::reserve(size_t bytes)
{
    if (bytes <= cap) return true;
    release();
    if (hipHostMalloc((void**)&p, bytes, hipHostMallocDefault) != hipSuccess) { p = nullptr; return false; }
    cap = bytes;
    return true;
}

void PinBuf::release()
{
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
}

void* Arena::get(size_t bytes)
{
    size_t b = (bytes + 255) & ~(size_t)255;
    if (measuring) { off += b; return (void*)(uintptr_t)256; }
    if (!base || off + b > cap) { failed = true; return nullptr; }
    void* p = base + off;
    off += b;
    return p;
}

PhaseTimer::~PhaseTimer()
{
    for (auto& e : pool) (void)hipEventDestroy(e);
}

void PhaseTimer::mark(int phase, hipStream_t s, bool begin)
{
    if (used == pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        pool.push_back(e);
    }
    hipEvent_t e = pool[used++];
    (void)hipEventRecord(e, s);
    if (begin) open[phase] = e;
    else if (open[phase]) { spans.push_back({phase, open[phase], e}); open[phase] = nullptr; }
}

void PhaseTimer::collect(double* out /* [NPHASE] ms */)
{
    for (int i = 0; i < NPHASE; ++i) out[i] = 0;
    for (auto& sp : spans) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, sp.b, sp.e) == hipSuccess) out[sp.phase] += ms;
    }
    spans.clear();
    used = 0;
    for (int i = 0; i < NPHASE; ++i) open[i] = nullptr;
}

KernelTimer::~KernelTimer()
{
    for (auto& e : pool) (void)hipEventDestroy(e);
}

void KernelTimer::begin(int n, int ncols, int prec, GemmWs& gs)
{
    gs.ev_start = gs.ev_main = gs.ev_end = nullptr;
    gs.plan_used = nullptr;
    if (!enabled) return;
    while (pool.size() < used + 3) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { enabled = false; return; }
        pool.push_back(e);
    }
    const size_t r = used / 3;
    if (recs.size() <= r) recs.resize(r + 1);
    recs[r] = Rec{n, ncols, prec, {0, 0, 0, 0}};
    gs.plan_used = recs[r].plan;
    gs.ev_start = pool[used];
    gs.ev_main = pool[used + 1];
    gs.ev_end = pool[used + 2];
}

void KernelTimer::end(const GemmWs& gs)
{
    if (gs.ev_start) used += 3;
}

double KernelTimer::collect(int* launches, double* step_ms)
{
    double t = 0, ts = 0;
    log.clear();
    for (size_t i = 0; i + 3 <= used; i += 3) {
        float m1 = 0, m2 = 0;
        (void)hipEventElapsedTime(&m1, pool[i], pool[i + 1]);
        (void)hipEventElapsedTime(&m2, pool[i], pool[i + 2]);
        t += m1;
        ts += m2;
        const Rec& r = recs[i / 3];
        const double row[9] = {(double)r.n, (double)r.ncols, (double)r.prec, (double)r.plan[0], (double)r.plan[1],
                               (double)r.plan[2], (double)r.plan[3], (double)m1, (double)m2};
        log.insert(log.end(), row, row + 9);
    }
    if (launches) *launches = (int)(used / 3);
    if (step_ms) *step_ms = ts;
    used = 0;
    return t;
}

const char* chfsi_status_string(chfsi_status s)
{
    switch (s) {
    case CHFSI_SUCCESS: return "success";
    case CHFSI_ERR_ARG: return "invalid argument";
    case CHFSI_ERR_NOT_HPD: return "S is not Hermitian positive definite";
    case CHFSI_ERR_NO_CONVERGENCE: return "no convergence within max_loops";
    case CHFSI_ERR_NUMERIC: return "non-finite values or breakdown";
    case CHFSI_ERR_DEVICE: return "HIP runtime error";
    case CHFSI_ERR_ALLOC: return "allocation failed";
    case CHFSI_ERR_TOO_LARGE: return "input exceeds the fixed scratch of the allocation-free filter";
    }
    return "unknown status";
}

void chfsi_default_params(chfsi_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->nev = 0;
    p->nex = 40;            // Table 3: blk = nev + 40
    p->deg = 25;            // Table 3: degree 25
    p->tol = 1e-10;         // Table 3: TOL 1e-10
    p->max_loops = 50;
    p->lanczos_steps = 25;  // within Table 3's "10 .. 3 blk"
    p->filter_precision = CHFSI_FP64;
    p->degree_policy = CHFSI_DEG_FIXED;
    p->deg_min = 4;
    p->deg_max = 30;
    p->seed = 0;
    p->have_bounds = 0;
    p->trace = 0;
    p->switch_residual = 0.0;
    p->deg_margin = 0;
}

chfsi_status chfsi_create(chfsi_handle* out, int device, void* hip_stream)
{
    if (!out) return CHFSI_ERR_ARG;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return CHFSI_ERR_DEVICE;
    chfsi_handle h = new (std::nothrow) chfsi_handle_s();
    if (!h) return CHFSI_ERR_ALLOC;
    h->device = device;
    h->stream = (hipStream_t)hip_stream;
    h->tile_cnt_len = 1 << 18;
    if (hipMalloc((void**)&h->tile_cnt, sizeof(int) * h->tile_cnt_len) != hipSuccess) {
        delete h;
        return CHFSI_ERR_ALLOC;
    }
    if (hipMemsetAsync(h->tile_cnt, 0, sizeof(int) * h->tile_cnt_len, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
        (void)hipFree(h->tile_cnt);
        delete h;
        return CHFSI_ERR_DEVICE;
    }
    *out = h;
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_destroy(chfsi_handle h)
{
    if (!h) return CHFSI_ERR_ARG;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    for (auto& l : h->lanes) (void)hipStreamSynchronize(l.st);
    if (h->ws.base) (void)hipFree(h->ws.base);
    if (h->lob.base) (void)hipFree(h->lob.base);
    if (h->fc.base) (void)hipFree(h->fc.base);
    for (auto& a : h->barena)
        if (a.base) (void)hipFree(a.base);
    h->pin.release();
    for (auto& pb : h->bpin) pb.release();
    h->btable_host.release();
    for (auto& g : h->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    if (h->btable) (void)hipFree(h->btable);
    for (auto& l : h->lanes) {
        if (l.sub) {
            if (l.sub->tile_cnt) (void)hipFree(l.sub->tile_cnt);
            l.sub->model = nullptr;   // the parent's
            delete l.sub;
        }
        if (l.ev) (void)hipEventDestroy(l.ev);
        if (l.st) (void)hipStreamDestroy(l.st);
    }
    for (auto& e : h->bev)
        if (e) (void)hipEventDestroy(e);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->model) (void)hipFree(h->model);
    if (h->tile_cnt) (void)hipFree(h->tile_cnt);
    delete h;
    return CHFSI_SUCCESS;
}

// ---------------------------------------------------------------------------------------------
// host-side small eigenproblem: symmetric tridiagonal T_k of Lanczos, cyclic Jacobi (k <= 3m).
// ---------------------------------------------------------------------------------------------

void host_tridiag_eig(int k, const double* al, const double* be, std::vector<double>& theta,
                      std::vector<double>& z1sq)
{
    std::vector<double> T((size_t)k * k, 0.0), V((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) {
        T[i + (size_t)i * k] = al[i];
        V[i + (size_t)i * k] = 1.0;
        if (i + 1 < k) { T[i + 1 + (size_t)i * k] = be[i]; T[i + (size_t)(i + 1) * k] = be[i]; }
    }
    double fro = 0;
    for (double v : T) fro += v * v;
    fro = std::sqrt(fro);
    for (int sweep = 0; sweep < 100; ++sweep) {
        bool any = false;
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                const double apq = T[p + (size_t)q * k];
                if (!(std::fabs(apq) > 1e-16 * fro)) continue;
                any = true;
                const double app = T[p + (size_t)p * k], aqq = T[q + (size_t)q * k];
                const double th = (aqq - app) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int i = 0; i < k; ++i) {   // columns p, q
                    const double x = T[i + (size_t)p * k], y = T[i + (size_t)q * k];
                    T[i + (size_t)p * k] = c * x - s * y;
                    T[i + (size_t)q * k] = s * x + c * y;
                    const double vx = V[i + (size_t)p * k], vy = V[i + (size_t)q * k];
                    V[i + (size_t)p * k] = c * vx - s * vy;
                    V[i + (size_t)q * k] = s * vx + c * vy;
                }
                for (int i = 0; i < k; ++i) {   // rows p, q
                    const double x = T[p + (size_t)i * k], y = T[q + (size_t)i * k];
                    T[p + (size_t)i * k] = c * x - s * y;
                    T[q + (size_t)i * k] = s * x + c * y;
                }
                T[p + (size_t)q * k] = 0.0;
                T[q + (size_t)p * k] = 0.0;
            }
        if (!any) break;
    }
    std::vector<int> ord(k);
    for (int i = 0; i < k; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return T[a + (size_t)a * k] < T[b + (size_t)b * k]; });
    theta.resize(k);
    z1sq.resize(k);
    for (int j = 0; j < k; ++j) {
        theta[j] = T[ord[j] + (size_t)ord[j] * k];
        const double z = V[0 + (size_t)ord[j] * k];
        z1sq[j] = z * z;
    }
}

// ---------------------------------------------------------------------------------------------
// steps of the method on device buffers
// ---------------------------------------------------------------------------------------------


#define TRY(x)                                              \
    do {                                                    \
        int rc_ = (int)(x);                                 \
        if (rc_ != 0) return CHFSI_ERR_DEVICE;              \
    } while (0)

// S = L L^H (L lower, strict upper part zeroed, dinv the inverses of its 64 x 64 diagonal blocks);
// the Cholesky info word is copied to *info_host (valid after the stream has been synchronised).
chfsi_status step_factor_enqueue(chfsi_handle h, int n, const zd* S, int lds, zd* L, zd* dinv, int* info_dev,
                                 int* info_host, const GemmWs& gw)
{
    hipStream_t st = h->stream;
    TRY(launch_zlacpy(st, n, n, S, lds, L, n));
    TRY(hipMemsetAsync(info_dev, 0, sizeof(int), st));
    TRY(chol_lower(st, n, L, n, info_dev, dinv, gw));
    TRY(hipMemcpyAsync(info_host, info_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    TRY(launch_zero_upper(st, n, L, n));
    return CHFSI_SUCCESS;
}

// S = L L^H (L lower, strict upper part zeroed), H = L^{-1} A L^{-H}, Hermitized.  Enqueues the
// whole reduction; the Cholesky info word is copied to *info_host (host memory, valid after the
// stream has been synchronised; nonzero = S not positive definite, H then meaningless).
chfsi_status step_reduce_enqueue(chfsi_handle h, int n, const zd* A, int lda, const zd* S, int lds, zd* H, zd* L,
                                 zd* dinv, zd* hwork, int* info_dev, int* info_host, const GemmWs& gw)
{
    hipStream_t st = h->stream;
    const chfsi_status fs = step_factor_enqueue(h, n, S, lds, L, dinv, info_dev, info_host, gw);
    if (fs != CHFSI_SUCCESS) return fs;
    TRY(launch_zlacpy(st, n, n, A, lda, H, n));
    TRY(hegst_lower(st, n, H, n, L, n, dinv, hwork, gw));        // H = L^{-1} A L^{-H}, lower triangles only
    return CHFSI_SUCCESS;
}

chfsi_status step_reduce(chfsi_handle h, int n, const zd* A, int lda, const zd* S, int lds, zd* H, zd* L, zd* dinv,
                         zd* hwork, int* info_dev, const GemmWs& gw)
{
    int info = 0;
    chfsi_status s = step_reduce_enqueue(h, n, A, lda, S, lds, H, L, dinv, hwork, info_dev, &info, gw);
    if (s != CHFSI_SUCCESS) return s;
    TRY(hipStreamSynchronize(h->stream));
    return info != 0 ? CHFSI_ERR_NOT_HPD : CHFSI_SUCCESS;
}

// k-step Lanczos with full reorthogonalisation (two classical Gram-Schmidt passes per step).
// Enqueues the k steps and the copies of alpha_1..k, beta_1..k to hal/hbe (host, valid after the
// stream has been synchronised).
chfsi_status step_lanczos_enqueue(chfsi_handle h, int n, const zd* H, int ldh, int k, unsigned long long seed,
                                  zd* LV, zd* w, zd* c, double* coef_dev, double* hal, double* hbe)
{
    hipStream_t st = h->stream;
    double* al = coef_dev;             // [k]
    double* be = coef_dev + k;         // [k]
    double* scr = coef_dev + 2 * k;    // [8] scratch: normalisation of v_1, complex products
    TRY(launch_philox_block(st, seed, 2, n, 1, LV, n));
    TRY(launch_lanczos_normalize(st, n, LV, LV, scr));
    for (int j = 0; j < k; ++j) {
        zd* vj = LV + (size_t)j * n;
        TRY(launch_coldots(st, n, n, H, ldh, vj, w));           // w = H v_j (H Hermitian)
        TRY(launch_lanczos_alpha(st, n, vj, w, j > 0 ? vj - n : nullptr, al + j, j > 0 ? be + j - 1 : nullptr,
                                 (zd*)(scr + 2)));
        for (int pass = 0; pass < 2; ++pass) {
            TRY(launch_coldots(st, n, j + 1, LV, n, w, c));
            TRY(launch_gemv_n(st, n, j + 1, LV, n, c, -1.0, w));
        }
        TRY(launch_lanczos_normalize(st, n, w, LV + (size_t)(j + 1) * n, be + j));
    }
    TRY(hipMemcpyAsync(hal, al, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(hbe, be, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    return CHFSI_SUCCESS;
}

// Host part of Lanczos: the tridiagonal T_k (cut at the first vanishing beta) and its
// eigen-decomposition: Ritz values theta and squared first components z1sq of the eigenvectors.
chfsi_status lanczos_finish(int k, const double* hal, const double* hbe, std::vector<double>& theta,
                            std::vector<double>& z1sq, double& beta_k, int& k_used)
{
    int kk = k;
    for (int j = 0; j < k; ++j)
        if (!(hbe[j] > 1e-300)) { kk = j + 1; break; }
    for (int j = 0; j < kk; ++j)
        if (!std::isfinite(hal[j]) || !std::isfinite(hbe[j])) return CHFSI_ERR_NUMERIC;
    host_tridiag_eig(kk, hal, hbe, theta, z1sq);
    beta_k = hbe[kk - 1];
    k_used = kk;
    return CHFSI_SUCCESS;
}

chfsi_status step_lanczos(chfsi_handle h, int n, const zd* H, int ldh, int k, unsigned long long seed, zd* LV,
                          zd* w, zd* c, double* coef_dev, std::vector<double>& theta, std::vector<double>& z1sq,
                          double& beta_k, int& k_used)
{
    std::vector<double> hal(k), hbe(k);
    chfsi_status s = step_lanczos_enqueue(h, n, H, ldh, k, seed, LV, w, c, coef_dev, hal.data(), hbe.data());
    if (s != CHFSI_SUCCESS) return s;
    TRY(hipStreamSynchronize(h->stream));
    return lanczos_finish(k, hal.data(), hbe.data(), theta, z1sq, beta_k, k_used);
}

// Y (n x ma) <- orthonormal basis: CGS twice against the nl locked columns YL, then shifted
// Cholesky QR followed by two Cholesky QR passes (shift s = 11 (n m + m (m+1)) u ||Y||_F^2 after
// column normalisation; Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, SISC 2020).  R's
// diagonal is real positive in every pass, so Q is the Q factor of Y.
// With host_tmp (host memory, one double) the first Gram matrix decides: when its largest
// off-diagonal row sum is below 1/2, Gershgorin bounds kappa(Y) by sqrt(3) and plain Cholesky QR
// twice (no shift) is already accurate to rounding, so the shifted pass is left out (one host
// synchronisation instead of one Cholesky QR pass).  With T (device, n x ma scratch) as well, the
// last pass is a first-order correction when its Gram matrix is the identity to 1e-9 (below).
chfsi_status step_orthonormalize(chfsi_handle h, int n, int ma, zd* Y, int ldy, int nl, const zd* YL, int ldyl,
                                 zd* G, zd* Cm, zd* dinv, double* dsc, int* info_dev, const GemmWs& gw,
                                 double* host_tmp, zd* T)
{
    hipStream_t st = h->stream;
    if (ma <= 0) return CHFSI_SUCCESS;
    if (nl > 0)
        for (int pass = 0; pass < 2; ++pass) {
            TRY(launch_zgemm(st, OP_C, OP_N, nl, ma, n, 1.0, YL, ldyl, Y, ldy, 0.0, Cm, nl, gw));
            TRY(launch_zgemm(st, OP_N, OP_N, n, ma, nl, -1.0, YL, ldyl, Cm, nl, 1.0, Y, ldy, gw));
        }
    TRY(launch_colnorms(st, n, ma, Y, ldy, dsc));
    TRY(launch_scale_cols_inv(st, n, ma, Y, ldy, dsc));
    const double u = 1.1102230246251565e-16;
    const double shift = 11.0 * ((double)n * ma + (double)ma * (ma + 1)) * u * (double)ma;
    bool shifted = true;
    for (int pass = 0; pass < (shifted ? 3 : 2); ++pass) {
        TRY(launch_zgemm(st, OP_C, OP_N, ma, ma, n, 1.0, Y, ldy, Y, ldy, 0.0, G, ma, gw));
        if (pass == 0 && host_tmp) {
            TRY(launch_max_rowsum_abs(st, ma, G, ma, dsc));
            TRY(hipMemcpyAsync(host_tmp, dsc, sizeof(double), hipMemcpyDeviceToHost, st));
            TRY(hipStreamSynchronize(st));
            shifted = !(host_tmp[0] - 1.0 < 0.5);
        }
        if (pass == 0 && shifted) TRY(launch_add_diag_const(st, ma, G, ma, shift));
        // The last pass starts from a block orthonormal to working accuracy: G = I + E with E
        // of the order of the previous pass's rounding.  Then R = I + F + O(|E|^2), F the strict
        // upper triangle of E plus half its diagonal, and Y <- Y (I - F) is orthonormal to
        // O(|E|^2): one product instead of a factorisation and a triangular solve, taken when
        // max_i sum_j |E_ij| <= 1e-9 (checked on the host).
        const bool last = pass == (shifted ? 2 : 1);
        if (last && pass > 0 && T && host_tmp) {
            TRY(launch_max_rowsum_off_identity(st, ma, G, ma, dsc));
            TRY(hipMemcpyAsync(host_tmp, dsc, sizeof(double), hipMemcpyDeviceToHost, st));
            TRY(hipStreamSynchronize(st));
            if (host_tmp[0] <= 1e-9) {
                TRY(launch_first_order_factor(st, ma, G, ma));
                TRY(launch_zlacpy(st, n, ma, Y, ldy, T, n));
                TRY(launch_zgemm(st, OP_N, OP_N, n, ma, ma, -1.0, T, n, G, ma, 1.0, Y, ldy, gw));
                continue;
            }
        }
        // G = L L^H = R^H R with R = L^H; Y <- Y R^{-1} = Y L^{-H}
        TRY(chol_lower(st, ma, G, ma, info_dev + pass, dinv, gw));
        TRY(trsm_right_lower_h(st, n, ma, G, ma, dinv, Y, ldy, gw));
    }
    return CHFSI_SUCCESS;
}

// Rayleigh-Ritz on orthonormal Y (n x ma): HY = H Y, G = Y^H HY, G = W diag(theta) W^H (ascending,
// phase-normalised W, block-Jacobi eigensolver of eig.hip), Y <- Y W, HY <- HY W, then
// r_j = ||HY_j - theta_j Y_j||.  eig_work: eig_work_bytes(ma) bytes of device memory; eig_host:
// eig_host_doubles(ma) doubles of host memory; eig_stop: see eig_jacobi.
chfsi_status step_rayleigh_ritz(chfsi_handle h, int n, const zd* H, int ldh, int ma, zd* Y, int ldy, zd* HY,
                                zd* T, zd* G, double* theta_dev, double* r_dev, void* eig_work, double* eig_host,
                                const GemmWs& gw, PhaseTimer* tm, double eig_stop)
{
    hipStream_t st = h->stream;
    {   // H Y has the shape of a filter step: the filter's tuned plan
        GemmWs g2 = gw;
        apply_tuned_plan(h, CHFSI_FP64, n, ma, g2);
        TRY(launch_zgemm(st, OP_N, OP_N, n, ma, n, 1.0, H, ldh, Y, ldy, 0.0, HY, n, g2));
    }
    TRY(launch_zgemm(st, OP_C, OP_N, ma, ma, n, 1.0, Y, ldy, HY, n, 0.0, G, ma, gw));
    int sweeps = 0;
    const int rc = eig_jacobi(st, ma, G, ma, theta_dev, eig_work, eig_host, &sweeps, eig_stop);
    if (rc == -1) return CHFSI_ERR_NUMERIC;
    TRY(rc);
    TRY(launch_phase_normalize(st, ma, ma, G, ma));
    TRY(launch_zgemm(st, OP_N, OP_N, n, ma, ma, 1.0, Y, ldy, G, ma, 0.0, T, n, gw));
    TRY(launch_zlacpy(st, n, ma, T, n, Y, ldy));
    TRY(launch_zgemm(st, OP_N, OP_N, n, ma, ma, 1.0, HY, n, G, ma, 0.0, T, n, gw));
    TRY(launch_zlacpy(st, n, ma, T, n, HY, n));
    if (tm) tm->mark(PH_RESID, st, true);
    TRY(launch_residual_norms(st, n, ma, HY, n, Y, ldy, theta_dev, r_dev));
    if (tm) tm->mark(PH_RESID, st, false);
    return CHFSI_SUCCESS;
}

// ---------------------------------------------------------------------------------------------
// the Chebyshev filter
// ---------------------------------------------------------------------------------------------

// Scaled recurrence coefficients: step 1 has alpha = sigma_1/e, beta = 0; step k+1 (k >= 1) has
// sigma_{k+1} = 1/(2/sigma_1 - sigma_k), alpha = 2 sigma_{k+1}/e, beta = -sigma_k sigma_{k+1}.
// Step k (0-based) on its own: sigma carries sigma_k from the previous call (ignored for k = 0).
FilterStep filter_step_coefficients(int k, double a, double b, double mu1, double& sigma)
{
    const double c = 0.5 * (a + b), e = 0.5 * (b - a);
    const double sigma1 = e / (mu1 - c);
    FilterStep fs;
    fs.shift = c;
    if (k == 0) {
        fs.alpha = sigma1 / e;
        fs.beta = 0.0;
        sigma = sigma1;
    } else {
        const double sn = 1.0 / (2.0 / sigma1 - sigma);
        fs.alpha = 2.0 * sn / e;
        fs.beta = -sigma * sn;
        sigma = sn;
    }
    return fs;
}

void filter_coefficients(int dmax, double a, double b, double mu1, std::vector<FilterStep>& steps)
{
    steps.resize(dmax);
    double sigma = 0;
    for (int k = 0; k < dmax; ++k) steps[k] = filter_step_coefficients(k, a, b, mu1, sigma);
}

// Filters the ma columns of Y whose degrees deg[] are sorted in non-increasing order.  T is a
// second n x ma buffer.  Step k (1-based) updates the first #{j : deg[j] >= k} columns; columns
// finishing on an odd step are copied back from T at the end (flag buffer on device).
template <typename C2, typename HT>
chfsi_status filter_sorted(chfsi_handle h, int n, const HT* Hm, int ldh, int ma, C2* Y, int ldy, C2* T, int ldt,
                           const std::vector<int>& deg, double a, double b, double mu1, int* flag_dev,
                           const GemmWs& gw, double& flops, long long& matvecs,
                           int (*step_fn)(hipStream_t, int, int, const HT*, int, const C2*, int, const C2*, int,
                                          C2*, int, FilterStep, const GemmWs&),
                           int (*copy_fn)(hipStream_t, int, int, const C2*, int, C2*, int, const int*), const zd* hy0)
{
    hipStream_t st = h->stream;
    if (ma <= 0) return CHFSI_SUCCESS;
    const int dmax = deg[0];
    if (dmax <= 0) return CHFSI_SUCCESS;
    std::vector<FilterStep> steps;
    filter_coefficients(dmax, a, b, mu1, steps);
    for (int k = 1; k <= dmax; ++k) {
        int w = 0;
        while (w < ma && deg[w] >= k) ++w;
        // Y_k lives in Y when k is even, in T when k is odd; Y_{k-1} in the other one
        const C2* yk = (k % 2 == 1) ? Y : T;        // input Y_{k-1}
        const int ldk = (k % 2 == 1) ? ldy : ldt;
        C2* yo = (k % 2 == 1) ? T : Y;              // output Y_k overwrites Y_{k-2}
        const int ldo = (k % 2 == 1) ? ldt : ldy;
        const C2* yp = (k == 1) ? yk : yo;          // beta == 0 on step 1: any finite input
        const int ldp = (k == 1) ? ldk : ldo;
        if (k == 1 && hy0) {   // H Y_0 known (hy0, ld n): step 1 without a product
            TRY(launch_first_step(st, n, w, steps[0].alpha, steps[0].shift, hy0, n, yk, ldk, yo, ldo));
            matvecs += w;        // the degree count; filter_flops counts the products performed
            continue;
        }
        GemmWs gs = gw;
        const int pr = sizeof(C2) == 16 ? CHFSI_FP64 : CHFSI_FP32;
        apply_tuned_plan(h, pr, n, w, gs);
        h->ktimer.begin(n, w, pr, gs);
        TRY(step_fn(st, n, w, Hm, ldh, yk, ldk, yp, ldp, yo, ldo, steps[k - 1], gs));
        h->ktimer.end(gs);
        flops += 8.0 * (double)n * (double)n * (double)w;
        matvecs += w;
    }
    // columns with an odd degree finished in T
    std::vector<int> odd(ma);
    bool any = false;
    for (int j = 0; j < ma; ++j) { odd[j] = deg[j] % 2; any |= odd[j] != 0; }
    if (any) {
        TRY(hipMemcpyAsync(flag_dev, odd.data(), sizeof(int) * ma, hipMemcpyHostToDevice, st));
        TRY(copy_fn(st, n, ma, T, ldt, Y, ldy, flag_dev));
        // the host vector must stay alive until the copy has been consumed
        TRY(hipStreamSynchronize(st));
    }
    return CHFSI_SUCCESS;
}

static int step_f64(hipStream_t s, int n, int w, const zd* H, int ldh, const zd* yk, int ldk, const zd* yp, int ldp,
                    zd* yo, int ldo, FilterStep fs, const GemmWs& gw)
{
    return launch_filter_step_f64(s, n, w, H, ldh, yk, ldk, yp, ldp, yo, ldo, fs, gw);
}
static int step_f32(hipStream_t s, int n, int w, const zf* H, int ldh, const zf* yk, int ldk, const zf* yp, int ldp,
                    zf* yo, int ldo, FilterStep fs, const GemmWs& gw)
{
    return launch_filter_step_f32(s, n, w, H, ldh, yk, ldk, yp, ldp, yo, ldo, fs, gw);
}

chfsi_status filter_f64(chfsi_handle h, int n, const zd* H, int ldh, int ma, zd* Y, int ldy, zd* T,
                        const std::vector<int>& deg, double a, double b, double mu1, int* flag_dev, const GemmWs& gw,
                        double& flops, long long& matvecs, const zd* hy0)
{
    return filter_sorted<zd, zd>(h, n, H, ldh, ma, Y, ldy, T, n, deg, a, b, mu1, flag_dev, gw, flops, matvecs,
                                 step_f64, launch_copy_cols_flag, hy0);
}

chfsi_status filter_f32(chfsi_handle h, int n, const zf* Hf, int ldh, int ma, zf* Yf, int ldy, zf* Tf,
                        const std::vector<int>& deg, double a, double b, double mu1, int* flag_dev, const GemmWs& gw,
                        double& flops, long long& matvecs, const zd* hy0)
{
    return filter_sorted<zf, zf>(h, n, Hf, ldh, ma, Yf, ldy, Tf, n, deg, a, b, mu1, flag_dev, gw, flops,
                                 matvecs, step_f32, launch_copy_cols_flag_c, hy0);
}
