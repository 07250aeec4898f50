// C ABI entry points of include/chfsi.h: the whole solver (Algorithm 1 inside the reduction of
// Section 3.2), the filter alone, the step-level entry points and the dense product.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "chfsi.h"
#include "common.h"
#include "driver.h"

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

struct SolveBufs {
    zd *H = nullptr, *L = nullptr;     // n x n (H aliases A for a standard FP64 problem)
    zf* Hf = nullptr;                  // n x n complex64 copy of H (low-precision filter)
    uint16_t* Hb = nullptr;            // BF16 planes of H
    zd *V = nullptr, *T = nullptr, *HY = nullptr;   // n x m
    zf *Vf = nullptr, *Tf = nullptr;   // n x m complex64
    uint16_t* ysplit = nullptr;        // BF16 split of Y_k
    zd *G = nullptr, *Cm = nullptr;    // m x m
    double *theta = nullptr, *r = nullptr, *E = nullptr, *lam = nullptr, *dsc = nullptr;
    int* info = nullptr;
    int* flag = nullptr;
    int* iperm = nullptr;
    zd *LV = nullptr, *lw = nullptr, *lc = nullptr;
    double* lcoef = nullptr;
    float* feat = nullptr;
    float* dpred = nullptr;
    GemmWs gw;                         // split-K partials + the handle's tile counters
};

void layout(Arena& ar, SolveBufs& b, int n, int m, int k, bool gen, int prec)
{
    const size_t nn = (size_t)n * n, nm = (size_t)n * m, mm = (size_t)m * m;
    if (gen) {
        b.H = ar.take<zd>(nn);
        b.L = ar.take<zd>(nn);
    }
    if (prec == CHFSI_FP32) b.Hf = ar.take<zf>(nn);
    if (prec == CHFSI_BF16X3 || prec == CHFSI_BF16X6) {
        const int nterms = prec == CHFSI_BF16X3 ? 2 : 3;
        b.Hb = ar.take<uint16_t>(bf16_hplanes_elems(n, nterms));
        b.ysplit = (uint16_t*)ar.get(bf16_ysplit_bytes(n, m, nterms));
    }
    b.V = ar.take<zd>(nm);
    b.T = ar.take<zd>(nm);
    b.HY = ar.take<zd>(nm);
    if (prec != CHFSI_FP64) {
        b.Vf = ar.take<zf>(nm);
        b.Tf = ar.take<zf>(nm);
    }
    b.G = ar.take<zd>(mm);
    b.Cm = ar.take<zd>(mm);
    b.theta = ar.take<double>(m);
    b.r = ar.take<double>(m);
    b.E = ar.take<double>(m + 8);
    b.lam = ar.take<double>(m);
    b.dsc = ar.take<double>((size_t)std::max(n, m) + 16);
    b.info = ar.take<int>(16);
    b.flag = ar.take<int>(m + 8);
    b.iperm = ar.take<int>(m + 8);
    b.LV = ar.take<zd>((size_t)n * (k + 1));
    b.lw = ar.take<zd>(n);
    b.lc = ar.take<zd>(k + 1);
    b.lcoef = ar.take<double>(2 * (size_t)k + 16);
    b.feat = ar.take<float>((size_t)m * MLP_NF + 16);
    b.dpred = ar.take<float>(m + 16);
    // split-K partials: the largest of the filter (n x m, K = n) and the Gram products (m x m, K = n)
    size_t ws = std::max(zgemm_ws_bytes(n, m, n, 16), zgemm_ws_bytes(m, m, n, 16));
    ws = std::max(ws, zgemm_ws_bytes(n, m, m, 16));
    b.gw.bytes = ws;
    b.gw.ws = ar.get(ws);
}

chfsi_status prepare(chfsi_handle h, SolveBufs& b, int n, int m, int k, bool gen, int prec)
{
    h->ws.begin(true);
    layout(h->ws, b, n, m, k, gen, prec);
    const size_t need = h->ws.off;
    if (need > h->ws.cap) {
        (void)hipStreamSynchronize(h->stream);
        h->ws.grow(need + (need >> 3));
        if (h->ws.cap < need) return CHFSI_ERR_ALLOC;
    }
    h->ws.begin(false);
    b = SolveBufs();
    layout(h->ws, b, n, m, k, gen, prec);
    b.gw.cnt = h->tile_cnt;
    b.gw.ncnt = h->tile_cnt_len;
    return h->ws.failed ? CHFSI_ERR_ALLOC : CHFSI_SUCCESS;
}

// uniform degree in [dmin, dmax] from Philox4x64-10, counter (loop, column, 4, 0), key (seed, 0)
int random_degree(unsigned long long seed, int loop, int col, int dmin, int dmax)
{
    uint64_t c[4] = {(uint64_t)loop, (uint64_t)col, 4, 0};
    uint64_t k0 = seed, k1 = 0;
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B97F4A7C15ULL; k1 += 0xBB67AE8584CAA73BULL; }
        const unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * c[0];
        const unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * c[2];
        const uint64_t y0 = (uint64_t)(p1 >> 64) ^ c[1] ^ k0, y2 = (uint64_t)(p0 >> 64) ^ c[3] ^ k1;
        c[1] = (uint64_t)p1;
        c[3] = (uint64_t)p0;
        c[0] = y0;
        c[2] = y2;
    }
    return dmin + (int)(c[0] % (uint64_t)(dmax - dmin + 1));
}

int analytic_degree(double theta, double r, double a, double b, double thr, int dmin, int dmax)
{
    const double c = 0.5 * (a + b), e = 0.5 * (b - a);
    const double t = (theta - c) / e;
    if (!(std::fabs(t) > 1.0) || !std::isfinite(r)) return dmax;
    if (!(r > thr)) return dmin;
    const double rho = std::fabs(t) + std::sqrt(t * t - 1.0);
    double d = std::ceil(std::log(r / thr) / std::log(rho));
    return (int)std::min<double>(dmax, std::max<double>(dmin, d));
}

// Filters the active block Y (n x ma) with per-column degrees deg and precision flags lowp
// (1 = low precision).  Columns are reordered: low-precision group first, each group sorted by
// non-increasing degree; the reordering is harmless because QR and Rayleigh-Ritz follow.
chfsi_status run_filter(chfsi_handle h, SolveBufs& b, int n, const zd* H, int ldh, int prec, int ma, zd* Y, int ldy,
                        std::vector<int>& deg, std::vector<int>& lowp, double a, double bb, double mu1,
                        double& flops, long long& matvecs)
{
    hipStream_t st = h->stream;
    std::vector<int> ord(ma);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
        if (lowp[x] != lowp[y]) return lowp[x] > lowp[y];
        return deg[x] > deg[y];
    });
    bool ident = true;
    for (int j = 0; j < ma; ++j) ident &= ord[j] == j;
    if (!ident) {
        TRY(hipMemcpyAsync(b.iperm, ord.data(), sizeof(int) * ma, hipMemcpyHostToDevice, st));
        TRY(launch_permute_cols(st, n, ma, Y, ldy, b.T, n, b.iperm));
        TRY(launch_zlacpy(st, n, ma, b.T, n, Y, ldy));
        std::vector<int> d2(ma), l2(ma);
        for (int j = 0; j < ma; ++j) { d2[j] = deg[ord[j]]; l2[j] = lowp[ord[j]]; }
        deg.swap(d2);
        lowp.swap(l2);
        TRY(hipStreamSynchronize(st));   // ord must outlive the async copy
    }
    int nlow = 0;
    while (nlow < ma && lowp[nlow]) ++nlow;
    if (nlow > 0 && prec != CHFSI_FP64) {
        std::vector<int> dl(deg.begin(), deg.begin() + nlow);
        TRY(launch_z2c(st, n, nlow, Y, ldy, b.Vf, n));
        if (prec == CHFSI_FP32) {
            TRYS(filter_f32(h, n, b.Hf, n, nlow, b.Vf, n, b.Tf, dl, a, bb, mu1, b.flag, b.gw,
                            flops, matvecs));
        } else {
            const int nterms = prec == CHFSI_BF16X3 ? 2 : 3;
            TRYS(filter_bf16(h, n, b.Hb, n, nterms, nlow, b.Vf, n, b.Tf, b.ysplit, dl, a, bb, mu1, b.flag,
                             b.gw, flops, matvecs));
        }
        TRY(launch_c2z(st, n, nlow, b.Vf, n, Y, ldy));
    }
    const int n64 = (prec == CHFSI_FP64) ? ma : ma - nlow;
    const int off = ma - n64;
    if (n64 > 0) {
        std::vector<int> dh(deg.begin() + off, deg.end());
        TRYS(filter_f64(h, n, H, ldh, n64, Y + (size_t)off * ldy, ldy, b.T, dh, a, bb, mu1, b.flag, b.gw, flops, matvecs));
    }
    return CHFSI_SUCCESS;
}

// X = L^{-H} V (or V), rho_j = ||A x_j - lambda_j S x_j|| / norm_a for all m columns
chfsi_status finalize(chfsi_handle h, SolveBufs& b, int n, int m, const zd* A, int lda, const zd* S, int lds,
                      zd* X, int ldx, const double* lambda, double norm_a, double* resid)
{
    hipStream_t st = h->stream;
    TRY(launch_zlacpy(st, n, m, b.V, n, X, ldx));
    if (S) {
        const rocblas_double_complex one(1.0, 0.0);
        if (rocblas_ztrsm(h->rb, rocblas_side_left, rocblas_fill_lower, rocblas_operation_conjugate_transpose,
                          rocblas_diagonal_non_unit, n, m, &one, reinterpret_cast<rocblas_double_complex*>(b.L), n,
                          reinterpret_cast<rocblas_double_complex*>(X), ldx) != rocblas_status_success)
            return CHFSI_ERR_DEVICE;
    }
    TRY(launch_zgemm(st, OP_N, OP_N, n, m, n, 1.0, A, lda, X, ldx, 0.0, b.HY, n, b.gw));
    const zd* SX = X;
    int ldsx = ldx;
    if (S) {
        TRY(launch_zgemm(st, OP_N, OP_N, n, m, n, 1.0, S, lds, X, ldx, 0.0, b.T, n, b.gw));
        SX = b.T;
        ldsx = n;
    }
    TRY(hipMemcpyAsync(b.lam, lambda, sizeof(double) * m, hipMemcpyHostToDevice, st));
    TRY(launch_residual_norms(st, n, m, b.HY, n, SX, ldsx, b.lam, b.r));
    TRY(hipMemcpyAsync(resid, b.r, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    for (int j = 0; j < m; ++j) resid[j] /= norm_a;
    return CHFSI_SUCCESS;
}

struct TraceRow { int loop, col; double t, lr, a, b; int d_prev, d; double r_after, thr; };

chfsi_status solve_impl(chfsi_handle h, int n, const zd* A, int lda, const zd* S, int lds, zd* X, int ldx,
                        int x_is_guess, double* lambda, double* resid, const chfsi_params& p, chfsi_stats& stt)
{
    hipStream_t st = h->stream;
    const int nev = p.nev, m = p.nev + p.nex;
    const int prec = p.filter_precision;
    if (n <= 0 || nev <= 0 || p.nex < 0 || m > n || lda < n || ldx < n || (S && lds < n) || !A || !X || !lambda ||
        !resid || p.deg < 0 || !(p.tol > 0) || p.max_loops < 1 || prec < 0 || prec > 3 || p.deg_min < 0 ||
        p.deg_max < p.deg_min || p.degree_policy < 0 || p.degree_policy > 3)
        return CHFSI_ERR_ARG;
    if (p.degree_policy == CHFSI_DEG_LEARNED && !h->has_model) return CHFSI_ERR_ARG;
    int k = p.lanczos_steps;
    k = std::max(k, 10);
    k = std::min(k, 3 * m);
    k = std::min(k, n);

    SolveBufs b;
    const bool gen = S != nullptr;
    TRYS(prepare(h, b, n, m, k, gen, prec));
    PhaseTimer& tm = h->timer;
    {
        double reset[NPHASE];
        tm.collect(reset);
        (void)h->ktimer.collect(nullptr);
    }
    auto t0 = std::chrono::steady_clock::now();
    tm.mark(PH_TOTAL, st, true);

    // --- reduction to standard form (Section 3.2)
    tm.mark(PH_REDUCE, st, true);
    const zd* H = A;
    int ldh = lda;
    if (S) {
        TRYS(step_reduce(h, n, A, lda, S, lds, b.H, b.L, b.info));
        H = b.H;
        ldh = n;
    }
    TRY(launch_max_colnorm(st, n, A, lda, b.dsc));
    double hs[2] = {0, 1};
    TRY(hipMemcpyAsync(&hs[0], b.dsc, sizeof(double), hipMemcpyDeviceToHost, st));
    if (S) {
        TRY(launch_max_rowsum_abs(st, n, S, lds, b.dsc));
        TRY(hipMemcpyAsync(&hs[1], b.dsc, sizeof(double), hipMemcpyDeviceToHost, st));
    }
    if (prec == CHFSI_FP32) TRY(launch_z2c(st, n, n, H, ldh, b.Hf, n));
    if (prec == CHFSI_BF16X3 || prec == CHFSI_BF16X6)
        TRY(launch_split_h_bf16(st, n, H, ldh, b.Hb, n, prec == CHFSI_BF16X3 ? 2 : 3));
    // starting block in standard coordinates
    if (x_is_guess) {
        if (S) TRY(launch_zgemm(st, OP_C, OP_N, n, m, n, 1.0, b.L, n, X, ldx, 0.0, b.V, n, b.gw));
        else TRY(launch_zlacpy(st, n, m, X, ldx, b.V, n));
    } else {
        TRY(launch_philox_block(st, p.seed, 1, n, m, b.V, n));
    }
    TRY(hipStreamSynchronize(st));
    tm.mark(PH_REDUCE, st, false);
    const double norm_a = hs[0], s_inf = hs[1];
    if (!std::isfinite(norm_a) || !std::isfinite(s_inf) || !(norm_a > 0)) return CHFSI_ERR_NUMERIC;
    const double thr = p.tol * norm_a / std::sqrt(s_inf);
    stt.norm_a = norm_a;

    // --- Lanczos bounds
    tm.mark(PH_LANCZOS, st, true);
    std::vector<double> lth, lz;
    double beta_k = 0;
    int kk = 0;
    TRYS(step_lanczos(h, n, H, ldh, k, p.seed, b.LV, b.lw, b.lc, b.lcoef, lth, lz, beta_k, kk));
    tm.mark(PH_LANCZOS, st, false);
    stt.lanczos_steps = kk;
    double bb = lth[kk - 1] + beta_k, mu1 = lth[0], a = lth[kk - 1];
    {
        const double frac = (double)m / n;
        double cum = 0;
        for (int j = 0; j < kk; ++j) {
            cum += lz[j];
            if (cum >= frac) { a = lth[j]; break; }
        }
        if (!(a > mu1) || !(a < bb)) a = 0.5 * (mu1 + bb);
    }
    if (p.have_bounds) {
        mu1 = p.mu1;
        a = p.a;
        if (!(a > mu1) || !(a < bb)) a = 0.5 * (mu1 + bb);
    }

    // --- inner loop of Algorithm 1
    std::vector<int> deg(m, p.deg), lowp(m, prec != CHFSI_FP64 ? 1 : 0);
    std::vector<int> deg_used(m, p.deg);
    std::vector<double> hth(m), hr(m), rprev(m, -1.0), rho(m);
    std::vector<int> last_row(m, -1);
    std::vector<TraceRow> trace;
    int nlocked = 0, loops = 0;
    chfsi_status status = CHFSI_ERR_NO_CONVERGENCE;
    double flops = 0;
    long long matvecs = 0, filtered = 0;
    int switches = 0;
    double sw_rel = p.switch_residual > 0 ? p.switch_residual
                    : (prec == CHFSI_BF16X3 ? 1e-3 : 1e-5);
    const double sw_thr = sw_rel * norm_a;

    for (int it = 0; it < p.max_loops; ++it) {
        const int ma = m - nlocked;
        zd* Ya = b.V + (size_t)nlocked * n;
        loops = it + 1;
        filtered += ma;

        tm.mark(PH_FILTER, st, true);
        std::vector<int> dact(deg.begin() + nlocked, deg.end()), lact(lowp.begin() + nlocked, lowp.end());
        TRYS(run_filter(h, b, n, H, ldh, prec, ma, Ya, n, dact, lact, a, bb, mu1, flops, matvecs));
        tm.mark(PH_FILTER, st, false);

        tm.mark(PH_QR, st, true);
        TRY(hipMemsetAsync(b.info, 0, sizeof(int) * 8, st));
        TRYS(step_orthonormalize(h, n, ma, Ya, n, nlocked, b.V, n, b.G, b.Cm, b.dsc, b.info, b.gw));
        tm.mark(PH_QR, st, false);

        tm.mark(PH_RR, st, true);
        TRYS(step_rayleigh_ritz(h, n, H, ldh, ma, Ya, n, b.HY, b.T, b.G, b.theta, b.E, b.r, b.info + 4, b.gw, &tm));
        tm.mark(PH_RR, st, false);

        tm.mark(PH_LOCK, st, true);
        int hinfo[8];
        TRY(hipMemcpyAsync(hth.data(), b.theta, sizeof(double) * ma, hipMemcpyDeviceToHost, st));
        TRY(hipMemcpyAsync(hr.data(), b.r, sizeof(double) * ma, hipMemcpyDeviceToHost, st));
        TRY(hipMemcpyAsync(hinfo, b.info, sizeof(int) * 8, hipMemcpyDeviceToHost, st));
        TRY(hipStreamSynchronize(st));
        for (int j = 0; j < 8; ++j)
            if (hinfo[j] != 0) { status = CHFSI_ERR_NUMERIC; break; }
        for (int j = 0; j < ma; ++j)
            if (!std::isfinite(hth[j]) || !std::isfinite(hr[j])) status = CHFSI_ERR_NUMERIC;
        if (status == CHFSI_ERR_NUMERIC) { tm.mark(PH_LOCK, st, false); break; }

        for (int j = 0; j < ma; ++j) deg_used[nlocked + j] = deg[nlocked + j];   // degrees of this loop
        // trace: close the rows of the previous loop, open rows for this one
        if (p.trace) {
            for (int j = 0; j < ma; ++j) {
                const int pos = nlocked + j;
                if (last_row[pos] >= 0) trace[last_row[pos]].r_after = hr[j];
            }
        }
        int cnt = 0;
        while (cnt < nev - nlocked && hr[cnt] <= thr) ++cnt;
        for (int j = 0; j < ma; ++j) { lambda[nlocked + j] = hth[j]; resid[nlocked + j] = hr[j]; }

        // bounds for the next filter
        const double a_new = hth[ma - 1];
        const double mu1_new = std::min(mu1, hth[0]);
        // per-column degree and precision for the next loop (absolute positions)
        const int nl2 = nlocked + cnt;
        for (int j = cnt; j < ma; ++j) {
            const int pos = nlocked + j;
            if (lowp[pos]) {
                const bool stagnated = rprev[pos] > 0 && hr[j] > 0.1 * rprev[pos];
                if (hr[j] <= sw_thr || stagnated) { lowp[pos] = 0; ++switches; }
            }
        }
        a = a_new;
        mu1 = mu1_new;
        if (!(a > mu1)) a = 0.5 * (mu1 + bb);
        if (p.degree_policy == CHFSI_DEG_ANALYTIC) {
            for (int j = cnt; j < ma; ++j)
                deg[nlocked + j] = analytic_degree(hth[j], hr[j], a, bb, thr, p.deg_min, p.deg_max);
        } else if (p.degree_policy == CHFSI_DEG_RANDOM) {
            for (int j = cnt; j < ma; ++j)
                deg[nlocked + j] = random_degree(p.seed, it, nlocked + j, p.deg_min, p.deg_max);
        } else if (p.degree_policy == CHFSI_DEG_LEARNED) {
            TRYS(learned_degrees(h, ma - cnt, b.theta + cnt, b.r + cnt, a, bb, mu1, thr,
                                 std::vector<int>(deg.begin() + nl2, deg.end()), b.feat, b.dpred, b.iperm,
                                 p.deg_min, p.deg_max, deg.data() + nl2,
                                 [&](int j) { return analytic_degree(hth[cnt + j], hr[cnt + j], a, bb, thr,
                                                                     p.deg_min, p.deg_max); }));
        }
        if (p.trace) {
            const double c2 = 0.5 * (a + bb), e2 = 0.5 * (bb - a);
            for (int j = cnt; j < ma; ++j) {
                const int pos = nlocked + j;
                TraceRow row;
                row.loop = it; row.col = pos; row.t = (hth[j] - c2) / e2;
                row.lr = std::log10(std::max(hr[j], 1e-300)); row.a = (a - mu1) / (bb - mu1);
                row.b = (bb - mu1) / (std::fabs(mu1) + std::fabs(bb)); row.d_prev = deg_used[pos];
                row.d = deg[pos]; row.r_after = -1.0;
                row.thr = thr;
                last_row[pos] = (int)trace.size();
                trace.push_back(row);
            }
        }
        for (int j = 0; j < ma; ++j) rprev[nlocked + j] = hr[j];
        nlocked = nl2;
        tm.mark(PH_LOCK, st, false);

        if (nlocked >= nev) {
            tm.mark(PH_BACK, st, true);
            TRYS(finalize(h, b, n, m, A, lda, S, lds, X, ldx, lambda, norm_a, resid));
            tm.mark(PH_BACK, st, false);
            int bad = -1;
            for (int j = 0; j < nev; ++j)
                if (!(resid[j] <= p.tol)) { bad = j; break; }
            if (bad < 0) { status = CHFSI_SUCCESS; break; }
            nlocked = bad;
            for (int j = bad; j < m; ++j) deg[j] = p.deg;
        }
    }
    if (status == CHFSI_ERR_NO_CONVERGENCE) {
        tm.mark(PH_BACK, st, true);
        TRYS(finalize(h, b, n, m, A, lda, S, lds, X, ldx, lambda, norm_a, resid));
        tm.mark(PH_BACK, st, false);
    }
    tm.mark(PH_TOTAL, st, false);
    TRY(hipStreamSynchronize(st));
    double ph[NPHASE];
    tm.collect(ph);
    stt.t_reduce = ph[PH_REDUCE]; stt.t_lanczos = ph[PH_LANCZOS]; stt.t_filter = ph[PH_FILTER];
    stt.t_qr = ph[PH_QR]; stt.t_rr = ph[PH_RR]; stt.t_resid = ph[PH_RESID]; stt.t_lock = ph[PH_LOCK];
    stt.t_back = ph[PH_BACK];
    stt.t_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    stt.loops = loops;
    stt.nlocked = std::min(nlocked, nev);
    stt.filtered_vectors = filtered;
    stt.matvecs = matvecs;
    stt.filter_flops = flops;
    stt.mu1 = mu1; stt.a = a; stt.b = bb;
    stt.precision_switches = switches;
    stt.t_filter_kernels = h->ktimer.collect(&stt.filter_launches, &stt.t_filter_steps);
    h->last_kernel_ms = stt.t_filter_kernels;
    h->last_kernel_launches = stt.filter_launches;
    stt.status = status;
    if (p.trace) {
        h->trace.clear();
        for (auto& r : trace) {
            const double row[CHFSI_TRACE_COLS] = {(double)r.loop, (double)r.col, r.t, r.lr, r.a, r.b,
                                                  (double)r.d_prev, (double)r.d, r.r_after, r.thr};
            h->trace.insert(h->trace.end(), row, row + CHFSI_TRACE_COLS);
        }
    }
    return status;
}

}  // namespace

extern "C" {

chfsi_status chfsi_solve(chfsi_handle h, int n, const void* A, int lda, const void* S, int lds, void* X, int ldx,
                         int x_is_guess, double* lambda, double* resid, const chfsi_params* p, chfsi_stats* stats)
{
    if (!h) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    chfsi_params prm;
    if (p) prm = *p; else chfsi_default_params(&prm);
    chfsi_stats stt;
    std::memset(&stt, 0, sizeof(stt));
    chfsi_status s = solve_impl(h, n, (const zd*)A, lda, (const zd*)S, lds, (zd*)X, ldx, x_is_guess, lambda, resid,
                                prm, stt);
    stt.status = s;
    if (stats) *stats = stt;
    return s;
}

chfsi_status chfsi_solve_batched(chfsi_handle h, int count, const chfsi_problem* probs, const chfsi_params* p,
                                 chfsi_stats* stats)
{
    if (!h || count < 0 || (count > 0 && !probs)) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    chfsi_params base;
    if (p) base = *p; else chfsi_default_params(&base);
    chfsi_status first = CHFSI_SUCCESS;
    for (int k = 0; k < count; ++k) {
        const chfsi_problem& q = probs[k];
        chfsi_params pk = base;
        pk.nev = q.nev;
        pk.nex = q.nex;
        chfsi_stats stt;
        std::memset(&stt, 0, sizeof(stt));
        chfsi_status s = solve_impl(h, q.n, (const zd*)q.A, q.lda, (const zd*)q.S, q.lds, (zd*)q.X, q.ldx,
                                    q.x_is_guess, q.lambda, q.resid, pk, stt);
        stt.status = s;
        if (stats) stats[k] = stt;
        if (s != CHFSI_SUCCESS && first == CHFSI_SUCCESS) first = s;
    }
    return first;
}

chfsi_status chfsi_filter(chfsi_handle h, int n, const void* Hv, int ldh, void* Yv, int ldy, int m, const int* deg,
                          int deg_uniform, double a, double b, double mu1, int prec)
{
    if (!h || !Hv || !Yv || n <= 0 || m < 0 || ldh < n || ldy < n || prec < 0 || prec > 3) return CHFSI_ERR_ARG;
    if (!(mu1 < a) || !(a < b)) return CHFSI_ERR_ARG;
    if (m == 0) return CHFSI_SUCCESS;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    std::vector<int> d(m, deg_uniform);
    if (deg) for (int j = 0; j < m; ++j) d[j] = deg[j];
    for (int j = 0; j < m; ++j) if (d[j] < 0) return CHFSI_ERR_ARG;
    SolveBufs bf;
    TRYS(prepare(h, bf, n, m, 10, false, prec));
    hipStream_t st = h->stream;
    const zd* H = (const zd*)Hv;
    zd* Y = (zd*)Yv;
    if (prec == CHFSI_FP32) TRY(launch_z2c(st, n, n, H, ldh, bf.Hf, n));
    if (prec == CHFSI_BF16X3 || prec == CHFSI_BF16X6)
        TRY(launch_split_h_bf16(st, n, H, ldh, bf.Hb, n, prec == CHFSI_BF16X3 ? 2 : 3));
    (void)h->ktimer.collect(nullptr);
    // the filter permutes columns by degree; undo that here so the caller sees its own order
    std::vector<int> ord(m);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] > d[y]; });
    std::vector<int> lowp(m, prec != CHFSI_FP64 ? 1 : 0), dd = d;
    double flops = 0;
    long long mv = 0;
    TRY(launch_zlacpy(st, n, m, Y, ldy, bf.V, n));
    TRYS(run_filter(h, bf, n, H, ldh, prec, m, bf.V, n, dd, lowp, a, b, mu1, flops, mv));
    // bf.V column j now holds input column ord[j]
    std::vector<int> inv(m);
    for (int j = 0; j < m; ++j) inv[ord[j]] = j;
    TRY(hipMemcpyAsync(bf.iperm, inv.data(), sizeof(int) * m, hipMemcpyHostToDevice, st));
    TRY(launch_permute_cols(st, n, m, bf.V, n, Y, ldy, bf.iperm));
    TRY(hipStreamSynchronize(st));
    h->last_kernel_ms = h->ktimer.collect(&h->last_kernel_launches);
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_filter_launch_log(chfsi_handle h, double* rows, int cap, int* count)
{
    if (!h || !count || cap < 0) return CHFSI_ERR_ARG;
    const int avail = (int)(h->ktimer.log.size() / 9);
    *count = avail;
    if (rows) std::memcpy(rows, h->ktimer.log.data(), sizeof(double) * 9 * std::min(avail, cap));
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_filter_kernel_time(chfsi_handle h, double* total_ms, int* launches)
{
    if (!h || !total_ms || !launches) return CHFSI_ERR_ARG;
    *total_ms = h->last_kernel_ms;
    *launches = h->last_kernel_launches;
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_reduce(chfsi_handle h, int n, const void* A, int lda, const void* S, int lds, void* H, void* L)
{
    if (!h || !A || !S || !H || !L || n <= 0 || lda < n || lds < n) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    SolveBufs b;
    TRYS(prepare(h, b, 1, 1, 1, false, CHFSI_FP64));
    TRYS(step_reduce(h, n, (const zd*)A, lda, (const zd*)S, lds, (zd*)H, (zd*)L, b.info));
    TRY(hipStreamSynchronize(h->stream));
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_lanczos(chfsi_handle h, int n, const void* H, int ldh, int k, unsigned long long seed,
                           double* theta, double* zw, double* beta_k, int* k_used)
{
    if (!h || !H || n <= 0 || ldh < n || k < 1 || k > n || !theta || !zw || !beta_k || !k_used) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    SolveBufs b;
    TRYS(prepare(h, b, n, 1, k, false, CHFSI_FP64));
    std::vector<double> th, z;
    double bk = 0;
    int kk = 0;
    TRYS(step_lanczos(h, n, (const zd*)H, ldh, k, seed, b.LV, b.lw, b.lc, b.lcoef, th, z, bk, kk));
    for (int j = 0; j < kk; ++j) { theta[j] = th[j]; zw[j] = z[j]; }
    *beta_k = bk;
    *k_used = kk;
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_orthonormalize(chfsi_handle h, int n, int m, void* Y, int ldy, int nl, const void* YL, int ldyl)
{
    if (!h || !Y || n <= 0 || m <= 0 || m > n || ldy < n || nl < 0 || (nl > 0 && (!YL || ldyl < n)) || nl + m > n)
        return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    SolveBufs b;
    const int mm = std::max(m, nl);
    TRYS(prepare(h, b, n, mm, 1, false, CHFSI_FP64));
    TRY(hipMemsetAsync(b.info, 0, sizeof(int) * 8, h->stream));
    TRYS(step_orthonormalize(h, n, m, (zd*)Y, ldy, nl, (const zd*)YL, ldyl, b.G, b.Cm, b.dsc, b.info, b.gw));
    int hinfo[3];
    TRY(hipMemcpyAsync(hinfo, b.info, sizeof(hinfo), hipMemcpyDeviceToHost, h->stream));
    TRY(hipStreamSynchronize(h->stream));
    for (int j = 0; j < 3; ++j) if (hinfo[j]) return CHFSI_ERR_NUMERIC;
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_rayleigh_ritz(chfsi_handle h, int n, const void* H, int ldh, int m, void* Y, int ldy,
                                 double* theta, double* resid)
{
    if (!h || !H || !Y || n <= 0 || m <= 0 || m > n || ldh < n || ldy < n || !theta || !resid) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    SolveBufs b;
    TRYS(prepare(h, b, n, m, 1, false, CHFSI_FP64));
    TRY(hipMemsetAsync(b.info, 0, sizeof(int) * 8, h->stream));
    TRYS(step_rayleigh_ritz(h, n, (const zd*)H, ldh, m, (zd*)Y, ldy, b.HY, b.T, b.G, b.theta, b.E, b.r, b.info,
                            b.gw, nullptr));
    int info = 0;
    TRY(hipMemcpyAsync(theta, b.theta, sizeof(double) * m, hipMemcpyDeviceToHost, h->stream));
    TRY(hipMemcpyAsync(resid, b.r, sizeof(double) * m, hipMemcpyDeviceToHost, h->stream));
    TRY(hipMemcpyAsync(&info, b.info, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    TRY(hipStreamSynchronize(h->stream));
    return info ? CHFSI_ERR_NUMERIC : CHFSI_SUCCESS;
}

chfsi_status chfsi_zgemm(chfsi_handle h, char transa, char transb, int m, int n, int k, double alpha, const void* A,
                         int lda, const void* B, int ldb, double beta, void* C, int ldc)
{
    if (!h || (transa != 'N' && transa != 'C') || (transb != 'N' && transb != 'C') || m < 0 || n < 0 || k < 0 ||
        !C || ldc < std::max(1, m))
        return CHFSI_ERR_ARG;
    const int ra = transa == 'N' ? m : k, rb = transb == 'N' ? k : n;
    if ((k > 0 && (!A || !B)) || lda < std::max(1, ra) || ldb < std::max(1, rb)) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    const size_t need = zgemm_ws_bytes(m, n, k, 16) + 256;
    h->ws.begin(true);
    (void)h->ws.get(need);
    if (h->ws.off > h->ws.cap) {
        (void)hipStreamSynchronize(h->stream);
        h->ws.grow(h->ws.off);
        if (h->ws.cap < h->ws.off) return CHFSI_ERR_ALLOC;
    }
    h->ws.begin(false);
    GemmWs gw;
    gw.ws = h->ws.get(need);
    gw.bytes = need;
    gw.cnt = h->tile_cnt;
    gw.ncnt = h->tile_cnt_len;
    TRY(launch_zgemm(h->stream, transa == 'N' ? OP_N : OP_C, transb == 'N' ? OP_N : OP_C, m, n, k, alpha,
                     (const zd*)A, lda, (const zd*)B, ldb, beta, (zd*)C, ldc, gw));
    TRY(hipStreamSynchronize(h->stream));
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_random_block(chfsi_handle h, unsigned long long seed, unsigned long long stream, int n, int m,
                                void* Y, int ldy)
{
    if (!h || !Y || n <= 0 || m < 0 || ldy < n) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    TRY(launch_philox_block(h->stream, seed, stream, n, m, (zd*)Y, ldy));
    TRY(hipStreamSynchronize(h->stream));
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_get_trace(chfsi_handle h, void* host_buf, size_t* nbytes)
{
    if (!h || !nbytes) return CHFSI_ERR_ARG;
    const size_t need = h->trace.size() * sizeof(double);
    if (!host_buf) { *nbytes = need; return CHFSI_SUCCESS; }
    if (*nbytes < need) { *nbytes = need; return CHFSI_ERR_ARG; }
    std::memcpy(host_buf, h->trace.data(), need);
    *nbytes = need;
    return CHFSI_SUCCESS;
}

}  // extern "C"
