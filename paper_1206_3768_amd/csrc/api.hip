// C ABI entry points of include/chfsi.h: the whole solver (Algorithm 1 inside the reduction of
// Section 3.2), the filter alone, the step-level entry points and the dense product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
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

void layout(Arena& ar, SolveBufs& b, int n, int m, int k, bool gen, int prec, int filter_ksplit, bool reduce_ws)
{
    const size_t nn = (size_t)n * n, nm = (size_t)n * m, mm = (size_t)m * m;
    if (gen) {
        b.H = ar.take<zd>(nn);
        b.L = ar.take<zd>(nn);
    }
    if (gen || reduce_ws) b.hwork = ar.take<zd>(hegst_work_elems(n));
    b.dinvL = ar.take<zd>(tri_dinv_elems(n));
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
    b.dinvG = ar.take<zd>(tri_dinv_elems(m));
    b.theta = ar.take<double>(m);
    b.r = ar.take<double>(m);
    b.E = ar.take<double>(m + 8);
    b.lam = ar.take<double>(m);
    b.dsc = ar.take<double>(2 * ((size_t)std::max(n, m) + 16));   // two independent scratch halves
    b.info = ar.take<int>(16);
    b.flag = ar.take<int>(m + 8);
    b.iperm = ar.take<int>(2 * (size_t)m + 16);   // a column order and its inverse
    b.LV = ar.take<zd>((size_t)n * (k + 1));
    b.lw = ar.take<zd>(n);
    b.lc = ar.take<zd>(k + 1);
    b.lcoef = ar.take<double>(2 * (size_t)k + 16);
    b.feat = ar.take<float>((size_t)m * MLP_NF + 16);
    b.dpred = ar.take<float>(m + 16);
    b.eigw = ar.get(eig_work_bytes(m));
    // split-K partials: the largest of the filter (n x m, K = n; automatic or tuned plan) and the
    // Gram products (m x m, K = n)
    size_t ws = std::max(zgemm_ws_bytes(n, m, n, 16), zgemm_ws_bytes(m, m, n, 16));
    ws = std::max(ws, zgemm_ws_bytes(n, m, m, 16));
    ws = std::max(ws, (size_t)filter_ksplit * n * m * 16);
    b.gw.bytes = ws;
    b.gw.ws = ar.get(ws);
}

chfsi_status prepare(chfsi_handle h, SolveBufs& b, int n, int m, int k, bool gen, int prec, bool reduce_ws = false)
{
    return prepare_bufs(h, h->ws, b, n, m, k, gen, prec, reduce_ws);
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

// Puts the columns of Y back into the order they had before the filter sorted them (the inverse
// permutation is at b.iperm + ma): the order of ascending Ritz values.  Cholesky QR keeps the span
// of every leading set of columns, so the nearly converged columns must lead; in the degree order
// they would be mixed with the unconverged ones, which costs the Rayleigh-Ritz eigensolver sweeps.
chfsi_status restore_column_order(chfsi_handle h, SolveBufs& b, int n, int ma, zd* Y, int ldy)
{
    hipStream_t st = h->stream;
    TRY(launch_permute_cols(st, n, ma, Y, ldy, b.T, n, b.iperm + ma));
    TRY(launch_zlacpy(st, n, ma, b.T, n, Y, ldy));
    return CHFSI_SUCCESS;
}

// Filters the active block Y (n x ma) with per-column degrees deg and precision flags lowp
// (1 = low precision).  Columns are reordered for the filter (low-precision group first, each group
// sorted by non-increasing degree) and put back into their order afterwards.  HY (nullable, ld n):
// H Y for the block's columns, which turns every filter's first step into an elementwise update; it
// is reordered with Y and not restored (it is consumed).
chfsi_status run_filter(chfsi_handle h, SolveBufs& b, int n, const zd* H, int ldh, int prec, int ma, zd* Y, int ldy,
                        std::vector<int>& deg, std::vector<int>& lowp, double a, double bb, double mu1,
                        double& flops, long long& matvecs, zd* HY = nullptr)
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
    std::vector<int> perm(2 * (size_t)ma);   // [order | inverse]
    if (!ident) {
        for (int j = 0; j < ma; ++j) { perm[j] = ord[j]; perm[ma + ord[j]] = j; }
        TRY(hipMemcpyAsync(b.iperm, perm.data(), sizeof(int) * 2 * ma, hipMemcpyHostToDevice, st));
        TRY(launch_permute_cols(st, n, ma, Y, ldy, b.T, n, b.iperm));
        TRY(launch_zlacpy(st, n, ma, b.T, n, Y, ldy));
        if (HY) {
            TRY(launch_permute_cols(st, n, ma, HY, n, b.T, n, b.iperm));
            TRY(launch_zlacpy(st, n, ma, b.T, n, HY, n));
        }
        std::vector<int> d2(ma), l2(ma);
        for (int j = 0; j < ma; ++j) { d2[j] = deg[ord[j]]; l2[j] = lowp[ord[j]]; }
        deg.swap(d2);
        lowp.swap(l2);
        TRY(hipStreamSynchronize(st));   // perm must outlive the async copy
    }
    int nlow = 0;
    while (nlow < ma && lowp[nlow]) ++nlow;
    if (nlow > 0 && prec != CHFSI_FP64) {
        std::vector<int> dl(deg.begin(), deg.begin() + nlow);
        TRY(launch_z2c(st, n, nlow, Y, ldy, b.Vf, n));
        if (prec == CHFSI_FP32) {
            TRYS(filter_f32(h, n, b.Hf, n, nlow, b.Vf, n, b.Tf, dl, a, bb, mu1, b.flag, b.gw,
                            flops, matvecs, HY));
        } else {
            const int nterms = prec == CHFSI_BF16X3 ? 2 : 3;
            TRYS(filter_bf16(h, n, b.Hb, n, nterms, nlow, b.Vf, n, b.Tf, b.ysplit, dl, a, bb, mu1, b.flag,
                             b.gw, flops, matvecs, HY));
        }
        TRY(launch_c2z(st, n, nlow, b.Vf, n, Y, ldy));
    }
    const int n64 = (prec == CHFSI_FP64) ? ma : ma - nlow;
    const int off = ma - n64;
    if (n64 > 0) {
        std::vector<int> dh(deg.begin() + off, deg.end());
        TRYS(filter_f64(h, n, H, ldh, n64, Y + (size_t)off * ldy, ldy, b.T, dh, a, bb, mu1, b.flag, b.gw, flops, matvecs,
                        HY ? HY + (size_t)off * n : nullptr));
    }
    if (!ident) TRYS(restore_column_order(h, b, n, ma, Y, ldy));
    return CHFSI_SUCCESS;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// the phases of one solve (state.h)
// ---------------------------------------------------------------------------------------------

chfsi_status prepare_bufs(chfsi_handle h, Arena& ar, SolveBufs& b, int n, int m, int k, bool gen, int prec,
                          bool reduce_ws)
{
    // the largest K split of a tuned filter plan that a step of this order may take
    int fks = 1;
    for (const TuneEntry& e : h->plans) {
        const double r = e.n > n ? (double)e.n / n : (double)n / e.n;
        if (r <= 1.5) fks = std::max(fks, e.ksplit);
    }
    ar.begin(true);
    layout(ar, b, n, m, k, gen, prec, fks, reduce_ws);
    const size_t need = ar.off;
    if (need > ar.cap) {
        (void)hipStreamSynchronize(h->stream);
        ar.grow(need + (need >> 3));
        if (ar.cap < need) return CHFSI_ERR_ALLOC;
    }
    ar.begin(false);
    b = SolveBufs();
    layout(ar, b, n, m, k, gen, prec, fks, reduce_ws);
    b.gw.cnt = h->tile_cnt;
    b.gw.ncnt = h->tile_cnt_len;
    return ar.failed ? CHFSI_ERR_ALLOC : CHFSI_SUCCESS;
}

chfsi_status st_define(SolveState& s, int n, const zd* A, int lda, const zd* S, int lds, zd* X, int ldx,
                       int x_is_guess, double* lambda, double* resid, const chfsi_params& p)
{
    const int nev = p.nev, m = p.nev + p.nex;
    const int prec = p.filter_precision;
    if (n <= 0 || nev <= 0 || p.nex < 0 || m > n || lda < n || ldx < n || (S && lds < n) || !A || !X || !lambda ||
        !resid || p.deg < 0 || !(p.tol > 0) || p.max_loops < 1 || prec < 0 || prec > 3 || p.deg_min < 0 ||
        p.deg_max < p.deg_min || p.degree_policy < 0 || p.degree_policy > 3)
        return CHFSI_ERR_ARG;
    s.n = n; s.nev = nev; s.m = m; s.prec = prec;
    s.A = A; s.lda = lda; s.S = S; s.lds = lds; s.X = X; s.ldx = ldx; s.x_is_guess = x_is_guess;
    s.lambda = lambda; s.resid = resid; s.p = p;
    int k = std::max(p.lanczos_steps, 10);
    k = std::min(k, 3 * m);
    s.k = std::min(k, n);
    return CHFSI_SUCCESS;
}

chfsi_status st_setup(chfsi_handle h, SolveState& s, Arena& ar, PinBuf& pin)
{
    if (s.p.degree_policy == CHFSI_DEG_LEARNED && !h->has_model) return CHFSI_ERR_ARG;
    TRYS(prepare_bufs(h, ar, s.b, s.n, s.m, s.k, s.S != nullptr, s.prec));
    const size_t nd = SolveState::pinned_doubles(s.m, s.k);
    if (!pin.reserve(sizeof(double) * nd + sizeof(int) * SolveState::pinned_ints(s.m))) return CHFSI_ERR_ALLOC;
    s.hd = (double*)pin.p;
    s.hi = (int*)(pin.p + sizeof(double) * nd);
    std::memset(s.hi, 0, sizeof(int) * 32);
    return CHFSI_SUCCESS;
}

static inline void mark(SolveState& s, int phase, hipStream_t st, bool begin)
{
    if (s.tm) s.tm->mark(phase, st, begin);
}

// Orders up to which H = L^{-1} A L^{-H} is formed from the explicit inverse L^{-1} (two products
// that skip its zero triangle, about 16 n^3 / 3 flops in three launches) rather than by the panel
// algorithm (4 n^3 flops in about ten launches per 64 columns): below it the launches dominate.
constexpr int EXPLICIT_REDUCTION_MAX_N = 3072;
inline bool explicit_reduction(int n) { return n <= EXPLICIT_REDUCTION_MAX_N; }

// The handle's cache of the last overlap's Cholesky factor: [copy of S | L | inverses of L's
// 64 x 64 diagonal blocks], all for order fc_n, and for the orders reduced with the explicit
// inverse also [L^{-1} | n x n product buffer].
struct FactorCache { zd *S, *L, *dinv, *Linv, *T; };
size_t factor_cache_bytes(int n)
{
    const size_t nn = (size_t)n * n;
    return ((explicit_reduction(n) ? 4 : 2) * nn + tri_dinv_elems(n)) * sizeof(zd);
}
FactorCache factor_cache(chfsi_handle h, int n)
{
    zd* base = (zd*)h->fc.base;
    const size_t nn = (size_t)n * n;
    zd* dinv = base + 2 * nn;
    zd* Linv = dinv + tri_dinv_elems(n);
    return {base, base + nn, dinv, explicit_reduction(n) ? Linv : nullptr, explicit_reduction(n) ? Linv + nn : nullptr};
}

// Reduction to standard form with the handle's factor cache: when S equals (bit for bit) the
// overlap of the cached factor, the Cholesky factorisation is skipped and only H = L^{-1} A L^{-H}
// is formed; otherwise S is factored as usual and the cache takes S, L and the block inverses
// (valid once the factorisation is known to have succeeded, see st_init_complete).  Small orders
// form H from the cached L^{-1}, computed once per factorisation; a fresh factorisation forms H
// the same way, so a solve that reuses the factor gives the same bits as one that does not.
chfsi_status reduce_with_cache(chfsi_handle h, SolveState& s)
{
    hipStream_t st = h->stream;
    SolveBufs& b = s.b;
    const int n = s.n;
    if (h->fc_enabled && h->fc_n == n && h->fc.base) {
        const FactorCache fc = factor_cache(h, n);
        int* dflag = b.info + 12;
        TRY(hipMemsetAsync(dflag, 0, sizeof(int), st));
        TRY(launch_any_diff(st, n, s.S, s.lds, fc.S, n, dflag));
        TRY(hipMemcpyAsync(&s.hi[1], dflag, sizeof(int), hipMemcpyDeviceToHost, st));
        TRY(hipStreamSynchronize(st));
        if (s.hi[1] == 0) {
            TRY(launch_zlacpy(st, n, n, fc.L, n, b.L, n));
            TRY(hipMemcpyAsync(b.dinvL, fc.dinv, sizeof(zd) * tri_dinv_elems(n), hipMemcpyDeviceToDevice, st));
            if (fc.Linv) {
                TRY(hegst_explicit(st, n, s.A, s.lda, fc.Linv, fc.T, b.H));
            } else {
                TRY(launch_zlacpy(st, n, n, s.A, s.lda, b.H, n));
                TRY(hegst_lower(st, n, b.H, n, b.L, n, b.dinvL, b.hwork, b.gw));
            }
            s.hi[0] = 0;
            s.fc_reused = true;
            return CHFSI_SUCCESS;
        }
    }
    if (!h->fc_enabled)
        return step_reduce_enqueue(h, n, s.A, s.lda, s.S, s.lds, b.H, b.L, b.dinvL, b.hwork, b.info, s.hi, b.gw);
    h->fc_n = 0;
    const size_t need = factor_cache_bytes(n);
    if (h->fc.cap < need) {
        TRY(hipStreamSynchronize(st));
        h->fc.grow(need);
    }
    if (h->fc.cap < need)   // no room: solve without the cache
        return step_reduce_enqueue(h, n, s.A, s.lda, s.S, s.lds, b.H, b.L, b.dinvL, b.hwork, b.info, s.hi, b.gw);
    const FactorCache fc = factor_cache(h, n);
    if (fc.Linv) {
        TRYS(step_factor_enqueue(h, n, s.S, s.lds, b.L, b.dinvL, b.info, s.hi, b.gw));
        TRY(tri_inverse_lower(st, n, b.L, n, b.dinvL, fc.Linv, n, b.gw));
        TRY(hegst_explicit(st, n, s.A, s.lda, fc.Linv, fc.T, b.H));
    } else {
        TRYS(step_reduce_enqueue(h, n, s.A, s.lda, s.S, s.lds, b.H, b.L, b.dinvL, b.hwork, b.info, s.hi, b.gw));
    }
    TRY(launch_zlacpy(st, n, n, s.S, s.lds, fc.S, n));
    TRY(launch_zlacpy(st, n, n, b.L, n, fc.L, n));
    TRY(hipMemcpyAsync(fc.dinv, b.dinvL, sizeof(zd) * tri_dinv_elems(n), hipMemcpyDeviceToDevice, st));
    s.fc_store = true;
    return CHFSI_SUCCESS;
}

chfsi_status st_init_enqueue(chfsi_handle h, SolveState& s)
{
    hipStream_t st = h->stream;
    SolveBufs& b = s.b;
    const int n = s.n, m = s.m;
    s.t0 = std::chrono::steady_clock::now();
    // --- reduction to standard form (Section 3.2)
    mark(s, PH_REDUCE, st, true);
    s.H = s.A;
    s.ldh = s.lda;
    s.hi[0] = 0;
    if (s.S) {
        TRYS(reduce_with_cache(h, s));
        s.H = b.H;
        s.ldh = n;
    }
    double* hn = s.h_norms();
    hn[1] = 1.0;
    TRY(launch_max_colnorm(st, n, s.A, s.lda, b.dsc));
    TRY(hipMemcpyAsync(&hn[0], b.dsc, sizeof(double), hipMemcpyDeviceToHost, st));
    if (s.S) {   // second half of dsc: no kernel rewrites a buffer with a copy from it pending
        double* d2 = b.dsc + std::max(n, m) + 16;
        TRY(launch_max_rowsum_abs(st, n, s.S, s.lds, d2));
        TRY(hipMemcpyAsync(&hn[1], d2, sizeof(double), hipMemcpyDeviceToHost, st));
    }
    if (s.prec == CHFSI_FP32) TRY(launch_z2c(st, n, n, s.H, s.ldh, b.Hf, n));
    if (s.prec == CHFSI_BF16X3 || s.prec == CHFSI_BF16X6)
        TRY(launch_split_h_bf16(st, n, s.H, s.ldh, b.Hb, n, s.prec == CHFSI_BF16X3 ? 2 : 3));
    // starting block in standard coordinates
    if (s.x_is_guess) {
        if (s.S) TRY(launch_zgemm(st, OP_C, OP_N, n, m, n, 1.0, b.L, n, s.X, s.ldx, 0.0, b.V, n, b.gw));
        else TRY(launch_zlacpy(st, n, m, s.X, s.ldx, b.V, n));
    } else {
        TRY(launch_philox_block(st, s.p.seed, 1, n, m, b.V, n));
    }
    mark(s, PH_REDUCE, st, false);
    // --- Lanczos bounds
    mark(s, PH_LANCZOS, st, true);
    TRYS(step_lanczos_enqueue(h, n, s.H, s.ldh, s.k, s.p.seed, b.LV, b.lw, b.lc, b.lcoef, s.h_al(), s.h_be()));
    mark(s, PH_LANCZOS, st, false);
    return CHFSI_SUCCESS;
}

chfsi_status st_init_complete(chfsi_handle h, SolveState& s)
{
    TRY(hipStreamSynchronize(h->stream));
    if (s.S && s.hi[0] != 0) return CHFSI_ERR_NOT_HPD;
    if (s.fc_store) h->fc_n = s.n;   // the factorisation succeeded: the cache is valid
    const chfsi_params& p = s.p;
    const int m = s.m;
    const double norm_a = s.h_norms()[0], s_inf = s.h_norms()[1];
    if (!std::isfinite(norm_a) || !std::isfinite(s_inf) || !(norm_a > 0)) return CHFSI_ERR_NUMERIC;
    s.norm_a = norm_a;
    s.thr = p.tol * norm_a / std::sqrt(s_inf);
    std::vector<double> lth, lz;
    double beta_k = 0;
    int kk = 0;
    TRYS(lanczos_finish(s.k, s.h_al(), s.h_be(), lth, lz, beta_k, kk));
    s.k = kk;
    // b = largest Ritz value + beta_k; a from the cumulative weight m / n; mu1 = smallest
    s.bb = lth[kk - 1] + beta_k;
    s.mu1 = lth[0];
    s.a = lth[kk - 1];
    {
        const double frac = (double)m / s.n;
        double cum = 0;
        for (int j = 0; j < kk; ++j) {
            cum += lz[j];
            if (cum >= frac) { s.a = lth[j]; break; }
        }
        if (!(s.a > s.mu1) || !(s.a < s.bb)) s.a = 0.5 * (s.mu1 + s.bb);
    }
    if (p.have_bounds) {
        s.mu1 = p.mu1;
        s.a = p.a;
        if (!(s.a > s.mu1) || !(s.a < s.bb)) s.a = 0.5 * (s.mu1 + s.bb);
    }
    s.deg.assign(m, p.deg);
    s.lowp.assign(m, s.prec != CHFSI_FP64 ? 1 : 0);
    s.deg_used.assign(m, p.deg);
    s.rprev.assign(m, -1.0);
    s.last_row.assign(m, -1);
    s.trace.clear();
    const double sw_rel = p.switch_residual > 0 ? p.switch_residual : (s.prec == CHFSI_BF16X3 ? 1e-3 : 1e-5);
    s.sw_thr = sw_rel * norm_a;
    return CHFSI_SUCCESS;
}

chfsi_status st_filter(chfsi_handle h, SolveState& s)
{
    const int ma = s.ma();
    mark(s, PH_FILTER, h->stream, true);
    std::vector<int> dact(s.deg.begin() + s.nlocked, s.deg.end()), lact(s.lowp.begin() + s.nlocked, s.lowp.end());
    zd* hy = s.hy_off >= 0 ? s.b.HY + (size_t)s.hy_off * s.n : nullptr;
    s.hy_off = -1;
    TRYS(run_filter(h, s.b, s.n, s.H, s.ldh, s.prec, ma, s.Ya(), s.n, dact, lact, s.a, s.bb, s.mu1, s.flops,
                    s.matvecs, hy));
    mark(s, PH_FILTER, h->stream, false);
    return CHFSI_SUCCESS;
}

chfsi_status st_order_columns(chfsi_handle h, SolveState& s, std::vector<int>& dsorted)
{
    hipStream_t st = h->stream;
    const int ma = s.ma(), n = s.n;
    std::vector<int> ord(ma);
    std::iota(ord.begin(), ord.end(), 0);
    const int* d = s.deg.data() + s.nlocked;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] > d[y]; });
    dsorted.resize(ma);
    bool ident = true;
    for (int j = 0; j < ma; ++j) { dsorted[j] = d[ord[j]]; ident &= ord[j] == j; }
    s.permuted = !ident;
    if (!ident) {
        int* perm = s.h_perm();   // pinned staging [2 m]: order, inverse
        for (int j = 0; j < ma; ++j) { perm[j] = ord[j]; perm[ma + ord[j]] = j; }
        TRY(hipMemcpyAsync(s.b.iperm, perm, sizeof(int) * 2 * ma, hipMemcpyHostToDevice, st));
        TRY(launch_permute_cols(st, n, ma, s.Ya(), n, s.b.T, n, s.b.iperm));
        TRY(launch_zlacpy(st, n, ma, s.b.T, n, s.Ya(), n));
        if (s.hy_off >= 0) {   // the image H Y of the block follows its columns
            zd* hy = s.b.HY + (size_t)s.hy_off * n;
            TRY(launch_permute_cols(st, n, ma, hy, n, s.b.T, n, s.b.iperm));
            TRY(launch_zlacpy(st, n, ma, s.b.T, n, hy, n));
        }
    }
    return CHFSI_SUCCESS;
}

chfsi_status st_loop_enqueue(chfsi_handle h, SolveState& s)
{
    hipStream_t st = h->stream;
    SolveBufs& b = s.b;
    const int ma = s.ma(), n = s.n;
    zd* Ya = s.Ya();
    s.loops += 1;
    s.filtered += ma;
    if (s.permuted) {   // the batched filter ran on degree-sorted columns (st_order_columns)
        TRYS(restore_column_order(h, b, n, ma, Ya, n));
        s.permuted = false;
    }
    mark(s, PH_QR, st, true);
    TRY(hipMemsetAsync(b.info, 0, sizeof(int) * 8, st));
    // (the eigensolver's pinned host buffer is free until Rayleigh-Ritz)
    TRYS(step_orthonormalize(h, n, ma, Ya, n, s.nlocked, b.V, n, b.G, b.Cm, b.dinvG, b.dsc, b.info, b.gw,
                             s.h_eig(), b.T));
    mark(s, PH_QR, st, false);
    mark(s, PH_RR, st, true);
    // the Rayleigh quotient is diagonalised to a tenth of the locking threshold: a Ritz vector
    // then differs from the exact one of the subspace by far less than the residual that locks it
    TRYS(step_rayleigh_ritz(h, n, s.H, s.ldh, ma, Ya, n, b.HY, b.T, b.G, b.theta, b.r, b.eigw, s.h_eig(), b.gw,
                            s.tm, 0.1 * s.thr));
    mark(s, PH_RR, st, false);
    TRY(hipMemcpyAsync(s.h_theta(), b.theta, sizeof(double) * ma, hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(s.h_r(), b.r, sizeof(double) * ma, hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(s.hi + 8, b.info, sizeof(int) * 8, hipMemcpyDeviceToHost, st));
    return CHFSI_SUCCESS;
}

chfsi_status st_loop_complete(chfsi_handle h, SolveState& s)
{
    hipStream_t st = h->stream;
    TRY(hipStreamSynchronize(st));
    const chfsi_params& p = s.p;
    const int ma = s.ma(), nev = s.nev, nlocked = s.nlocked, it = s.loops - 1;
    const double* hth = s.h_theta();
    const double* hr = s.h_r();
    for (int j = 0; j < 8; ++j)
        if (s.hi[8 + j] != 0) return CHFSI_ERR_NUMERIC;
    for (int j = 0; j < ma; ++j)
        if (!std::isfinite(hth[j]) || !std::isfinite(hr[j])) return CHFSI_ERR_NUMERIC;
    mark(s, PH_LOCK, st, true);

    for (int j = 0; j < ma; ++j) s.deg_used[nlocked + j] = s.deg[nlocked + j];   // degrees of this loop
    // trace: close the rows of the previous loop
    if (p.trace)
        for (int j = 0; j < ma; ++j) {
            const int pos = nlocked + j;
            if (s.last_row[pos] >= 0) s.trace[s.last_row[pos]].r_after = hr[j];
        }
    int cnt = 0;
    while (cnt < nev - nlocked && hr[cnt] <= s.thr) ++cnt;
    for (int j = 0; j < ma; ++j) { s.lambda[nlocked + j] = hth[j]; s.resid[nlocked + j] = hr[j]; }

    // per-column precision for the next loop: back to FP64 once a residual is small or stagnates
    const int nl2 = nlocked + cnt;
    for (int j = cnt; j < ma; ++j) {
        const int pos = nlocked + j;
        if (s.lowp[pos]) {
            const bool stagnated = s.rprev[pos] > 0 && hr[j] > 0.1 * s.rprev[pos];
            if (hr[j] <= s.sw_thr || stagnated) { s.lowp[pos] = 0; ++s.switches; }
        }
    }
    // bounds for the next filter
    s.a = hth[ma - 1];
    s.mu1 = std::min(s.mu1, hth[0]);
    if (!(s.a > s.mu1)) s.a = 0.5 * (s.mu1 + s.bb);
    const double a = s.a, bb = s.bb, mu1 = s.mu1, thr = s.thr;
    if (p.degree_policy == CHFSI_DEG_ANALYTIC) {
        for (int j = cnt; j < ma; ++j)
            s.deg[nlocked + j] = analytic_degree(hth[j], hr[j], a, bb, thr, p.deg_min, p.deg_max);
    } else if (p.degree_policy == CHFSI_DEG_RANDOM) {
        for (int j = cnt; j < ma; ++j)
            s.deg[nlocked + j] = random_degree(p.seed, it, nlocked + j, p.deg_min, p.deg_max);
    } else if (p.degree_policy == CHFSI_DEG_LEARNED) {
        TRYS(learned_degrees(h, ma - cnt, s.b.theta + cnt, s.b.r + cnt, a, bb, mu1, thr,
                             std::vector<int>(s.deg.begin() + nl2, s.deg.end()), s.b.feat, s.b.dpred, s.b.iperm,
                             p.deg_min, p.deg_max, s.deg.data() + nl2,
                             [&](int j) { return analytic_degree(hth[cnt + j], hr[cnt + j], a, bb, thr,
                                                                 p.deg_min, p.deg_max); }));
    }
    if (p.deg_margin != 0 && (p.degree_policy == CHFSI_DEG_ANALYTIC || p.degree_policy == CHFSI_DEG_LEARNED))
        for (int j = cnt; j < ma; ++j)
            s.deg[nlocked + j] = std::max(p.deg_min, std::min(p.deg_max, s.deg[nlocked + j] + p.deg_margin));
    // With a per-vector degree (analytic or learned, chosen to bring each residual to the locking
    // threshold in one loop) a column keeps the low-precision filter for the next loop only while
    // that loop is not expected to take its residual below the switch level: predicted r / rho^d,
    // rho = |t| + sqrt(t^2 - 1) the growth per step of T_d at its Ritz value (the model of the
    // analytic rule).  A vector filtered in low precision stops near that level, so filtering it
    // there in low precision would cost one more loop.  (With a fixed degree the prediction is
    // looser and the switch waits for the residual itself.)
    if (s.prec != CHFSI_FP64 && (p.degree_policy == CHFSI_DEG_ANALYTIC || p.degree_policy == CHFSI_DEG_LEARNED)) {
        const double c2 = 0.5 * (a + bb), e2 = 0.5 * (bb - a), lthr = std::log10(s.sw_thr);
        for (int j = cnt; j < ma; ++j) {
            const int pos = nlocked + j;
            const double t = (hth[j] - c2) / e2;
            if (!s.lowp[pos] || !(std::fabs(t) > 1.0)) continue;
            const double rho = std::fabs(t) + std::sqrt(t * t - 1.0);
            if (std::log10(std::max(hr[j], 1e-300)) - s.deg[pos] * std::log10(rho) <= lthr) {
                s.lowp[pos] = 0;
                ++s.switches;
            }
        }
    }
    if (p.trace) {
        const double c2 = 0.5 * (a + bb), e2 = 0.5 * (bb - a);
        for (int j = cnt; j < ma; ++j) {
            const int pos = nlocked + j;
            TraceRow row;
            row.loop = it; row.col = pos; row.t = (hth[j] - c2) / e2;
            row.lr = std::log10(std::max(hr[j], 1e-300)); row.a = (a - mu1) / (bb - mu1);
            row.b = (bb - mu1) / (std::fabs(mu1) + std::fabs(bb)); row.d_prev = s.deg_used[pos];
            row.d = s.deg[pos]; row.r_after = -1.0;
            row.thr = thr;
            s.last_row[pos] = (int)s.trace.size();
            s.trace.push_back(row);
        }
    }
    for (int j = 0; j < ma; ++j) s.rprev[nlocked + j] = hr[j];
    s.nlocked = nl2;
    // HY = H Ya from this loop's Rayleigh-Ritz step: its columns from cnt on are the next block's
    s.hy_off = cnt;
    mark(s, PH_LOCK, st, false);
    s.want_final = s.nlocked >= nev;
    return CHFSI_SUCCESS;
}

// X = L^{-H} V (or V), rho_j = ||A x_j - lambda_j S x_j|| / ||A||_lo for all m columns
chfsi_status st_final_enqueue(chfsi_handle h, SolveState& s)
{
    hipStream_t st = h->stream;
    SolveBufs& b = s.b;
    const int n = s.n, m = s.m;
    s.hy_off = -1;   // HY is overwritten below
    mark(s, PH_BACK, st, true);
    if (s.S && h->fc_enabled && h->fc_n == n && explicit_reduction(n)) {
        // the cache holds this overlap's L^{-1}: X = L^{-H} V is one product
        TRY(launch_zgemm(st, OP_C, OP_N, n, m, n, 1.0, factor_cache(h, n).Linv, n, b.V, n, 0.0, s.X, s.ldx, b.gw));
    } else {
        TRY(launch_zlacpy(st, n, m, b.V, n, s.X, s.ldx));
        if (s.S) TRY(trsm_left_lower_h(st, n, m, b.L, n, b.dinvL, s.X, s.ldx, b.gw));   // X = L^{-H} V
    }
    // the verification products have the shape of a filter step: the filter's tuned plan
    GemmWs gv = b.gw;
    apply_tuned_plan(h, CHFSI_FP64, n, m, gv);
    TRY(launch_zgemm(st, OP_N, OP_N, n, m, n, 1.0, s.A, s.lda, s.X, s.ldx, 0.0, b.HY, n, gv));
    const zd* SX = s.X;
    int ldsx = s.ldx;
    if (s.S) {
        TRY(launch_zgemm(st, OP_N, OP_N, n, m, n, 1.0, s.S, s.lds, s.X, s.ldx, 0.0, b.T, n, gv));
        SX = b.T;
        ldsx = n;
    }
    std::memcpy(s.h_lam(), s.lambda, sizeof(double) * m);
    TRY(hipMemcpyAsync(b.lam, s.h_lam(), sizeof(double) * m, hipMemcpyHostToDevice, st));
    TRY(launch_residual_norms(st, n, m, b.HY, n, SX, ldsx, b.lam, b.r));
    TRY(hipMemcpyAsync(s.h_res(), b.r, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    mark(s, PH_BACK, st, false);
    return CHFSI_SUCCESS;
}

static chfsi_status final_results(chfsi_handle h, SolveState& s)
{
    TRY(hipStreamSynchronize(h->stream));
    for (int j = 0; j < s.m; ++j) s.resid[j] = s.h_res()[j] / s.norm_a;
    s.finalized = true;
    return CHFSI_SUCCESS;
}

chfsi_status st_final_complete(chfsi_handle h, SolveState& s)
{
    TRYS(final_results(h, s));
    s.want_final = false;
    int bad = -1;
    for (int j = 0; j < s.nev; ++j)
        if (!(s.resid[j] <= s.p.tol)) { bad = j; break; }
    if (bad < 0) {
        s.status = CHFSI_SUCCESS;
        s.done = true;
        return CHFSI_SUCCESS;
    }
    // a locked pair failed the verification in generalized coordinates: unlock from there on
    s.nlocked = bad;
    for (int j = bad; j < s.m; ++j) s.deg[j] = s.p.deg;
    return CHFSI_SUCCESS;
}

void st_finish(chfsi_handle h, SolveState& s, chfsi_stats& stt)
{
    if (s.status == CHFSI_ERR_NO_CONVERGENCE && !s.finalized && s.hd) {
        if (st_final_enqueue(h, s) != CHFSI_SUCCESS || final_results(h, s) != CHFSI_SUCCESS)
            s.status = CHFSI_ERR_DEVICE;
    }
    stt.loops = s.loops;
    stt.nlocked = std::min(s.nlocked, s.nev);
    stt.filtered_vectors = s.filtered;
    stt.matvecs = s.matvecs;
    stt.filter_flops = s.flops;
    stt.mu1 = s.mu1; stt.a = s.a; stt.b = s.bb;
    stt.norm_a = s.norm_a;
    stt.lanczos_steps = s.k;
    stt.precision_switches = s.switches;
    stt.t_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - s.t0).count();
    stt.status = s.status;
}

static void store_trace(chfsi_handle h, const SolveState& s)
{
    h->trace.clear();
    for (auto& r : s.trace) {
        const double row[CHFSI_TRACE_COLS] = {(double)r.loop, (double)r.col, r.t, r.lr, r.a, r.b,
                                              (double)r.d_prev, (double)r.d, r.r_after, r.thr};
        h->trace.insert(h->trace.end(), row, row + CHFSI_TRACE_COLS);
    }
}

chfsi_status solve_impl(chfsi_handle h, int n, const zd* A, int lda, const zd* S, int lds, zd* X, int ldx,
                        int x_is_guess, double* lambda, double* resid, const chfsi_params& p, chfsi_stats& stt)
{
    hipStream_t st = h->stream;
    SolveState s;
    TRYS(st_define(s, n, A, lda, S, lds, X, ldx, x_is_guess, lambda, resid, p));
    TRYS(st_setup(h, s, h->ws, h->pin));
    PhaseTimer& tm = h->timer;
    {
        double reset[NPHASE];
        tm.collect(reset);
        (void)h->ktimer.collect(nullptr);
    }
    s.tm = &tm;
    tm.mark(PH_TOTAL, st, true);
    chfsi_status rc = st_init_enqueue(h, s);
    if (rc == CHFSI_SUCCESS) rc = st_init_complete(h, s);
    if (rc != CHFSI_SUCCESS) {
        (void)hipStreamSynchronize(st);
        return rc;
    }
    while (!s.done && s.loops < p.max_loops) {
        rc = st_filter(h, s);
        if (rc == CHFSI_SUCCESS) rc = st_loop_enqueue(h, s);
        if (rc == CHFSI_SUCCESS) rc = st_loop_complete(h, s);
        if (rc == CHFSI_SUCCESS && s.want_final) {
            rc = st_final_enqueue(h, s);
            if (rc == CHFSI_SUCCESS) rc = st_final_complete(h, s);
        }
        if (rc == CHFSI_ERR_NUMERIC) { s.status = rc; break; }
        if (rc != CHFSI_SUCCESS) { (void)hipStreamSynchronize(st); return rc; }
    }
    st_finish(h, s, stt);
    tm.mark(PH_TOTAL, st, false);
    TRY(hipStreamSynchronize(st));
    double ph[NPHASE];
    tm.collect(ph);
    stt.t_reduce = ph[PH_REDUCE]; stt.t_lanczos = ph[PH_LANCZOS]; stt.t_filter = ph[PH_FILTER];
    stt.factor_reused = s.fc_reused ? 1 : 0;
    stt.t_qr = ph[PH_QR]; stt.t_rr = ph[PH_RR]; stt.t_resid = ph[PH_RESID]; stt.t_lock = ph[PH_LOCK];
    stt.t_back = ph[PH_BACK];
    stt.t_filter_kernels = h->ktimer.collect(&stt.filter_launches, &stt.t_filter_steps);
    h->last_kernel_ms = stt.t_filter_kernels;
    h->last_kernel_launches = stt.filter_launches;
    if (p.trace) store_trace(h, s);
    return s.status;
}

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
    // (run_filter sorts the columns by degree for the filter and puts them back afterwards)
    std::vector<int> lowp(m, prec != CHFSI_FP64 ? 1 : 0), dd = d;
    double flops = 0;
    long long mv = 0;
    TRYS(run_filter(h, bf, n, H, ldh, prec, m, Y, ldy, dd, lowp, a, b, mu1, flops, mv));
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
    TRYS(prepare(h, b, n, 1, 1, false, CHFSI_FP64, true));
    TRYS(step_reduce(h, n, (const zd*)A, lda, (const zd*)S, lds, (zd*)H, (zd*)L, b.dinvL, b.hwork, b.info, b.gw));
    TRY(hipStreamSynchronize(h->stream));
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_reduce_explicit(chfsi_handle h, int n, const void* A, int lda, const void* S, int lds, void* H,
                                   void* L)
{
    if (!h || !A || !S || !H || !L || n <= 0 || lda < n || lds < n) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    SolveBufs b;
    TRYS(prepare(h, b, n, 1, 1, false, CHFSI_FP64, true));
    hipStream_t st = h->stream;
    zd* work = nullptr;   // [L^{-1} | product buffer]
    if (hipMalloc((void**)&work, 2 * (size_t)n * n * sizeof(zd)) != hipSuccess) return CHFSI_ERR_ALLOC;
    int info = 0;
    chfsi_status rc = step_factor_enqueue(h, n, (const zd*)S, lds, (zd*)L, b.dinvL, b.info, &info, b.gw);
    if (rc == CHFSI_SUCCESS && tri_inverse_lower(st, n, (const zd*)L, n, b.dinvL, work, n, b.gw) != 0)
        rc = CHFSI_ERR_DEVICE;
    if (rc == CHFSI_SUCCESS &&
        hegst_explicit(st, n, (const zd*)A, lda, work, work + (size_t)n * n, (zd*)H) != 0)
        rc = CHFSI_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess && rc == CHFSI_SUCCESS) rc = CHFSI_ERR_DEVICE;
    (void)hipFree(work);
    if (rc == CHFSI_SUCCESS && info != 0) rc = CHFSI_ERR_NOT_HPD;
    return rc;
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
    TRYS(step_orthonormalize(h, n, m, (zd*)Y, ldy, nl, (const zd*)YL, ldyl, b.G, b.Cm, b.dinvG, b.dsc, b.info, b.gw));
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
    std::vector<double> ehost(eig_host_doubles(m));
    TRYS(step_rayleigh_ritz(h, n, (const zd*)H, ldh, m, (zd*)Y, ldy, b.HY, b.T, b.G, b.theta, b.r, b.eigw, ehost.data(),
                            b.gw, nullptr));
    int info = 0;
    TRY(hipMemcpyAsync(theta, b.theta, sizeof(double) * m, hipMemcpyDeviceToHost, h->stream));
    TRY(hipMemcpyAsync(resid, b.r, sizeof(double) * m, hipMemcpyDeviceToHost, h->stream));
    TRY(hipMemcpyAsync(&info, b.info, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    TRY(hipStreamSynchronize(h->stream));
    return info ? CHFSI_ERR_NUMERIC : CHFSI_SUCCESS;
}

// Correlation of successive eigenvector blocks (Section 2.2 and Fig. 1): O = Xp^H S Xc, the angle of
// each pair (xp_i, xc_i) from the part of xc_i off xp_i, and the principal angles between the spans
// from the eigenvalues of R^H S R with R = Xc - Xp O (R explicit: no cancellation for small angles).
chfsi_status chfsi_correlation(chfsi_handle h, int n, int m, const void* Sv, int lds, const void* Xpv, int ldxp,
                               const void* Xcv, int ldxc, void* Ov, int ldo, double* sin_pair, double* sin_sub)
{
    if (!h || !Xpv || !Xcv || !Ov || n <= 0 || m <= 0 || m > n || ldxp < n || ldxc < n || ldo < m ||
        (Sv && lds < n) || !sin_pair || !sin_sub)
        return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    SolveBufs b;
    TRYS(prepare(h, b, n, m, 1, false, CHFSI_FP64));
    hipStream_t st = h->stream;
    const zd* S = (const zd*)Sv;
    const zd* Xp = (const zd*)Xpv;
    const zd* Xc = (const zd*)Xcv;
    zd* O = (zd*)Ov;
    // S times an n x m block (or the block itself for the standard problem)
    auto s_times = [&](const zd* X, int ldx, const zd** SX, int* ldsx) -> chfsi_status {
        if (!S) { *SX = X; *ldsx = ldx; return CHFSI_SUCCESS; }
        TRY(launch_zgemm(st, OP_N, OP_N, n, m, n, 1.0, S, lds, X, ldx, 0.0, b.HY, n, b.gw));
        *SX = b.HY;
        *ldsx = n;
        return CHFSI_SUCCESS;
    };
    const zd* SX = nullptr;
    int ldsx = 0;
    TRYS(s_times(Xc, ldxc, &SX, &ldsx));
    TRY(launch_zgemm(st, OP_C, OP_N, m, m, n, 1.0, Xp, ldxp, SX, ldsx, 0.0, O, ldo, b.gw));
    TRY(launch_pair_dots(st, n, m, Xc, ldxc, SX, ldsx, b.r));              // ||xc_i||_S^2
    TRY(launch_sub_diag_scaled(st, n, m, Xc, ldxc, Xp, ldxp, O, ldo, b.T, n));
    TRYS(s_times(b.T, n, &SX, &ldsx));
    TRY(launch_pair_dots(st, n, m, b.T, n, SX, ldsx, b.lam));             // ||xc_i - o_ii xp_i||_S^2
    std::vector<double> num(m), den(m), w(m);
    TRY(hipMemcpyAsync(num.data(), b.lam, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    TRY(hipMemcpyAsync(den.data(), b.r, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    // R = Xc - Xp O, G = R^H S R
    TRY(launch_zlacpy(st, n, m, Xc, ldxc, b.T, n));
    TRY(launch_zgemm(st, OP_N, OP_N, n, m, m, -1.0, Xp, ldxp, O, ldo, 1.0, b.T, n, b.gw));
    TRYS(s_times(b.T, n, &SX, &ldsx));
    TRY(launch_zgemm(st, OP_C, OP_N, m, m, n, 1.0, b.T, n, SX, ldsx, 0.0, b.G, m, b.gw));
    std::vector<double> ehost(eig_host_doubles(m));
    int sweeps = 0;
    const int rc = eig_jacobi(st, m, b.G, m, b.theta, b.eigw, ehost.data(), &sweeps);
    if (rc == -1) return CHFSI_ERR_NUMERIC;
    TRY(rc);
    TRY(hipMemcpyAsync(w.data(), b.theta, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    TRY(hipStreamSynchronize(st));
    for (int i = 0; i < m; ++i) {
        if (!std::isfinite(num[i]) || !std::isfinite(den[i]) || !(den[i] > 0) || !std::isfinite(w[i]))
            return CHFSI_ERR_NUMERIC;
        sin_pair[i] = std::sqrt(std::max(num[i], 0.0) / den[i]);
        sin_sub[i] = std::sqrt(std::max(w[i], 0.0));
    }
    return CHFSI_SUCCESS;
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
