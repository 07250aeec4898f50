// Project autotuner of the filter-step kernel: per (precision, n, block width) the fastest tile
// plan, timed with hipEvents on scratch buffers: FP64 / FP32 among the 32/64 output tiles, K splits
// of 1..16 and the two split-K summation modes; the BF16-split filters among 64 x 64 (and, for the
// two-term split, the pipelined 128 x 128) tiles and K splits of 1..16 (their K split always sums
// in the kernel).  The table lives in the handle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "chfsi.h"
#include "common.h"
#include "driver.h"

void apply_tuned_plan(chfsi_handle h, int prec, int n, int ncols, GemmWs& gw)
{
    // tuned n closest to n (ratio within 1.5), then the narrowest tuned width >= ncols, else the widest
    int nbest = -1;
    double rbest = 1.5;
    for (const TuneEntry& e : h->plans) {
        if (e.prec != prec) continue;
        const double r = e.n > n ? (double)e.n / n : (double)n / e.n;
        if (r <= rbest) { rbest = r; nbest = e.n; }
    }
    if (nbest < 0) return;
    const TuneEntry* best = nullptr;
    for (const TuneEntry& e : h->plans) {
        if (e.prec != prec || e.n != nbest || e.m < ncols) continue;
        if (!best || e.m < best->m) best = &e;
    }
    if (!best)
        for (const TuneEntry& e : h->plans)
            if (e.prec == prec && e.n == nbest && (!best || e.m > best->m)) best = &e;
    if (!best) return;
    gw.plan_bm = best->bm;
    gw.plan_bn = best->bn;
    gw.plan_ksplit = best->ksplit;
    gw.plan_mode = best->mode;
}

namespace {

void set_entry(chfsi_handle h, int prec, int n, int m, int bm, int bn, int ks, int mode)
{
    for (TuneEntry& e : h->plans)
        if (e.prec == prec && e.n == n && e.m == m) {
            e.bm = bm; e.bn = bn; e.ksplit = ks; e.mode = mode;
            return;
        }
    h->plans.push_back({prec, n, m, bm, bn, ks, mode});
}

inline bool is_bf16(int prec) { return prec == CHFSI_BF16X3 || prec == CHFSI_BF16X6; }

// a BF16-split plan: square tiles of 64, or 128 for the two-term split
inline bool bf16_tile_ok(int prec, int bm, int bn) { return bm == bn && (bm == 64 || (bm == 128 && prec == CHFSI_BF16X3)); }

// BF16-split tuning: H = 0 split into planes, Y blocks zero, every candidate timed over 5 steps
chfsi_status autotune_bf16(chfsi_handle h, int n, int m, int prec, chfsi_tile_plan* best_out, double* best_ms)
{
    hipStream_t st = h->stream;
    const int nterms = prec == CHFSI_BF16X3 ? 2 : 3;
    const int ksmax = 16;
    void *H = nullptr, *P = nullptr, *Ys = nullptr, *Y0 = nullptr, *Y1 = nullptr, *ws = nullptr;
    const size_t wsb = (size_t)ksmax * n * m * sizeof(zf);
    chfsi_status rc = CHFSI_SUCCESS;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMalloc(&H, (size_t)n * n * sizeof(zd)) != hipSuccess ||
        hipMalloc(&P, bf16_hplanes_elems(n, nterms) * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&Ys, bf16_ysplit_bytes(n, m, nterms)) != hipSuccess ||
        hipMalloc(&Y0, (size_t)n * m * sizeof(zf)) != hipSuccess || hipMalloc(&Y1, (size_t)n * m * sizeof(zf)) != hipSuccess ||
        hipMalloc(&ws, wsb) != hipSuccess)
        rc = CHFSI_ERR_ALLOC;
    if (rc == CHFSI_SUCCESS &&
        (hipMemsetAsync(H, 0, (size_t)n * n * sizeof(zd), st) != hipSuccess ||
         hipMemsetAsync(Y0, 0, (size_t)n * m * sizeof(zf), st) != hipSuccess ||
         hipMemsetAsync(Y1, 0, (size_t)n * m * sizeof(zf), st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
         hipEventCreate(&e1) != hipSuccess ||
         launch_split_h_bf16(st, n, (const zd*)H, n, (uint16_t*)P, 0, nterms) != 0))
        rc = CHFSI_ERR_DEVICE;
    FilterStep fs = {0.5, -0.25, 0.1};
    float best = 1e30f;
    int btile = 64, bks = 1;
    const int np = (n + 31) / 32 * 32;
    for (int tile : {128, 64})
        for (int ks : {1, 2, 4, 8, 16}) {
            if (rc != CHFSI_SUCCESS) break;
            if (!bf16_tile_ok(prec, tile, tile)) continue;
            if (ks > 1 && np / ks < 64) continue;
            const long tiles = (long)((n + tile - 1) / tile) * ((m + tile - 1) / tile);
            if (ks > 1 && tiles > h->tile_cnt_len) continue;
            GemmWs gw;
            gw.ws = ws; gw.bytes = wsb; gw.cnt = h->tile_cnt; gw.ncnt = h->tile_cnt_len;
            gw.plan_bm = tile; gw.plan_bn = tile; gw.plan_ksplit = ks; gw.plan_mode = 2;
            auto step = [&]() {
                return launch_filter_step_bf16(st, n, m, (const uint16_t*)P, 0, nterms, (const zf*)Y0, n, (const zf*)Y1,
                                               n, (zf*)Y1, n, fs, (uint16_t*)Ys, gw);
            };
            if (step() || step()) { rc = CHFSI_ERR_DEVICE; break; }
            const int reps = 5;
            (void)hipEventRecord(e0, st);
            for (int r = 0; r < reps; ++r)
                if (step()) rc = CHFSI_ERR_DEVICE;
            (void)hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) { rc = CHFSI_ERR_DEVICE; break; }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms /= reps;
            if (ms < best) { best = ms; btile = tile; bks = ks; }
        }
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (void* p : {H, P, Ys, Y0, Y1, ws})
        if (p) (void)hipFree(p);
    if (rc != CHFSI_SUCCESS) return rc;
    set_entry(h, prec, n, m, btile, btile, bks, 2);
    if (best_out) { best_out->bm = btile; best_out->bn = btile; best_out->ksplit = bks; best_out->fused = bks > 1; }
    if (best_ms) *best_ms = best;
    return CHFSI_SUCCESS;
}

}  // namespace

extern "C" {

chfsi_status chfsi_set_filter_plan(chfsi_handle h, int n, int m, int prec, const chfsi_tile_plan* plan)
{
    if (!h || n <= 0 || m <= 0 || (prec != CHFSI_FP64 && prec != CHFSI_FP32 && !is_bf16(prec))) return CHFSI_ERR_ARG;
    if (!plan) {
        h->plans.erase(std::remove_if(h->plans.begin(), h->plans.end(),
                                      [&](const TuneEntry& e) { return e.prec == prec && e.n == n && e.m == m; }),
                       h->plans.end());
        return CHFSI_SUCCESS;
    }
    if (plan->ksplit < 1 || plan->ksplit > 64) return CHFSI_ERR_ARG;
    if (is_bf16(prec)) {
        if (!bf16_tile_ok(prec, plan->bm, plan->bn)) return CHFSI_ERR_ARG;
        set_entry(h, prec, n, m, plan->bm, plan->bn, plan->ksplit, 2);
        return CHFSI_SUCCESS;
    }
    if ((plan->bm != 32 && plan->bm != 64) || (plan->bn != 32 && plan->bn != 64)) return CHFSI_ERR_ARG;
    set_entry(h, prec, n, m, plan->bm, plan->bn, plan->ksplit, plan->fused ? 2 : 1);
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_autotune_filter(chfsi_handle h, int n, int m, int prec, chfsi_tile_plan* best_out, double* best_ms)
{
    if (!h || n <= 0 || m <= 0 || m > n || (prec != CHFSI_FP64 && prec != CHFSI_FP32 && !is_bf16(prec)))
        return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    if (is_bf16(prec)) return autotune_bf16(h, n, m, prec, best_out, best_ms);
    hipStream_t st = h->stream;
    const size_t eb = prec == CHFSI_FP64 ? 16 : 8;
    const int ksmax = 16;
    void *H = nullptr, *Y0 = nullptr, *Y1 = nullptr, *ws = nullptr;
    const size_t wsb = (size_t)ksmax * n * m * eb;
    chfsi_status rc = CHFSI_SUCCESS;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMalloc(&H, (size_t)n * n * eb) != hipSuccess || hipMalloc(&Y0, (size_t)n * m * eb) != hipSuccess ||
        hipMalloc(&Y1, (size_t)n * m * eb) != hipSuccess || hipMalloc(&ws, wsb) != hipSuccess) {
        rc = CHFSI_ERR_ALLOC;
    }
    if (rc == CHFSI_SUCCESS &&
        (hipMemsetAsync(H, 0, (size_t)n * n * eb, st) != hipSuccess ||
         hipMemsetAsync(Y0, 0, (size_t)n * m * eb, st) != hipSuccess ||
         hipMemsetAsync(Y1, 0, (size_t)n * m * eb, st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
         hipEventCreate(&e1) != hipSuccess))
        rc = CHFSI_ERR_DEVICE;
    FilterStep fs = {0.5, -0.25, 0.1};
    float best = 1e30f;
    int bbm = 64, bbn = 64, bks = 1, bmode = 1;
    for (int bm : {64, 32})
        for (int bn : {64, 32})
            for (int ks : {1, 2, 4, 8, 16})
                for (int mode : {1, 2}) {
                    if (rc != CHFSI_SUCCESS) break;
                    if (ks == 1 && mode == 2) continue;
                    if (ks > 1 && n / ks < 64) continue;
                    const long tiles = (long)((n + bm - 1) / bm) * ((m + bn - 1) / bn);
                    if (mode == 2 && tiles > h->tile_cnt_len) continue;
                    GemmWs gw;
                    gw.ws = ws; gw.bytes = wsb; gw.cnt = h->tile_cnt; gw.ncnt = h->tile_cnt_len;
                    gw.plan_bm = bm; gw.plan_bn = bn; gw.plan_ksplit = ks; gw.plan_mode = mode;
                    auto step = [&]() {
                        return prec == CHFSI_FP64
                                   ? launch_filter_step_f64(st, n, m, (const zd*)H, n, (const zd*)Y0, n, (const zd*)Y1, n,
                                                            (zd*)Y1, n, fs, gw)
                                   : launch_filter_step_f32(st, n, m, (const zf*)H, n, (const zf*)Y0, n, (const zf*)Y1, n,
                                                            (zf*)Y1, n, fs, gw);
                    };
                    if (step() || step()) { rc = CHFSI_ERR_DEVICE; break; }
                    const int reps = 5;
                    (void)hipEventRecord(e0, st);
                    for (int r = 0; r < reps; ++r)
                        if (step()) rc = CHFSI_ERR_DEVICE;
                    (void)hipEventRecord(e1, st);
                    if (hipEventSynchronize(e1) != hipSuccess) { rc = CHFSI_ERR_DEVICE; break; }
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    ms /= reps;
                    if (ms < best) { best = ms; bbm = bm; bbn = bn; bks = ks; bmode = mode; }
                }
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (H) (void)hipFree(H);
    if (Y0) (void)hipFree(Y0);
    if (Y1) (void)hipFree(Y1);
    if (ws) (void)hipFree(ws);
    if (rc != CHFSI_SUCCESS) return rc;
    set_entry(h, prec, n, m, bbm, bbn, bks, bks > 1 ? bmode : 1);
    if (best_out) { best_out->bm = bbm; best_out->bn = bbn; best_out->ksplit = bks; best_out->fused = bmode == 2 && bks > 1; }
    if (best_ms) *best_ms = best;
    return CHFSI_SUCCESS;
}

}  // extern "C"
