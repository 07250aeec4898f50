// Batched solver: the k-point problems of one self-consistent cycle (Section 2.1: one generalized
// eigenproblem per k-point, all independent, of different orders) advance through Algorithm 1 in
// lockstep loops.  Each filter step of all unconverged problems is ONE persistent launch over a
// work list of output tiles of every problem; the steps of a loop are captured once in a HIP graph
// and replayed, their work lists read from a device table that is refreshed before each replay.
// The small dense steps (QR, Rayleigh-Ritz, locking, verification) stay per problem, spread over
// several streams ("lanes"), each driven by a host thread of its own: those steps wait on the host
// (eigensolver sweeps, QR pass decisions, the lock decision), so only separate threads let the
// latency-bound kernels of different problems overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

#include "chfsi.h"
#include "common.h"
#include "driver.h"
#include "gemm_tile.h"
#include "state.h"

namespace {

constexpr int BATCH_MAXP = 64;   // problems per persistent launch (larger batches are chunked)
constexpr int NUM_XCD = 8;       // gfx950: workgroup w runs on XCD w % 8
constexpr int MAX_LANES = 8;     // streams for the per-problem dense steps (default 3)

// One problem of a filter step: Yo = alpha (H Yk - shift Yk) + beta Yp on columns [0, w).  bm x bn
// is its output tile in the per-problem kernel (ignored by the one-tile kernels).
struct BatchProb {
    const zd* H;
    const zd* Yk;
    const zd* Yp;
    zd* Yo;
    int n, ldh, ldk, ldp, ldo, w, bm, bn;
    double alpha, beta, shift;
};

struct BatchStep {
    int nprob, pad[3];
    BatchProb p[BATCH_MAXP];
};

using chfsi_tile::TileShape;

// Persistent filter step over every problem of `step`.  The row tiles of each problem are cut
// into NUM_XCD equal ranges, range x going to the workgroups on XCD x, so every XCD gets an equal
// share of every problem (balanced although K = n differs between problems) and the tiles that
// share rows of H run on one XCD, close in time (neighbouring workgroups take neighbouring column
// tiles of one row panel), where they share its L2.  gridDim.x is a multiple of NUM_XCD.
template <int BM, int BN>
__global__ __launch_bounds__(256) void k_filter_batched(const BatchStep* __restrict__ step)
{
    typedef TileShape<double, BM, BN> S;
    typedef d4 ACC;
    __shared__ zd As[2 * S::AS_ELEMS];
    __shared__ zd Bs[2 * S::BS_ELEMS];
    __shared__ int pre[BATCH_MAXP + 1], r0s[BATCH_MAXP], tns[BATCH_MAXP];
    const int x = blockIdx.x % NUM_XCD, q = blockIdx.x / NUM_XCD, Q = gridDim.x / NUM_XCD;
    const int np = min(step->nprob, BATCH_MAXP);
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int p = 0; p < np; ++p) {
            const int n = step->p[p].n, w = step->p[p].w;
            const int tm = (n + BM - 1) / BM, tn = (w + BN - 1) / BN;
            const int r0 = (int)((long)x * tm / NUM_XCD), r1 = (int)((long)(x + 1) * tm / NUM_XCD);
            pre[p] = acc;
            r0s[p] = r0;
            tns[p] = tn;
            acc += (r1 - r0) * tn;
        }
        pre[np] = acc;
    }
    __syncthreads();
    const int total = pre[np];
    int p = 0;
    for (int f = q; f < total; f += Q) {
        while (pre[p + 1] <= f) ++p;
        const BatchProb b = step->p[p];
        const int loc = f - pre[p];
        const int i0 = (r0s[p] + loc / tns[p]) * BM, j0 = (loc % tns[p]) * BN;
        ACC accr[S::MI][S::NJ], acci[S::MI][S::NJ];
        chfsi_tile::tile_mainloop<double, OP_N, OP_N, BM, BN>(b.H, b.ldh, b.n, b.Yk, b.ldk, b.w, i0, j0, 0, b.n, As,
                                                              Bs, accr, acci);
#pragma unroll
        for (int bi = 0; bi < S::MI; ++bi)
#pragma unroll
            for (int bj = 0; bj < S::NJ; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = chfsi_tile::tile_row<double, BM, BN>(i0, bi);
                    const int j = chfsi_tile::tile_col<double, BM, BN>(j0, bj, r);
                    if (i < b.n && j < b.w) {
                        const zd yk = b.Yk[(size_t)i + (size_t)j * b.ldk];
                        const zd yp = b.Yp[(size_t)i + (size_t)j * b.ldp];
                        zd o;
                        o.x = b.alpha * (accr[bi][bj][r] - b.shift * yk.x) + b.beta * yp.x;
                        o.y = b.alpha * (acci[bi][bj][r] - b.shift * yk.y) + b.beta * yp.y;
                        b.Yo[(size_t)i + (size_t)j * b.ldo] = o;
                    }
                }
        __syncthreads();   // the next tile refills As/Bs
    }
}

// One output tile of problem b with the BM x BN shape (As, Bs: LDS of at least that shape's size).
template <int BM, int BN>
__device__ inline void batched_tile(const BatchProb& b, int i0, int j0, zd* As, zd* Bs)
{
    typedef TileShape<double, BM, BN> S;
    d4 accr[S::MI][S::NJ], acci[S::MI][S::NJ];
    chfsi_tile::tile_mainloop<double, OP_N, OP_N, BM, BN>(b.H, b.ldh, b.n, b.Yk, b.ldk, b.w, i0, j0, 0, b.n, As, Bs,
                                                          accr, acci);
#pragma unroll
    for (int bi = 0; bi < S::MI; ++bi)
#pragma unroll
        for (int bj = 0; bj < S::NJ; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = chfsi_tile::tile_row<double, BM, BN>(i0, bi);
                const int j = chfsi_tile::tile_col<double, BM, BN>(j0, bj, r);
                if (i < b.n && j < b.w) {
                    const zd yk = b.Yk[(size_t)i + (size_t)j * b.ldk];
                    const zd yp = b.Yp[(size_t)i + (size_t)j * b.ldp];
                    zd o;
                    o.x = b.alpha * (accr[bi][bj][r] - b.shift * yk.x) + b.beta * yp.x;
                    o.y = b.alpha * (acci[bi][bj][r] - b.shift * yk.y) + b.beta * yp.y;
                    b.Yo[(size_t)i + (size_t)j * b.ldo] = o;
                }
            }
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int AS_MAX = cmax(cmax(TileShape<double, 64, 64>::AS_ELEMS, TileShape<double, 64, 32>::AS_ELEMS),
                            cmax(TileShape<double, 32, 64>::AS_ELEMS, TileShape<double, 32, 32>::AS_ELEMS));
constexpr int BS_MAX = cmax(cmax(TileShape<double, 64, 64>::BS_ELEMS, TileShape<double, 64, 32>::BS_ELEMS),
                            cmax(TileShape<double, 32, 64>::BS_ELEMS, TileShape<double, 32, 32>::BS_ELEMS));

// Persistent filter step with a tile shape per problem (b.bm x b.bn, each 32 or 64): the same work
// list and XCD split as k_filter_batched, each problem cut into its own tiles; every work item
// runs the tile loop of its problem's shape.  LDS and registers are those of the largest shape.
__global__ __launch_bounds__(256) void k_filter_batched_mixed(const BatchStep* __restrict__ step)
{
    __shared__ zd As[2 * AS_MAX];
    __shared__ zd Bs[2 * BS_MAX];
    __shared__ int pre[BATCH_MAXP + 1], r0s[BATCH_MAXP], tns[BATCH_MAXP];
    const int x = blockIdx.x % NUM_XCD, q = blockIdx.x / NUM_XCD, Q = gridDim.x / NUM_XCD;
    const int np = min(step->nprob, BATCH_MAXP);
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int p = 0; p < np; ++p) {
            const int n = step->p[p].n, w = step->p[p].w, bm = step->p[p].bm, bn = step->p[p].bn;
            const int tm = (n + bm - 1) / bm, tn = (w + bn - 1) / bn;
            const int r0 = (int)((long)x * tm / NUM_XCD), r1 = (int)((long)(x + 1) * tm / NUM_XCD);
            pre[p] = acc;
            r0s[p] = r0;
            tns[p] = tn;
            acc += (r1 - r0) * tn;
        }
        pre[np] = acc;
    }
    __syncthreads();
    const int total = pre[np];
    int p = 0;
    for (int f = q; f < total; f += Q) {
        while (pre[p + 1] <= f) ++p;
        const BatchProb b = step->p[p];
        const int loc = f - pre[p];
        const int i0 = (r0s[p] + loc / tns[p]) * b.bm, j0 = (loc % tns[p]) * b.bn;
        if (b.bm == 64 && b.bn == 64) batched_tile<64, 64>(b, i0, j0, As, Bs);
        else if (b.bm == 64) batched_tile<64, 32>(b, i0, j0, As, Bs);
        else if (b.bn == 64) batched_tile<32, 64>(b, i0, j0, As, Bs);
        else batched_tile<32, 32>(b, i0, j0, As, Bs);
        __syncthreads();   // the next tile refills As/Bs
    }
}

template <int BM, int BN> const void* kernel_of() { return (const void*)k_filter_batched<BM, BN>; }

// bm = bn = 0 selects the per-problem kernel
const void* batched_kernel(int bm, int bn)
{
    if (bm == 0 && bn == 0) return (const void*)k_filter_batched_mixed;
    if (bm == 64 && bn == 64) return kernel_of<64, 64>();
    if (bm == 64 && bn == 32) return kernel_of<64, 32>();
    if (bm == 32 && bn == 64) return kernel_of<32, 64>();
    return kernel_of<32, 32>();
}

// persistent grid: every workgroup resident at once (CUs x occupancy), a multiple of NUM_XCD
int batched_grid(int device, int bm, int bn)
{
    int cus = 0, occ = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batched_kernel(bm, bn), 256, 0) != hipSuccess || occ <= 0)
        occ = 1;
    int g = cus * occ;
    g -= g % NUM_XCD;
    return std::max(g, NUM_XCD);
}

int launch_batched(hipStream_t s, const BatchStep* step, int bm, int bn, int grid)
{
    if (bm == 0 && bn == 0) hipLaunchKernelGGL(k_filter_batched_mixed, dim3(grid), dim3(256), 0, s, step);
    else if (bm == 64 && bn == 64) hipLaunchKernelGGL((k_filter_batched<64, 64>), dim3(grid), dim3(256), 0, s, step);
    else if (bm == 64 && bn == 32) hipLaunchKernelGGL((k_filter_batched<64, 32>), dim3(grid), dim3(256), 0, s, step);
    else if (bm == 32 && bn == 64) hipLaunchKernelGGL((k_filter_batched<32, 64>), dim3(grid), dim3(256), 0, s, step);
    else hipLaunchKernelGGL((k_filter_batched<32, 32>), dim3(grid), dim3(256), 0, s, step);
    return (int)hipGetLastError();
}

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

chfsi_status ensure_lanes(chfsi_handle h)
{
    while ((int)h->lanes.size() < MAX_LANES) {
        Lane l;
        if (hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking) != hipSuccess) return CHFSI_ERR_DEVICE;
        if (hipEventCreateWithFlags(&l.ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamDestroy(l.st);
            return CHFSI_ERR_DEVICE;
        }
        l.sub = new (std::nothrow) chfsi_handle_s();
        bool ok = l.sub != nullptr;
        if (ok) {
            l.sub->device = h->device;
            l.sub->stream = l.st;
            l.sub->fc_enabled = false;   // each problem of a batch has its own overlap
            l.sub->tile_cnt_len = 1 << 16;
            ok = hipMalloc((void**)&l.sub->tile_cnt, sizeof(int) * l.sub->tile_cnt_len) == hipSuccess;
            if (!ok) l.sub->tile_cnt = nullptr;
            ok = ok && hipMemsetAsync(l.sub->tile_cnt, 0, sizeof(int) * l.sub->tile_cnt_len, l.st) == hipSuccess &&
                 hipStreamSynchronize(l.st) == hipSuccess;
        }
        if (!ok) {
            if (l.sub && l.sub->tile_cnt) (void)hipFree(l.sub->tile_cnt);
            delete l.sub;
            (void)hipEventDestroy(l.ev);
            (void)hipStreamDestroy(l.st);
            return CHFSI_ERR_DEVICE;
        }
        h->lanes.push_back(l);
    }
    for (auto& e : h->bev)
        if (!e && hipEventCreate(&e) != hipSuccess) return CHFSI_ERR_DEVICE;
    if (!h->cap_stream && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return CHFSI_ERR_DEVICE;
    return CHFSI_SUCCESS;
}

void sync_lanes(chfsi_handle h)
{
    for (auto& l : h->lanes) (void)hipStreamSynchronize(l.st);
}

// Tile of a problem of order n and block width m in the per-problem kernel: its tuned (or set)
// entry, else the batch's one tile.
void batched_tile_of(chfsi_handle h, int n, int m, int& bm, int& bn)
{
    bm = h->batch_bm;
    bn = h->batch_bn;
    for (const auto& e : h->batch_tiles)
        if (e[0] == n && e[1] == m) { bm = e[2]; bn = e[3]; return; }
}

// Makes the step tables hold `steps` steps; a reallocation invalidates the captured graphs.
chfsi_status ensure_table(chfsi_handle h, int steps)
{
    const size_t need = sizeof(BatchStep) * (size_t)std::max(steps, 32);
    if (!h->btable_host.reserve(need)) return CHFSI_ERR_ALLOC;
    if (need <= h->btable_cap) return CHFSI_SUCCESS;
    (void)hipStreamSynchronize(h->stream);
    for (auto& g : h->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    h->graphs.clear();
    if (h->btable) (void)hipFree(h->btable);
    h->btable = nullptr;
    h->btable_cap = 0;
    if (hipMalloc(&h->btable, need) != hipSuccess) { h->btable = nullptr; return CHFSI_ERR_ALLOC; }
    h->btable_cap = need;
    return CHFSI_SUCCESS;
}

// The graph of `steps` persistent launches reading step tables 0 .. steps-1 (captured on first use).
chfsi_status get_graph(chfsi_handle h, int steps, int bm, int bn, int grid, hipGraphExec_t& exec)
{
    for (auto& g : h->graphs)
        if (g.steps == steps && g.bm == bm && g.bn == bn && g.grid == grid && g.table == h->btable) {
            exec = g.exec;
            return CHFSI_SUCCESS;
        }
    BatchGraph g;
    g.steps = steps; g.bm = bm; g.bn = bn; g.grid = grid; g.table = h->btable;
    hipStream_t st = h->cap_stream;   // nothing else is ever enqueued on it
    TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int rc = 0;
    for (int k = 0; k < steps && rc == 0; ++k)
        rc = launch_batched(st, (const BatchStep*)h->btable + k, bm, bn, grid);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    if (rc != 0 || ec != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return CHFSI_ERR_DEVICE;
    }
    if (hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return CHFSI_ERR_DEVICE;
    }
    g.graph = graph;
    h->graphs.push_back(g);
    exec = g.exec;
    return CHFSI_SUCCESS;
}

struct Slot {
    SolveState s;
    int lane = 0;
    std::vector<int> dsorted;   // degrees of the active columns in filter order
};

// One loop's filter of every slot in `act`: tables, one graph replay (or dmax launches), and the
// copy-back of columns whose degree is odd (their result sits in T).
chfsi_status batched_filter(chfsi_handle h, std::vector<Slot>& sl, const std::vector<int>& act)
{
    hipStream_t st = h->stream;
    int dmax = 0;
    for (int i : act) dmax = std::max(dmax, sl[i].dsorted.empty() ? 0 : sl[i].dsorted[0]);
    for (int i : act)
        if (sl[i].dsorted.empty()) sl[i].dsorted.push_back(0);   // no active column: no step
    if (dmax <= 0) return CHFSI_SUCCESS;
    TRYS(ensure_table(h, dmax));
    BatchStep* tab = (BatchStep*)h->btable_host.p;
    std::vector<std::vector<FilterStep>> coef(act.size());
    for (size_t u = 0; u < act.size(); ++u) {
        const SolveState& s = sl[act[u]].s;
        filter_coefficients(std::max(1, sl[act[u]].dsorted[0]), s.a, s.bb, s.mu1, coef[u]);
    }
    // step 1 of a problem whose block image H Y_0 is known (after a Rayleigh-Ritz step) needs no
    // product: it is formed elementwise before the persistent steps
    struct First {
        SolveState* s;
        int w;
        double alpha, shift;
    };
    std::vector<First> first;
    for (int k = 1; k <= dmax; ++k) {
        BatchStep& t = tab[k - 1];
        t.nprob = 0;
        for (size_t u = 0; u < act.size(); ++u) {
            Slot& z = sl[act[u]];
            SolveState& s = z.s;
            const int ma = s.ma();
            int w = 0;
            while (w < ma && z.dsorted[w] >= k) ++w;
            if (w == 0) continue;
            if (k == 1 && s.hy_off >= 0) {
                first.push_back({&s, w, coef[u][0].alpha, coef[u][0].shift});
                s.matvecs += w;   // the degree count; the flop counts hold the products performed
                continue;
            }
            // Y_k lives in Ya when k is even, in T when k is odd; Y_{k-1} in the other buffer
            zd* Ya = s.Ya();
            zd* T = s.b.T;
            BatchProb& bp = t.p[t.nprob++];
            bp.H = s.H;
            bp.ldh = s.ldh;
            bp.n = s.n;
            bp.w = w;
            batched_tile_of(h, s.n, s.m, bp.bm, bp.bn);
            bp.Yk = (k % 2 == 1) ? Ya : T;
            bp.Yo = (k % 2 == 1) ? T : Ya;
            bp.Yp = (k == 1) ? bp.Yk : bp.Yo;   // beta = 0 on step 1: any finite input
            bp.ldk = bp.ldp = bp.ldo = s.n;
            const FilterStep& fs = coef[u][k - 1];
            bp.alpha = fs.alpha;
            bp.beta = fs.beta;
            bp.shift = fs.shift;
            s.flops += 8.0 * (double)s.n * (double)s.n * (double)w;
            s.matvecs += w;
            h->batch_flops += 8.0 * (double)s.n * (double)s.n * (double)w;
        }
    }
    const int bm = h->batch_mixed ? 0 : h->batch_bm, bn = h->batch_mixed ? 0 : h->batch_bn;
    const int grid = batched_grid(h->device, bm, bn);
    TRY(hipMemcpyAsync(h->btable, tab, sizeof(BatchStep) * dmax, hipMemcpyHostToDevice, st));
    TRY(hipEventRecord(h->bev[0], st));
    for (const First& f : first) {
        SolveState& s = *f.s;
        TRY(launch_first_step(st, s.n, f.w, f.alpha, f.shift, s.b.HY + (size_t)s.hy_off * s.n, s.n, s.Ya(), s.n,
                              s.b.T, s.n));
    }
    for (int i : act) sl[i].s.hy_off = -1;
    if (h->batch_use_graph) {
        hipGraphExec_t exec = nullptr;
        TRYS(get_graph(h, dmax, bm, bn, grid, exec));
        TRY(hipGraphLaunch(exec, st));
        h->batch_graph_launches += 1;
    } else {
        for (int k = 0; k < dmax; ++k) TRY(launch_batched(st, (const BatchStep*)h->btable + k, bm, bn, grid));
    }
    h->batch_kernel_launches += dmax;
    TRY(hipEventRecord(h->bev[1], st));
    // columns whose degree is odd finished in T
    for (int i : act) {
        Slot& z = sl[i];
        SolveState& s = z.s;
        const int ma = s.ma();
        int* flag = s.h_flags();   // pinned staging [m], disjoint from the column order's
        bool any = false;
        for (int j = 0; j < ma; ++j) { flag[j] = z.dsorted[j] % 2; any |= flag[j] != 0; }
        if (!any) continue;
        TRY(hipMemcpyAsync(s.b.flag, flag, sizeof(int) * ma, hipMemcpyHostToDevice, st));
        TRY(launch_copy_cols_flag(st, s.n, ma, s.b.T, s.n, s.Ya(), s.n, s.b.flag));
    }
    return CHFSI_SUCCESS;
}

chfsi_status fail(Slot& z, chfsi_status rc)
{
    z.s.status = rc;
    z.s.done = true;
    return rc;
}

// Copies what the lane handles read from the main handle (tuned plans, degree model).
void refresh_lanes(chfsi_handle h)
{
    const int nl = std::min(h->batch_lanes, (int)h->lanes.size());
    for (int l = 0; l < nl; ++l) {
        chfsi_handle sub = h->lanes[l].sub;
        sub->plans = h->plans;
        sub->model = h->model;
        sub->has_model = h->has_model;
    }
}

// Runs step(sub, slot) for every problem in `act` through the handle of its lane (the lane's stream,
// split-K counters and pinned state), one host thread per lane when there are several: the
// per-problem phases wait on the host (the reduction's pivot check, eigensolver sweeps, QR pass
// decisions, the lock decision), so only separate threads let those of different problems overlap
// on the device.  A problem whose step fails is marked done with its status.  The main handle is
// never touched by a lane thread.
template <class F>
void run_on_lanes(chfsi_handle h, std::vector<Slot>& sl, const std::vector<int>& act,
                  std::vector<chfsi_status>& rcs, F step)
{
    const int nl = std::min(h->batch_lanes, (int)h->lanes.size());
    auto work = [&](int l) {
        chfsi_handle sub = h->lanes[l].sub;
        if (hipSetDevice(h->device) != hipSuccess) {
            for (int i : act)
                if (sl[i].lane == l) rcs[i] = fail(sl[i], CHFSI_ERR_DEVICE);
            return;
        }
        for (int i : act) {
            Slot& z = sl[i];
            if (z.lane != l || z.s.done) continue;
            try {   // nothing may escape a thread (host allocations of the steps can throw)
                const chfsi_status rc = step(sub, z);
                if (rc != CHFSI_SUCCESS) rcs[i] = fail(z, rc);
            } catch (...) {
                rcs[i] = fail(z, CHFSI_ERR_ALLOC);
            }
        }
    };
    if (nl <= 1) {
        work(0);
        return;
    }
    std::vector<std::thread> th;
    int started = 0;
    try {
        for (int l = 1; l < nl; ++l) {
            th.emplace_back(work, l);
            ++started;
        }
    } catch (...) {
        // fewer threads than lanes: the calling thread takes the lanes left over
    }
    work(0);
    for (int l = started + 1; l < nl; ++l) work(l);
    for (auto& t : th) t.join();
}

// reduction to standard form, norms and Lanczos of one problem (its lane's stream)
chfsi_status init_step(chfsi_handle sub, Slot& z)
{
    chfsi_status rc = st_init_enqueue(sub, z.s);
    if (rc == CHFSI_SUCCESS) rc = st_init_complete(sub, z.s);
    return rc;
}

// the loop's dense steps: QR, Rayleigh-Ritz, lock decision and, once nev pairs are locked, the
// verification
chfsi_status loop_step(chfsi_handle sub, Slot& z)
{
    chfsi_status rc = st_loop_enqueue(sub, z.s);
    if (rc != CHFSI_SUCCESS || z.s.done) return rc;
    rc = st_loop_complete(sub, z.s);
    if (rc == CHFSI_SUCCESS && z.s.want_final) rc = st_final_enqueue(sub, z.s);
    if (rc != CHFSI_SUCCESS || z.s.done || !z.s.want_final) return rc;
    return st_final_complete(sub, z.s);
}

chfsi_status solve_chunk(chfsi_handle h, int count, const chfsi_problem* probs, const chfsi_params& base,
                         chfsi_stats* stats, int first_index)
{
    std::vector<Slot> sl(count);
    std::vector<chfsi_status> rcs(count, CHFSI_SUCCESS);
    if ((int)h->barena.size() < first_index + count) {
        h->barena.resize(first_index + count);
        h->bpin.resize(first_index + count);
    }
    const int nl = std::max(1, std::min(h->batch_lanes, (int)h->lanes.size()));
    refresh_lanes(h);
    auto t0 = std::chrono::steady_clock::now();
    // buffers of every problem (one arena and one pinned staging buffer each), then the initial
    // phases (reduction, Lanczos) on the problems' lanes
    std::vector<int> all;
    for (int i = 0; i < count; ++i) {
        const chfsi_problem& q = probs[i];
        chfsi_params pk = base;
        pk.nev = q.nev;
        pk.nex = q.nex;
        Slot& z = sl[i];
        z.lane = i % nl;
        chfsi_status rc = st_define(z.s, q.n, (const zd*)q.A, q.lda, (const zd*)q.S, q.lds, (zd*)q.X, q.ldx,
                                    q.x_is_guess, q.lambda, q.resid, pk);
        if (rc == CHFSI_SUCCESS) rc = st_setup(h, z.s, h->barena[first_index + i], h->bpin[first_index + i]);
        if (rc == CHFSI_SUCCESS) {   // split-K counters of the problem's lane
            z.s.b.gw.cnt = h->lanes[z.lane].sub->tile_cnt;
            z.s.b.gw.ncnt = h->lanes[z.lane].sub->tile_cnt_len;
            all.push_back(i);
        } else {
            rcs[i] = fail(z, rc);
        }
    }
    // the arenas may have been (re)allocated: nothing of them is in flight on any stream
    run_on_lanes(h, sl, all, rcs, init_step);
    for (;;) {
        std::vector<int> act;
        for (int i = 0; i < count; ++i)
            if (!sl[i].s.done && sl[i].s.loops < sl[i].s.p.max_loops) act.push_back(i);
        if (act.empty()) break;
        // column order by degree on each problem's lane, then the lanes join the main stream
        for (int i : act) {
            const chfsi_status rc = st_order_columns(h->lanes[sl[i].lane].sub, sl[i].s, sl[i].dsorted);
            if (rc != CHFSI_SUCCESS) return rc;
        }
        for (auto& l : h->lanes) {
            TRY(hipEventRecord(l.ev, l.st));
            TRY(hipStreamWaitEvent(h->stream, l.ev, 0));
        }
        TRYS(batched_filter(h, sl, act));
        TRY(hipEventRecord(h->bev[2], h->stream));
        for (auto& l : h->lanes) TRY(hipStreamWaitEvent(l.st, h->bev[2], 0));
        // QR, Rayleigh-Ritz, the host decisions and the verification of every problem
        run_on_lanes(h, sl, act, rcs, loop_step);
        float ms = 0;
        if (hipEventElapsedTime(&ms, h->bev[0], h->bev[1]) == hipSuccess) h->batch_filter_ms += ms;
    }
    chfsi_status first = CHFSI_SUCCESS;
    for (int i = 0; i < count; ++i) {
        Slot& z = sl[i];
        chfsi_stats stt;
        std::memset(&stt, 0, sizeof(stt));
        if (rcs[i] == CHFSI_SUCCESS || rcs[i] == CHFSI_ERR_NUMERIC) st_finish(h->lanes[z.lane].sub, z.s, stt);
        else stt.status = rcs[i];
        const chfsi_status si = rcs[i] == CHFSI_SUCCESS ? z.s.status : rcs[i];
        stt.status = si;
        if (stats) stats[i] = stt;
        if (si != CHFSI_SUCCESS && first == CHFSI_SUCCESS) first = si;
    }
    for (auto& l : h->lanes) TRY(hipStreamSynchronize(l.st));
    const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats)
        for (int i = 0; i < count; ++i) stats[i].t_total = wall;
    return first;
}

}  // namespace

extern "C" {

chfsi_status chfsi_solve_batched(chfsi_handle h, int count, const chfsi_problem* probs, const chfsi_params* p,
                                 chfsi_stats* stats)
{
    if (!h || count < 0 || (count > 0 && !probs)) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    chfsi_params base;
    if (p) base = *p; else chfsi_default_params(&base);
    if (base.filter_precision != CHFSI_FP64) return CHFSI_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        const chfsi_problem& q = probs[i];
        if (q.n <= 0 || q.nev <= 0 || q.nex < 0 || q.nev + q.nex > q.n) return CHFSI_ERR_ARG;
    }
    h->batch_filter_ms = 0;
    h->batch_flops = 0;
    h->batch_graph_launches = 0;
    h->batch_kernel_launches = 0;
    if (count == 0) return CHFSI_SUCCESS;
    TRYS(ensure_lanes(h));
    TRY(hipStreamSynchronize(h->stream));
    chfsi_status first = CHFSI_SUCCESS;
    for (int c0 = 0; c0 < count; c0 += BATCH_MAXP) {
        const int c = std::min(BATCH_MAXP, count - c0);
        const chfsi_status s = solve_chunk(h, c, probs + c0, base, stats ? stats + c0 : nullptr, c0);
        sync_lanes(h);
        if (s != CHFSI_SUCCESS && first == CHFSI_SUCCESS) first = s;
    }
    TRY(hipStreamSynchronize(h->stream));
    return first;
}

chfsi_status chfsi_set_batched_plan(chfsi_handle h, const chfsi_tile_plan* plan, int use_graph, int lanes)
{
    if (!h || lanes < 0 || lanes > MAX_LANES) return CHFSI_ERR_ARG;
    if (lanes > 0) h->batch_lanes = lanes;
    if (plan) {
        if ((plan->bm != 32 && plan->bm != 64) || (plan->bn != 32 && plan->bn != 64)) return CHFSI_ERR_ARG;
        h->batch_bm = plan->bm;
        h->batch_bn = plan->bn;
        h->batch_mixed = false;
    }
    h->batch_use_graph = use_graph != 0;
    return CHFSI_SUCCESS;
}

}  // extern "C"

namespace {

// Checks the problems of a tuning call and builds a one-step table over all of them (scratch
// outputs in *out, one n x m block per problem, freed by the caller).
chfsi_status tune_setup(chfsi_handle h, int count, const chfsi_problem* probs, BatchStep& tab, zd** out)
{
    *out = nullptr;
    if (!h || count <= 0 || count > BATCH_MAXP || !probs) return CHFSI_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        const chfsi_problem& q = probs[i];
        if (q.n <= 0 || q.nev <= 0 || q.nex < 0 || q.nev + q.nex > q.n || !q.A || !q.X || q.lda < q.n ||
            q.ldx < q.n)
            return CHFSI_ERR_ARG;
    }
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    TRYS(ensure_lanes(h));
    TRYS(ensure_table(h, 1));
    std::vector<size_t> off(count);
    size_t tot = 0;
    for (int i = 0; i < count; ++i) {
        off[i] = tot;
        tot += (size_t)probs[i].n * (probs[i].nev + probs[i].nex);
    }
    if (hipMalloc((void**)out, sizeof(zd) * tot) != hipSuccess) { *out = nullptr; return CHFSI_ERR_ALLOC; }
    tab.nprob = count;
    for (int i = 0; i < count; ++i) {
        const chfsi_problem& q = probs[i];
        BatchProb& bp = tab.p[i];
        bp.H = (const zd*)q.A;
        bp.ldh = q.lda;
        bp.n = q.n;
        bp.w = q.nev + q.nex;
        bp.bm = h->batch_bm;
        bp.bn = h->batch_bn;
        bp.Yk = (const zd*)q.X;
        bp.ldk = q.ldx;
        bp.Yp = (const zd*)q.X;
        bp.ldp = q.ldx;
        bp.Yo = *out + off[i];
        bp.ldo = q.n;
        bp.alpha = 1e-3;
        bp.beta = -0.5;
        bp.shift = 0.1;
    }
    return CHFSI_SUCCESS;
}

// ms per launch of the step table in device slot 0 with tile bm x bn (0 x 0: per problem),
// after two warm-up launches; negative on a device error
double time_table(chfsi_handle h, int bm, int bn)
{
    hipStream_t st = h->stream;
    const int grid = batched_grid(h->device, bm, bn);
    for (int w = 0; w < 2; ++w)
        if (launch_batched(st, (const BatchStep*)h->btable, bm, bn, grid) != 0) return -1.0;
    (void)hipEventRecord(h->bev[0], st);
    for (int r = 0; r < 5; ++r)
        if (launch_batched(st, (const BatchStep*)h->btable, bm, bn, grid) != 0) return -1.0;
    (void)hipEventRecord(h->bev[1], st);
    if (hipEventSynchronize(h->bev[1]) != hipSuccess) return -1.0;
    float ms = 0;
    if (hipEventElapsedTime(&ms, h->bev[0], h->bev[1]) != hipSuccess) return -1.0;
    return ms / 5;
}

void set_tile_entry(chfsi_handle h, int n, int m, int bm, int bn)
{
    for (auto& e : h->batch_tiles)
        if (e[0] == n && e[1] == m) { e[2] = bm; e[3] = bn; return; }
    h->batch_tiles.push_back({n, m, bm, bn});
}

const int TILE_CAND[4][2] = {{64, 64}, {64, 32}, {32, 64}, {32, 32}};

}  // namespace

extern "C" {

chfsi_status chfsi_autotune_batched(chfsi_handle h, int count, const chfsi_problem* probs, chfsi_tile_plan* best,
                                    double* best_ms)
{
    if (!h) return CHFSI_ERR_ARG;
    std::unique_ptr<BatchStep> tab(new (std::nothrow) BatchStep());
    if (!tab) return CHFSI_ERR_ALLOC;
    zd* out = nullptr;
    TRYS(tune_setup(h, count, probs, *tab, &out));
    chfsi_status rc = CHFSI_SUCCESS;
    if (hipMemcpy(h->btable, tab.get(), sizeof(BatchStep), hipMemcpyHostToDevice) != hipSuccess) rc = CHFSI_ERR_DEVICE;
    double bms = 1e30;
    int bi = 0;
    for (int c = 0; c < 4 && rc == CHFSI_SUCCESS; ++c) {
        const double ms = time_table(h, TILE_CAND[c][0], TILE_CAND[c][1]);
        if (ms < 0) rc = CHFSI_ERR_DEVICE;
        else if (ms < bms) { bms = ms; bi = c; }
    }
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(out);
    if (rc != CHFSI_SUCCESS) return rc;
    h->batch_bm = TILE_CAND[bi][0];
    h->batch_bn = TILE_CAND[bi][1];
    h->batch_mixed = false;
    if (best) { best->bm = h->batch_bm; best->bn = h->batch_bn; best->ksplit = 1; best->fused = 0; }
    if (best_ms) *best_ms = bms;
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_autotune_batched_tiles(chfsi_handle h, int count, const chfsi_problem* probs,
                                          chfsi_tile_plan* tiles, double* batch_ms)
{
    if (!h) return CHFSI_ERR_ARG;
    std::unique_ptr<BatchStep> tab(new (std::nothrow) BatchStep());
    if (!tab) return CHFSI_ERR_ALLOC;
    zd* out = nullptr;
    TRYS(tune_setup(h, count, probs, *tab, &out));
    chfsi_status rc = CHFSI_SUCCESS;
    auto upload = [&]() {
        return hipMemcpy(h->btable, tab.get(), sizeof(BatchStep), hipMemcpyHostToDevice) == hipSuccess;
    };
    // 1. the whole batch with each one-tile kernel
    double uni_ms = 1e30;
    int ui = 0;
    if (!upload()) rc = CHFSI_ERR_DEVICE;
    for (int c = 0; c < 4 && rc == CHFSI_SUCCESS; ++c) {
        const double ms = time_table(h, TILE_CAND[c][0], TILE_CAND[c][1]);
        if (ms < 0) rc = CHFSI_ERR_DEVICE;
        else if (ms < uni_ms) { uni_ms = ms; ui = c; }
    }
    // 2. the kernel with a tile per problem, from the best one tile: the problems ordered by n cut
    //    into four groups, each group trying every shape with the others fixed, timed on the batch
    std::vector<int> shape(count, ui), ord(count);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return probs[a].n < probs[b].n; });
    auto apply = [&]() {
        for (int i = 0; i < count; ++i) { tab->p[i].bm = TILE_CAND[shape[i]][0]; tab->p[i].bn = TILE_CAND[shape[i]][1]; }
    };
    double mix_ms = -1.0;
    if (rc == CHFSI_SUCCESS) {
        apply();
        if (!upload() || (mix_ms = time_table(h, 0, 0)) < 0) rc = CHFSI_ERR_DEVICE;
    }
    const int groups = std::min(4, count);
    for (int gi = 0; gi < groups && rc == CHFSI_SUCCESS; ++gi) {
        const int lo = gi * count / groups, hi = (gi + 1) * count / groups;
        const int keep = shape[ord[lo]];
        int best_c = keep;
        for (int c = 0; c < 4 && rc == CHFSI_SUCCESS; ++c) {
            if (c == keep) continue;
            for (int k = lo; k < hi; ++k) shape[ord[k]] = c;
            apply();
            double ms = -1.0;
            if (!upload() || (ms = time_table(h, 0, 0)) < 0) { rc = CHFSI_ERR_DEVICE; break; }
            if (ms < mix_ms) { mix_ms = ms; best_c = c; }
        }
        for (int k = lo; k < hi; ++k) shape[ord[k]] = best_c;
    }
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(out);
    if (rc != CHFSI_SUCCESS) return rc;
    // 3. the faster of the two kernels serves later solves
    const bool mixed = mix_ms < uni_ms;
    h->batch_bm = TILE_CAND[ui][0];
    h->batch_bn = TILE_CAND[ui][1];
    for (int i = 0; i < count; ++i) {
        const int c = mixed ? shape[i] : ui;
        set_tile_entry(h, probs[i].n, probs[i].nev + probs[i].nex, TILE_CAND[c][0], TILE_CAND[c][1]);
        if (tiles) { tiles[i].bm = TILE_CAND[c][0]; tiles[i].bn = TILE_CAND[c][1]; tiles[i].ksplit = 1; tiles[i].fused = 0; }
    }
    h->batch_mixed = mixed;
    if (batch_ms) *batch_ms = mixed ? mix_ms : uni_ms;
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_set_batched_tiles(chfsi_handle h, int count, const chfsi_problem* probs,
                                     const chfsi_tile_plan* tiles)
{
    if (!h) return CHFSI_ERR_ARG;
    if (!tiles) {
        h->batch_tiles.clear();
        h->batch_mixed = false;
        return CHFSI_SUCCESS;
    }
    if (count <= 0 || !probs) return CHFSI_ERR_ARG;
    for (int i = 0; i < count; ++i)
        if ((tiles[i].bm != 32 && tiles[i].bm != 64) || (tiles[i].bn != 32 && tiles[i].bn != 64) || probs[i].n <= 0 ||
            probs[i].nev <= 0 || probs[i].nex < 0)
            return CHFSI_ERR_ARG;
    for (int i = 0; i < count; ++i) set_tile_entry(h, probs[i].n, probs[i].nev + probs[i].nex, tiles[i].bm, tiles[i].bn);
    h->batch_mixed = true;
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_batched_info(chfsi_handle h, double* filter_ms, double* filter_flops, int* graph_launches,
                                int* kernel_launches)
{
    if (!h) return CHFSI_ERR_ARG;
    if (filter_ms) *filter_ms = h->batch_filter_ms;
    if (filter_flops) *filter_flops = h->batch_flops;
    if (graph_launches) *graph_launches = h->batch_graph_launches;
    if (kernel_launches) *kernel_launches = h->batch_kernel_launches;
    return CHFSI_SUCCESS;
}

}  // extern "C"
