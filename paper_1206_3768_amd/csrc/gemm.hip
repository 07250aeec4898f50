// Complex GEMM on CDNA4 matrix cores, with the Chebyshev three-term recurrence fused into the
// epilogue (Algorithm 1, filtering step: Y_{k+1} = alpha (H - cI) Y_k + beta Y_{k-1}).
//
// The MFMA tile itself (operand staging, transposed complex MFMA) lives in gemm_tile.h.  Tiles
// are enumerated so that consecutive tiles (same rows of A, neighbouring column tiles) land on the
// same XCD: the hardware hands workgroup w to XCD w % 8.  Split-K writes partial tiles to a
// workspace; the last K-slice to finish a tile sums the partials in slice order (deterministic)
// and applies the epilogue, so one launch is one filter step.
#include "common.h"
#include "gemm_tile.h"

namespace {

using chfsi_tile::CT;
using chfsi_tile::TileShape;

enum { EPI_GEMM = 0, EPI_FILTER = 1 };

// scalar arguments (pointers are passed as separate kernel arguments)
struct GDims {
    int M, N, K;
    int lda, ldb, ldc, ldyk, ldyp;
    double alpha, beta, shift;
    int kchunk, tiles_m, tiles_n, ksplit;
    int tri;   // TRI_* flags (single K slice only)
};

// logical tile of workgroup w such that each XCD owns one contiguous range of tiles
__device__ __forceinline__ int xcd_remap(int w, int nt)
{
    const int X = 8;
    const int per = nt / X, rem = nt % X;
    const int x = w % X, q = w / X;
    return x * per + (x < rem ? x : rem) + q;
}

template <typename T, int EPI>
__device__ __forceinline__ void epilogue_store(const GDims& g, typename CT<T>::c* C,
                                               const typename CT<T>::c* Yk, const typename CT<T>::c* Yp,
                                               int i, int j, T vr, T vi)
{
    typedef typename CT<T>::c C2;
    if (EPI == EPI_GEMM) {
        const T al = (T)g.alpha, be = (T)g.beta;
        C2 o;
        o.x = al * vr;
        o.y = al * vi;
        if (g.beta != 0.0) {
            const C2 c = C[(size_t)i + (size_t)j * g.ldc];
            o.x += be * c.x;
            o.y += be * c.y;
        }
        C[(size_t)i + (size_t)j * g.ldc] = o;
    } else {
        const T al = (T)g.alpha, be = (T)g.beta, sh = (T)g.shift;
        const C2 yk = Yk[(size_t)i + (size_t)j * g.ldyk];
        const C2 yp = Yp[(size_t)i + (size_t)j * g.ldyp];
        C2 o;
        o.x = al * (vr - sh * yk.x) + be * yp.x;
        o.y = al * (vi - sh * yk.y) + be * yp.y;
        C[(size_t)i + (size_t)j * g.ldc] = o;
    }
}

// MODE 0: one K-slice, the epilogue is applied directly.
// MODE 1: this launch is one of ksplit K-slices of each output tile and only writes its partial
//         tile; k_splitk_reduce (the next launch on the stream) sums the partials in slice order.
// MODE 2: as 1, but the last slice to arrive (per-tile counter) sums the partials in slice order
//         and applies the epilogue, then clears the counter.  Needs device-scope fences (an L2
//         write-back per workgroup on gfx950), so it pays off only for few, long K-slices.
// Every mode sums in a fixed order, so results do not depend on the arrival order.
template <typename T, int OPA, int OPB, int EPI, int BM, int BN, int MODE>
__global__ __launch_bounds__(256) void k_zgemm(GDims g, const typename CT<T>::c* __restrict__ A,
                                               const typename CT<T>::c* __restrict__ B, typename CT<T>::c* C,
                                               const typename CT<T>::c* Yk, const typename CT<T>::c* Yp,
                                               typename CT<T>::c* __restrict__ P, int* __restrict__ cnt)
{
    typedef typename CT<T>::c C2;
    typedef typename CT<T>::acc ACC;
    typedef TileShape<T, BM, BN> S;
    __shared__ C2 As[2 * S::AS_ELEMS];
    __shared__ C2 Bs[2 * S::BS_ELEMS];
    constexpr int MI = S::MI, NJ = S::NJ;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int it, jt, ks;
    if (g.tri & TRI_C_LOWER) {
        // tiles on or below the diagonal only (BM == BN), row by row: tile t is (it, jt) with
        // t = it (it + 1) / 2 + jt, jt <= it
        const int nt = g.tiles_m * (g.tiles_m + 1) / 2;
        int tile = xcd_remap(blockIdx.x, nt);
        // op(B) upper triangular: the work grows with jt, the last rows' tiles go out first
        if (g.tri & TRI_B_UPPER) tile = nt - 1 - tile;
        int r = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
        while (r * (r + 1) / 2 > tile) --r;
        while ((r + 1) * (r + 2) / 2 <= tile) ++r;
        it = r;
        jt = tile - r * (r + 1) / 2;
        ks = 0;
    } else {
        const int nt = g.tiles_m * g.tiles_n * g.ksplit;
        const int tile = xcd_remap(blockIdx.x, nt);
        // tile order (ks, it, jt), jt fastest: the contiguous range of tiles that one XCD receives
        // covers one K slice, so that the XCD's L2 holds only that slice of op(B) (and the column
        // tiles of one row block share its op(A) panel)
        jt = tile % g.tiles_n;
        const int r1 = tile / g.tiles_n;
        it = r1 % g.tiles_m;
        ks = r1 / g.tiles_m;
        // op(A) lower triangular: the row tile's work grows with it, the longest go out first
        if (g.tri & TRI_A_LOWER) it = g.tiles_m - 1 - it;
    }
    const int i0 = it * BM, j0 = jt * BN;
    int kb = ks * g.kchunk;
    int ke = min(g.K, kb + g.kchunk);
    // op(B) zero in the rows above the 64-block after the output column's: the products start there
    if (g.tri & TRI_B_BLOCK_LOWER) kb = max(kb, ((j0 >> 6) + 1) << 6);
    // op(A) zero right of the diagonal, op(B) zero below it: the products end at the tile's last
    // row (column)
    if (g.tri & TRI_A_LOWER) ke = min(ke, i0 + BM);
    if (g.tri & TRI_B_UPPER) ke = min(ke, j0 + BN);
    const int wr = (wave & 1) * (BM / 2), wc = (wave >> 1) * (BN / 2);

    ACC accr[MI][NJ], acci[MI][NJ];
    chfsi_tile::tile_mainloop<T, OPA, OPB, BM, BN>(A, g.lda, g.M, B, g.ldb, g.N, i0, j0, kb, ke, As, Bs, accr, acci);

    if (MODE == 0) {
#pragma unroll
        for (int bi = 0; bi < MI; ++bi)
#pragma unroll
            for (int bj = 0; bj < NJ; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + wr + bi * 16 + (lane & 15);
                    const int j = j0 + wc + bj * 16 + chfsi_tile::drow(T(0), lane, r);
                    if (i < g.M && j < g.N) epilogue_store<T, EPI>(g, C, Yk, Yp, i, j, accr[bi][bj][r], acci[bi][bj][r]);
                }
        return;
    }
    // split-K: publish this slice's partial tile
    const size_t slab = (size_t)g.M * g.N;
#pragma unroll
    for (int bi = 0; bi < MI; ++bi)
#pragma unroll
        for (int bj = 0; bj < NJ; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wr + bi * 16 + (lane & 15);
                const int j = j0 + wc + bj * 16 + chfsi_tile::drow(T(0), lane, r);
                if (i < g.M && j < g.N) {
                    C2 o;
                    o.x = accr[bi][bj][r];
                    o.y = acci[bi][bj][r];
                    P[(size_t)ks * slab + (size_t)i + (size_t)j * g.M] = o;
                }
            }
    if (MODE == 1) return;
    __threadfence();
    __shared__ int s_last;
    __syncthreads();
    if (tid == 0) {
        const int old = atomicAdd(&cnt[it * g.tiles_n + jt], 1);
        s_last = (old == g.ksplit - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
#pragma unroll
    for (int bi = 0; bi < MI; ++bi)
#pragma unroll
        for (int bj = 0; bj < NJ; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wr + bi * 16 + (lane & 15);
                const int j = j0 + wc + bj * 16 + chfsi_tile::drow(T(0), lane, r);
                if (i < g.M && j < g.N) {
                    T vr = 0, vi = 0;
                    for (int s = 0; s < g.ksplit; ++s) {
                        const C2 p = P[(size_t)s * slab + (size_t)i + (size_t)j * g.M];
                        vr += p.x;
                        vi += p.y;
                    }
                    epilogue_store<T, EPI>(g, C, Yk, Yp, i, j, vr, vi);
                }
            }
    if (tid == 0) cnt[it * g.tiles_n + jt] = 0;
}

// Sums the ksplit partial tiles written by a MODE 1 launch in slice order and applies the epilogue.
template <typename T, int EPI>
__global__ __launch_bounds__(256) void k_splitk_reduce(GDims g, typename CT<T>::c* C, const typename CT<T>::c* Yk,
                                                       const typename CT<T>::c* Yp,
                                                       const typename CT<T>::c* __restrict__ P)
{
    typedef typename CT<T>::c C2;
    const size_t slab = (size_t)g.M * g.N;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < slab; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % g.M), j = (int)(e / g.M);
        T vr = 0, vi = 0;
        for (int s = 0; s < g.ksplit; ++s) {
            const C2 p = P[(size_t)s * slab + e];
            vr += p.x;
            vi += p.y;
        }
        epilogue_store<T, EPI>(g, C, Yk, Yp, i, j, vr, vi);
    }
}

struct Plan { int bm, bn, ksplit, kchunk, tiles_m, tiles_n, mode; };

// Tile/split choice.  A plan forced by the caller (autotuned) wins if the workspace allows it.
// Otherwise the largest tile (64 x 64, 64 x 32 / 32 x 64, 32 x 32; no 64-wide side on a dimension
// of 32 or less) that still gives one workgroup per CU (256 CUs), else 32 x 32; then K slices of at least 64 until there are two workgroups per
// CU, the partials summed by a second kernel.  Small products (the Gram matrices and rotations of
// the dense steps) would otherwise run on a fraction of the CUs.
Plan make_plan(int M, int N, int K, const GemmWs& gw, int elem_bytes)
{
    constexpr long CUS = 256;
    Plan p;
    int ks = 1;
    p.mode = 1;
    const bool forced = gw.plan_bm > 0;
    if (forced) {
        p.bm = gw.plan_bm;
        p.bn = gw.plan_bn;
        ks = gw.plan_ksplit > 0 ? gw.plan_ksplit : 1;
        p.mode = gw.plan_mode;
    } else {
        auto count = [&](int bm, int bn) { return (long)((M + bm - 1) / bm) * ((N + bn - 1) / bn); };
        const bool wide_m = M > 32, wide_n = N > 32;   // a 64-wide side would be half empty otherwise
        p.bm = 32;
        p.bn = 32;
        if (wide_m && wide_n && count(64, 64) >= CUS) { p.bm = 64; p.bn = 64; }
        else if (wide_m && (M >= N || !wide_n) && count(64, 32) >= CUS) { p.bm = 64; p.bn = 32; }
        else if (wide_n && (N > M || !wide_m) && count(32, 64) >= CUS) { p.bm = 32; p.bn = 64; }
    }
    p.tiles_m = (M + p.bm - 1) / p.bm;
    p.tiles_n = (N + p.bn - 1) / p.bn;
    const long tiles = (long)p.tiles_m * p.tiles_n;
    if (!forced)
        while (tiles * ks < 2 * CUS && (long)K / (2 * ks) >= 64) ks *= 2;
    if (!gw.ws || (p.mode == 2 && (!gw.cnt || tiles > gw.ncnt))) ks = 1;
    while (ks > 1 && (size_t)ks * M * N * (size_t)elem_bytes > gw.bytes) ks /= 2;
    int kc = (K + ks - 1) / ks;
    kc = (kc + 15) / 16 * 16;
    p.kchunk = kc > 0 ? kc : 16;
    p.ksplit = K > 0 ? (K + p.kchunk - 1) / p.kchunk : 1;
    if (p.ksplit <= 1) p.mode = 0;
    return p;
}

template <typename T, int OPA, int OPB, int EPI, int BM, int BN>
void launch_tile(hipStream_t s, hipEvent_t e0, hipEvent_t e1, int nt, int mode, const GDims& g,
                 const typename CT<T>::c* A, const typename CT<T>::c* B, typename CT<T>::c* C,
                 const typename CT<T>::c* Yk, const typename CT<T>::c* Yp, typename CT<T>::c* P, int* cnt)
{
    if (mode == 0)
        launch_timed(k_zgemm<T, OPA, OPB, EPI, BM, BN, 0>, dim3(nt), dim3(256), s, e0, e1, g, A, B, C, Yk, Yp, P, cnt);
    else if (mode == 1)
        launch_timed(k_zgemm<T, OPA, OPB, EPI, BM, BN, 1>, dim3(nt), dim3(256), s, e0, e1, g, A, B, C, Yk, Yp, P, cnt);
    else
        launch_timed(k_zgemm<T, OPA, OPB, EPI, BM, BN, 2>, dim3(nt), dim3(256), s, e0, e1, g, A, B, C, Yk, Yp, P, cnt);
}

template <typename T, int OPA, int OPB, int EPI>
int run(hipStream_t s, GDims g, const Plan& p, const typename CT<T>::c* A, const typename CT<T>::c* B,
        typename CT<T>::c* C, const typename CT<T>::c* Yk, const typename CT<T>::c* Yp, const GemmWs& gw)
{
    g.kchunk = p.kchunk; g.tiles_m = p.tiles_m; g.tiles_n = p.tiles_n; g.ksplit = p.ksplit;
    const int nt = (g.tri & TRI_C_LOWER) ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n * p.ksplit;
    if (gw.plan_used) {
        gw.plan_used[0] = p.bm; gw.plan_used[1] = p.bn; gw.plan_used[2] = p.ksplit; gw.plan_used[3] = p.mode;
    }
    const bool timed = gw.ev_start && gw.ev_main && gw.ev_end;
    if (nt <= 0) {
        if (timed) {
            (void)hipEventRecord(gw.ev_start, s);
            (void)hipEventRecord(gw.ev_main, s);
            (void)hipEventRecord(gw.ev_end, s);
        }
        return 0;
    }
    typedef typename CT<T>::c C2;
    C2* P = (C2*)gw.ws;
    const hipEvent_t e0 = timed ? gw.ev_start : nullptr, e1 = timed ? gw.ev_main : nullptr;
    if (p.bm == 64 && p.bn == 64) launch_tile<T, OPA, OPB, EPI, 64, 64>(s, e0, e1, nt, p.mode, g, A, B, C, Yk, Yp, P, gw.cnt);
    else if (p.bm == 64) launch_tile<T, OPA, OPB, EPI, 64, 32>(s, e0, e1, nt, p.mode, g, A, B, C, Yk, Yp, P, gw.cnt);
    else if (p.bn == 64) launch_tile<T, OPA, OPB, EPI, 32, 64>(s, e0, e1, nt, p.mode, g, A, B, C, Yk, Yp, P, gw.cnt);
    else launch_tile<T, OPA, OPB, EPI, 32, 32>(s, e0, e1, nt, p.mode, g, A, B, C, Yk, Yp, P, gw.cnt);
    if (p.mode == 1) {
        const size_t total = (size_t)g.M * g.N;
        int blocks = (int)((total + 255) / 256);
        if (blocks > 4096) blocks = 4096;
        launch_timed(k_splitk_reduce<T, EPI>, dim3(blocks), dim3(256), s, nullptr, timed ? gw.ev_end : nullptr, g, C,
                     Yk, Yp, P);
    } else if (timed) {
        (void)hipEventRecord(gw.ev_end, s);
    }
    return (int)hipGetLastError();
}

}  // namespace

// C = alpha op(A) op(B) + beta C restricted by the TRI_* flags (one K slice, no workspace):
//  TRI_C_LOWER        only the output tiles on or below the diagonal (M == N); the diagonal tiles
//                     are computed whole, so entries just above the diagonal may be written too
//  TRI_B_BLOCK_LOWER  op(B) is zero above its block diagonal of 64 x 64 blocks and below it only
//                     strictly: column block c of op(B) is nonzero in rows >= 64 (c + 1) only, and
//                     the rows above are never read
//  TRI_A_LOWER        op(A) is lower triangular (K == M): its entries right of the diagonal are
//                     taken as zero (a tile's products end at its last row)
//  TRI_B_UPPER        op(B) is upper triangular (K == N): its entries below the diagonal are taken
//                     as zero
int launch_zgemm_tri(hipStream_t s, int tri, int opa, int opb, int M, int N, int K, double alpha, const zd* A,
                     int lda, const zd* B, int ldb, double beta, zd* C, int ldc)
{
    if (M <= 0 || N <= 0) return 0;
    if ((tri & TRI_C_LOWER) && M != N) return (int)hipErrorInvalidValue;
    GDims g = {};
    g.M = M; g.N = N; g.K = K; g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.alpha = alpha; g.beta = beta;
    g.tri = tri;
    Plan p;
    p.mode = 0;
    p.ksplit = 1;
    p.kchunk = K > 0 ? K : 16;
    auto count = [&](int b) {
        const long tm = (M + b - 1) / b, tn = (N + b - 1) / b;
        return (tri & TRI_C_LOWER) ? tm * (tm + 1) / 2 : tm * tn;
    };
    p.bm = p.bn = (M > 32 && N > 32 && count(64) >= 256) ? 64 : 32;
    p.tiles_m = (M + p.bm - 1) / p.bm;
    p.tiles_n = (N + p.bn - 1) / p.bn;
    GemmWs none;
    if (opa == OP_N && opb == OP_N) return run<double, OP_N, OP_N, EPI_GEMM>(s, g, p, A, B, C, nullptr, nullptr, none);
    if (opa == OP_N && opb == OP_C) return run<double, OP_N, OP_C, EPI_GEMM>(s, g, p, A, B, C, nullptr, nullptr, none);
    return (int)hipErrorInvalidValue;
}

size_t zgemm_ws_bytes(int M, int N, int K, int elem_bytes)
{
    GemmWs probe;
    probe.ws = (void*)1;
    probe.bytes = (size_t)-1;
    probe.cnt = (int*)1;
    probe.ncnt = 1 << 30;
    Plan p = make_plan(M, N, K, probe, elem_bytes);
    return (size_t)p.ksplit * M * N * elem_bytes;
}

int launch_zgemm(hipStream_t s, int opa, int opb, int M, int N, int K, double alpha, const zd* A, int lda,
                 const zd* B, int ldb, double beta, zd* C, int ldc, const GemmWs& gw)
{
    if (M <= 0 || N <= 0) return 0;
    GDims g = {};
    g.M = M; g.N = N; g.K = K; g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.alpha = alpha; g.beta = beta;
    Plan p = make_plan(M, N, K, gw, 16);
    if (opa == OP_N && opb == OP_N) return run<double, OP_N, OP_N, EPI_GEMM>(s, g, p, A, B, C, nullptr, nullptr, gw);
    if (opa == OP_C && opb == OP_N) return run<double, OP_C, OP_N, EPI_GEMM>(s, g, p, A, B, C, nullptr, nullptr, gw);
    if (opa == OP_N && opb == OP_C) return run<double, OP_N, OP_C, EPI_GEMM>(s, g, p, A, B, C, nullptr, nullptr, gw);
    return run<double, OP_C, OP_C, EPI_GEMM>(s, g, p, A, B, C, nullptr, nullptr, gw);
}

int launch_filter_step_f64(hipStream_t s, int n, int ncols, const zd* H, int ldh, const zd* Yk, int ldyk,
                           const zd* Yprev, int ldyp, zd* Yout, int ldyo, FilterStep fs, const GemmWs& gw)
{
    if (n <= 0 || ncols <= 0) return 0;
    GDims g = {};
    g.M = n; g.N = ncols; g.K = n; g.lda = ldh; g.ldb = ldyk; g.ldc = ldyo; g.ldyk = ldyk; g.ldyp = ldyp;
    g.alpha = fs.alpha; g.beta = fs.beta; g.shift = fs.shift;
    Plan p = make_plan(n, ncols, n, gw, 16);
    return run<double, OP_N, OP_N, EPI_FILTER>(s, g, p, H, Yk, Yout, Yk, Yprev, gw);
}

int launch_filter_step_f32(hipStream_t s, int n, int ncols, const zf* H, int ldh, const zf* Yk, int ldyk,
                           const zf* Yprev, int ldyp, zf* Yout, int ldyo, FilterStep fs, const GemmWs& gw)
{
    if (n <= 0 || ncols <= 0) return 0;
    GDims g = {};
    g.M = n; g.N = ncols; g.K = n; g.lda = ldh; g.ldb = ldyk; g.ldc = ldyo; g.ldyk = ldyk; g.ldyp = ldyp;
    g.alpha = fs.alpha; g.beta = fs.beta; g.shift = fs.shift;
    Plan p = make_plan(n, ncols, n, gw, 8);
    return run<float, OP_N, OP_N, EPI_FILTER>(s, g, p, H, Yk, Yout, Yk, Yprev, gw);
}
