// Complex GEMM on CDNA4 matrix cores, with the Chebyshev three-term recurrence fused into the
// epilogue (Algorithm 1, filtering step: Y_{k+1} = alpha (H - cI) Y_k + beta Y_{k-1}).
//
// Complex products run as four real products on v_mfma_f64_16x16x4f64 (FP64) or
// v_mfma_f32_16x16x4f32 (FP32).  The MFMA is used "transposed": its A operand carries op(B)
// (row index = output column j) and its B operand carries op(A) (column index = output row i),
// so that each lane ends up owning 4 output elements of one output row i, and 16 lanes store 16
// consecutive rows of one column: 256 contiguous bytes per store instruction for complex128.
//
// Workgroup = 4 waves (256 threads) computing a BM x BN complex output tile, each wave a
// (BM/2) x (BN/2) sub-tile of 16x16 MFMA blocks.  Operands are staged through LDS in k-stages of
// 16 complex elements with double buffering (one barrier per stage) and register prefetch of the
// next stage's global loads.  Tiles are enumerated so that consecutive tiles (same rows of A,
// neighbouring column tiles) land on the same XCD: the hardware hands workgroup w to XCD w % 8.
// Split-K writes partial tiles to a workspace; the last K-slice to finish a tile sums the partials
// in slice order (deterministic) and applies the epilogue, so one launch is one filter step.
#include "common.h"

namespace {

template <typename T> struct CT;
template <> struct CT<double> { typedef double2 c; typedef d4 acc; };
template <> struct CT<float> { typedef float2 c; typedef f4 acc; };

__device__ inline d4 mfma16(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4 mfma16(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

enum { EPI_GEMM = 0, EPI_FILTER = 1 };

template <typename T>
struct GArgs {
    typedef typename CT<T>::c C2;
    int M, N, K;
    const C2* A; int lda;
    const C2* B; int ldb;
    C2* C; int ldc;
    double alpha, beta, shift;
    const C2* Yk; int ldyk;
    const C2* Yp; int ldyp;
    C2* P;                 // split-K partials: ksplit blocks of M x N (leading dimension M)
    int* cnt;              // split-K arrival counter per output tile (zero before and after)
    int kchunk, tiles_m, tiles_n, ksplit;
};

// logical tile of workgroup w such that each XCD owns one contiguous range of tiles
__device__ inline int xcd_remap(int w, int nt)
{
    const int X = 8;
    const int per = nt / X, rem = nt % X;
    const int x = w % X, q = w / X;
    return x * per + (x < rem ? x : rem) + q;
}

template <typename C2> __device__ inline C2 cconj(C2 v) { v.y = -v.y; return v; }

// Row of the 16x16 MFMA result held in register r of lane l.  Measured on gfx950:
// v_mfma_f32_16x16x4f32 holds row 4 (l/16) + r, v_mfma_f64_16x16x4f64 holds row 4 r + l/16;
// both hold column l % 16.
__device__ inline int drow(double, int lane, int r) { return 4 * r + (lane >> 4); }
__device__ inline int drow(float, int lane, int r) { return 4 * (lane >> 4) + r; }

template <typename T, int EPI>
__device__ inline void epilogue_store(const GArgs<T>& g, int i, int j, int ks, T vr, T vi)
{
    typedef typename CT<T>::c C2;
    (void)ks;
    if (EPI == EPI_GEMM) {
        const T al = (T)g.alpha, be = (T)g.beta;
        C2 o;
        o.x = al * vr; o.y = al * vi;
        if (g.beta != 0.0) {
            C2 c = g.C[(size_t)i + (size_t)j * g.ldc];
            o.x += be * c.x; o.y += be * c.y;
        }
        g.C[(size_t)i + (size_t)j * g.ldc] = o;
    } else {
        const T al = (T)g.alpha, be = (T)g.beta, sh = (T)g.shift;
        C2 yk = g.Yk[(size_t)i + (size_t)j * g.ldyk];
        C2 yp = g.Yp[(size_t)i + (size_t)j * g.ldyp];
        C2 o;
        o.x = al * (vr - sh * yk.x) + be * yp.x;
        o.y = al * (vi - sh * yk.y) + be * yp.y;
        g.C[(size_t)i + (size_t)j * g.ldc] = o;
    }
}

// SPLIT: this launch is one of ksplit K-slices of each output tile.  Every slice writes its partial
// tile; the last slice to arrive (per-tile counter) sums the ksplit partials in slice order and
// applies the epilogue, then clears the counter.  The sum order does not depend on arrival order.
template <typename T, int OPA, int OPB, int EPI, int BM, int BN, bool SPLIT>
__global__ __launch_bounds__(256) void k_zgemm(GArgs<T> g)
{
    typedef typename CT<T>::c C2;
    typedef typename CT<T>::acc ACC;
    constexpr int BK = 16;
    constexpr int LDA_S = BM + 1, LDB_S = BN + 1;   // +1 element: conflict-free transposed stores
    __shared__ C2 As[2][BK * LDA_S];
    __shared__ C2 Bs[2][BK * LDB_S];
    constexpr int NPA = BM * BK / 256, NPB = BN * BK / 256;
    constexpr int MI = BM / 32, NJ = BN / 32;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nt = g.tiles_m * g.tiles_n * g.ksplit;
    const int tile = xcd_remap(blockIdx.x, nt);
    const int jt = tile % g.tiles_n;
    const int r1 = tile / g.tiles_n;
    const int ks = r1 % g.ksplit;
    const int it = r1 / g.ksplit;
    const int i0 = it * BM, j0 = jt * BN;
    const int kb = ks * g.kchunk;
    const int ke = min(g.K, kb + g.kchunk);
    const int nstages = ke > kb ? (ke - kb + BK - 1) / BK : 0;
    const int wr = (wave & 1) * (BM / 2), wc = (wave >> 1) * (BN / 2);

    ACC accr[MI][NJ], acci[MI][NJ];
#pragma unroll
    for (int bi = 0; bi < MI; ++bi)
#pragma unroll
        for (int bj = 0; bj < NJ; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) { accr[bi][bj][r] = 0; acci[bi][bj][r] = 0; }

    C2 ra[NPA], rb[NPB];
    const C2 zero = {0, 0};

    auto gload = [&](int k0) {
#pragma unroll
        for (int p = 0; p < NPA; ++p) {
            const int e = tid + 256 * p;
            if (OPA == OP_N) {
                const int i = e % BM, k = e / BM, gi = i0 + i, gk = k0 + k;
                ra[p] = (gi < g.M && gk < ke) ? g.A[(size_t)gi + (size_t)gk * g.lda] : zero;
            } else {
                const int k = e % BK, i = e / BK, gi = i0 + i, gk = k0 + k;
                ra[p] = (gi < g.M && gk < ke) ? cconj(g.A[(size_t)gk + (size_t)gi * g.lda]) : zero;
            }
        }
#pragma unroll
        for (int p = 0; p < NPB; ++p) {
            const int e = tid + 256 * p;
            if (OPB == OP_N) {
                const int k = e % BK, j = e / BK, gk = k0 + k, gj = j0 + j;
                rb[p] = (gj < g.N && gk < ke) ? g.B[(size_t)gk + (size_t)gj * g.ldb] : zero;
            } else {
                const int j = e % BN, k = e / BN, gk = k0 + k, gj = j0 + j;
                rb[p] = (gj < g.N && gk < ke) ? cconj(g.B[(size_t)gj + (size_t)gk * g.ldb]) : zero;
            }
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int p = 0; p < NPA; ++p) {
            const int e = tid + 256 * p;
            const int i = (OPA == OP_N) ? e % BM : e / BK;
            const int k = (OPA == OP_N) ? e / BM : e % BK;
            As[buf][k * LDA_S + i] = ra[p];
        }
#pragma unroll
        for (int p = 0; p < NPB; ++p) {
            const int e = tid + 256 * p;
            const int j = (OPB == OP_N) ? e / BK : e % BN;
            const int k = (OPB == OP_N) ? e % BK : e / BN;
            Bs[buf][k * LDB_S + j] = rb[p];
        }
    };
    auto compute = [&](int buf) {
        const C2* as = As[buf];
        const C2* bs = Bs[buf];
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            C2 a[MI], b[NJ];
#pragma unroll
            for (int bi = 0; bi < MI; ++bi) a[bi] = as[kr * LDA_S + wr + bi * 16 + (lane & 15)];
#pragma unroll
            for (int bj = 0; bj < NJ; ++bj) b[bj] = bs[kr * LDB_S + wc + bj * 16 + (lane & 15)];
            // re += Bre Are ; im += Bim Are   (all blocks), then re -= Bim Aim ; im += Bre Aim
#pragma unroll
            for (int bi = 0; bi < MI; ++bi)
#pragma unroll
                for (int bj = 0; bj < NJ; ++bj) {
                    accr[bi][bj] = mfma16(b[bj].x, a[bi].x, accr[bi][bj]);
                    acci[bi][bj] = mfma16(b[bj].y, a[bi].x, acci[bi][bj]);
                }
#pragma unroll
            for (int bi = 0; bi < MI; ++bi)
#pragma unroll
                for (int bj = 0; bj < NJ; ++bj) {
                    accr[bi][bj] = mfma16(-b[bj].y, a[bi].y, accr[bi][bj]);
                    acci[bi][bj] = mfma16(b[bj].x, a[bi].y, acci[bi][bj]);
                }
        }
    };

    if (nstages > 0) {
        gload(kb);
        sstore(0);
        __syncthreads();
        for (int s = 0; s < nstages; ++s) {
            const int buf = s & 1;
            if (s + 1 < nstages) gload(kb + (s + 1) * BK);
            compute(buf);
            if (s + 1 < nstages) sstore(buf ^ 1);
            __syncthreads();
        }
    }

    if (!SPLIT) {
#pragma unroll
        for (int bi = 0; bi < MI; ++bi)
#pragma unroll
            for (int bj = 0; bj < NJ; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + wr + bi * 16 + (lane & 15);
                    const int j = j0 + wc + bj * 16 + drow(T(0), lane, r);
                    if (i < g.M && j < g.N) epilogue_store<T, EPI>(g, i, j, ks, accr[bi][bj][r], acci[bi][bj][r]);
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
                const int j = j0 + wc + bj * 16 + drow(T(0), lane, r);
                if (i < g.M && j < g.N) {
                    C2 o;
                    o.x = accr[bi][bj][r];
                    o.y = acci[bi][bj][r];
                    g.P[(size_t)ks * slab + (size_t)i + (size_t)j * g.M] = o;
                }
            }
    __threadfence();
    __shared__ int s_last;
    __syncthreads();
    if (tid == 0) {
        const int old = atomicAdd(&g.cnt[it * g.tiles_n + jt], 1);
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
                const int j = j0 + wc + bj * 16 + drow(T(0), lane, r);
                if (i < g.M && j < g.N) {
                    T vr = 0, vi = 0;
                    for (int s = 0; s < g.ksplit; ++s) {
                        const C2 p = g.P[(size_t)s * slab + (size_t)i + (size_t)j * g.M];
                        vr += p.x;
                        vi += p.y;
                    }
                    epilogue_store<T, EPI>(g, i, j, 0, vr, vi);
                }
            }
    if (tid == 0) g.cnt[it * g.tiles_n + jt] = 0;
}

struct Plan { int bm, bn, ksplit, kchunk, tiles_m, tiles_n; };

// Tile/split choice: enough workgroups for two per CU on 256 CUs, K slices of at least 256, and
// the split limited by the partial buffer and the counter array.
Plan make_plan(int M, int N, int K, const GemmWs& gw, int elem_bytes)
{
    Plan p;
    p.bm = 64;
    p.bn = N <= 32 ? 32 : 64;
    p.tiles_m = (M + p.bm - 1) / p.bm;
    p.tiles_n = (N + p.bn - 1) / p.bn;
    const long tiles = (long)p.tiles_m * p.tiles_n;
    int ks = 1;
    while (tiles * ks < 512 && (long)K / (2 * ks) >= 256) ks *= 2;
    if (!gw.ws || !gw.cnt || tiles > gw.ncnt) ks = 1;
    while (ks > 1 && (size_t)ks * M * N * (size_t)elem_bytes > gw.bytes) ks /= 2;
    int kc = (K + ks - 1) / ks;
    kc = (kc + 15) / 16 * 16;
    p.kchunk = kc > 0 ? kc : 16;
    p.ksplit = K > 0 ? (K + p.kchunk - 1) / p.kchunk : 1;
    return p;
}

template <typename T, int OPA, int OPB, int EPI>
int run(hipStream_t s, GArgs<T> g, const Plan& p)
{
    g.kchunk = p.kchunk; g.tiles_m = p.tiles_m; g.tiles_n = p.tiles_n; g.ksplit = p.ksplit;
    const int nt = p.tiles_m * p.tiles_n * p.ksplit;
    if (nt <= 0) return 0;
#define LAUNCH(BN_, SP) hipLaunchKernelGGL((k_zgemm<T, OPA, OPB, EPI, 64, BN_, SP>), dim3(nt), dim3(256), 0, s, g)
    if (p.ksplit > 1) {
        if (p.bn == 32) LAUNCH(32, true); else LAUNCH(64, true);
    } else {
        if (p.bn == 32) LAUNCH(32, false); else LAUNCH(64, false);
    }
#undef LAUNCH
    return (int)hipGetLastError();
}

}  // namespace

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
    GArgs<double> g = {};
    g.M = M; g.N = N; g.K = K; g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
    g.alpha = alpha; g.beta = beta; g.P = (zd*)gw.ws; g.cnt = gw.cnt;
    Plan p = make_plan(M, N, K, gw, 16);
    if (opa == OP_N && opb == OP_N) return run<double, OP_N, OP_N, EPI_GEMM>(s, g, p);
    if (opa == OP_C && opb == OP_N) return run<double, OP_C, OP_N, EPI_GEMM>(s, g, p);
    if (opa == OP_N && opb == OP_C) return run<double, OP_N, OP_C, EPI_GEMM>(s, g, p);
    return run<double, OP_C, OP_C, EPI_GEMM>(s, g, p);
}

int launch_filter_step_f64(hipStream_t s, int n, int ncols, const zd* H, int ldh, const zd* Yk, int ldyk,
                           const zd* Yprev, int ldyp, zd* Yout, int ldyo, FilterStep fs, const GemmWs& gw)
{
    if (n <= 0 || ncols <= 0) return 0;
    GArgs<double> g = {};
    g.M = n; g.N = ncols; g.K = n; g.A = H; g.lda = ldh; g.B = Yk; g.ldb = ldyk; g.C = Yout; g.ldc = ldyo;
    g.alpha = fs.alpha; g.beta = fs.beta; g.shift = fs.shift; g.Yk = Yk; g.ldyk = ldyk; g.Yp = Yprev;
    g.ldyp = ldyp; g.P = (zd*)gw.ws; g.cnt = gw.cnt;
    Plan p = make_plan(n, ncols, n, gw, 16);
    return run<double, OP_N, OP_N, EPI_FILTER>(s, g, p);
}

int launch_filter_step_f32(hipStream_t s, int n, int ncols, const zf* H, int ldh, const zf* Yk, int ldyk,
                           const zf* Yprev, int ldyp, zf* Yout, int ldyo, FilterStep fs, const GemmWs& gw)
{
    if (n <= 0 || ncols <= 0) return 0;
    GArgs<float> g = {};
    g.M = n; g.N = ncols; g.K = n; g.A = H; g.lda = ldh; g.B = Yk; g.ldb = ldyk; g.C = Yout; g.ldc = ldyo;
    g.alpha = fs.alpha; g.beta = fs.beta; g.shift = fs.shift; g.Yk = Yk; g.ldyk = ldyk; g.Yp = Yprev;
    g.ldyp = ldyp; g.P = (zf*)gw.ws; g.cnt = gw.cnt;
    Plan p = make_plan(n, ncols, n, gw, 8);
    return run<float, OP_N, OP_N, EPI_FILTER>(s, g, p);
}
