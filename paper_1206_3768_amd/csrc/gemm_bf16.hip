// BF16-split Chebyshev filter step on CDNA4 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Each real operand x is split into bf16 terms x ~ x_0 + x_1 (+ x_2), every term the bf16
// rounding (to nearest even) of what the previous terms leave.  A real product is then the sum of
// the term products with t_x + t_y < nterms: 3 products for two terms ("x3", ~16 significant
// bits) or 6 for three terms ("x6", ~24 bits, FP32-like), accumulated in FP32.  A complex product
// is four real products: re += Hre Yre - Him Yim, im += Hre Yim + Him Yre.
//
// Layouts.  H is split once per solve into 2*nterms planes (term t, part re/im) stored row-major
// (row i, k contiguous): since H is Hermitian, row i of H is the conjugate of column i, so each
// plane row is written from one contiguous column.  Y_k (complex64) is split each step into planes
// stored column-major (k contiguous).  Both are zero-padded to a multiple of 32 in k, so an MFMA
// operand (8 consecutive k of one row or column) is one 16-byte load.  The MFMA A operand carries
// Y (row = output column j) and the B operand carries H (column = output row i), as in the FP64
// kernel, so each lane stores complete complex64 outputs of one row.
#include "common.h"
#include "driver.h"

#include <algorithm>
#include <vector>

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

__host__ __device__ inline uint16_t f32_to_bf16_rne(float x)
{
    uint32_t u;
    __builtin_memcpy(&u, &x, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float x;
    __builtin_memcpy(&x, &u, 4);
    return x;
}

// split of a double (H) and of a float (Y): term t = bf16(float(remainder)), remainder -= term
__device__ inline void split_terms_d(double x, int nterms, uint16_t* out)
{
    double r = x;
    for (int t = 0; t < nterms; ++t) {
        const uint16_t b = f32_to_bf16_rne((float)r);
        out[t] = b;
        r -= (double)bf16_to_f32(b);
    }
}

__device__ inline void split_terms_f(float x, int nterms, uint16_t* out)
{
    float r = x;
    for (int t = 0; t < nterms; ++t) {
        const uint16_t b = f32_to_bf16_rne(r);
        out[t] = b;
        r -= bf16_to_f32(b);
    }
}

inline int pad32(int n) { return (n + 31) / 32 * 32; }

// H planes: plane (t, part) element (i, k) at planes[(2t + part) * np * np + i * np + k]
//   = term t of Re/Im H[i, k] = term t of Re H[k, i], -Im H[k, i]  (H Hermitian)
__global__ void k_split_h(int n, int np, const zd* __restrict__ H, int ldh, uint16_t* __restrict__ planes, int nterms)
{
    const size_t total = (size_t)np * np;
    const size_t ps = total;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(e % np), i = (int)(e / np);   // consecutive threads: consecutive k of row i
        zd v = make_double2(0.0, 0.0);
        if (i < n && k < n) {
            const zd c = H[(size_t)k + (size_t)i * ldh];   // column i, row k: contiguous in k
            v = make_double2(c.x, -c.y);
        }
        uint16_t tr[3], ti[3];
        split_terms_d(v.x, nterms, tr);
        split_terms_d(v.y, nterms, ti);
        for (int t = 0; t < nterms; ++t) {
            planes[(size_t)(2 * t) * ps + e] = tr[t];
            planes[(size_t)(2 * t + 1) * ps + e] = ti[t];
        }
    }
}

// Y planes: plane (t, part) element (k, j) at ys[(2t + part) * np * ncp + j * np + k]
__global__ void k_split_y(int n, int np, int ncols, int ncp, const zf* __restrict__ Y, int ldy,
                          uint16_t* __restrict__ ys, int nterms)
{
    const size_t total = (size_t)np * ncp;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(e % np), j = (int)(e / np);
        zf v = make_float2(0.f, 0.f);
        if (k < n && j < ncols) v = Y[(size_t)k + (size_t)j * ldy];
        uint16_t tr[3], ti[3];
        split_terms_f(v.x, nterms, tr);
        split_terms_f(v.y, nterms, ti);
        for (int t = 0; t < nterms; ++t) {
            ys[(size_t)(2 * t) * total + e] = tr[t];
            ys[(size_t)(2 * t + 1) * total + e] = ti[t];
        }
    }
}

__device__ inline int xcd_remap(int w, int nt)
{
    const int X = 8;
    const int per = nt / X, rem = nt % X;
    const int x = w % X, q = w / X;
    return x * per + (x < rem ? x : rem) + q;
}

struct BArgs {
    int n, np, ncols, ncp, nterms;
    const uint16_t* Hp;     // planes, row-major, np x np each
    const uint16_t* Ys;     // planes, column-major, np x ncp each
    const zf* Yk; int ldyk;
    const zf* Yp; int ldyp;
    zf* Yo; int ldyo;
    float alpha, beta, shift;
    zf* P;                  // split-K partials [ksplit][ncols][n]
    int* cnt;               // split-K arrival counter per output tile (zero before and after)
    int kchunk, tiles_m, tiles_n, ksplit;
};

// LDS row swizzle of the filter kernels: the 16-byte chunk c of tile row r (32 bf16 of k per row,
// 64 bytes, no padding) sits at chunk position c ^ swz(r).  A 16-byte fragment read (lane l: row
// l%16 of a 16-row block, chunk l/16) is served 32 lanes = 512 bytes per LDS cycle on gfx950
// (measured: a plain, padded or 8-row-swizzled 64-byte row layout costs 4 extra cycles per read, a
// linear one none).  The 32 lanes then cover rows r and r+8 with two chunks each, and the four
// (row, chunk) pairs that share a 64-byte bank window must take four different positions: bit 1 of
// swz flips between r and r+8, and swz takes four values on r, r+4, r+8, r+12 and on r, r+2, r+4,
// r+6 (also conflict-free when 16 or 8 lanes are served per cycle).
__device__ __forceinline__ int swz(int r) { return (((r >> 1) ^ (r >> 3)) & 1) | ((((r >> 2) ^ (r >> 3)) & 1) << 1); }

// One filter step on a BM x BN tile (BM = BN = 32 WT), 4 waves of (16 WT) x (16 WT) outputs, each
// a WT x WT array of 16 x 16 MFMA blocks.  WT = 2: 64 x 64 tiles (two workgroups per CU); WT = 4:
// 128 x 128 tiles (one workgroup per CU, the whole LDS), whose waves read half the LDS bytes per
// MFMA and whose workgroups fetch half the L2 bytes per MFMA.
template <int NT, bool SPLIT, int WT>
__global__ __launch_bounds__(256) void k_filter_bf16(BArgs g)
{
    constexpr int BM = 32 * WT, BN = 32 * WT, BK = 32;
    constexpr int NPL = 2 * NT;                  // planes per operand
    constexpr int RS = BK;                       // LDS row stride in bf16 (64 bytes, chunks swizzled)
    constexpr int RL = BM / 64;                  // 64-row slabs a thread loads per plane
    __shared__ __attribute__((aligned(16))) uint16_t Hs[2][NPL][BM * RS];
    __shared__ __attribute__((aligned(16))) uint16_t Ys[2][NPL][BN * RS];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nt = g.tiles_m * g.tiles_n * g.ksplit;
    const int tile = xcd_remap(blockIdx.x, nt);
    const int jt = tile % g.tiles_n;
    const int r1 = tile / g.tiles_n;
    const int ks = r1 % g.ksplit;
    const int it = r1 / g.ksplit;
    const int i0 = it * BM, j0 = jt * BN;
    const int kb = ks * g.kchunk;
    const int ke = min(g.np, kb + g.kchunk);
    const int nstages = ke > kb ? (ke - kb) / BK : 0;
    const int wr = (wave & 1) * (16 * WT), wc = (wave >> 1) * (16 * WT);

    f4 accr[WT][WT], acci[WT][WT];
#pragma unroll
    for (int a = 0; a < WT; ++a)
#pragma unroll
        for (int b = 0; b < WT; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) { accr[a][b][r] = 0.f; acci[a][b][r] = 0.f; }

    // global -> register: thread t moves 16 bytes (8 k) of row/col t/4 (+ 64 q), chunk t%4, per plane.
    // Rows of H beyond the padded order and columns of Y beyond the padded width are clamped to the
    // last one instead of masked: they only reach output rows / columns that are never stored, and
    // the loads stay branch-free
    const int lrow = tid >> 2, lch = tid & 3;
    u4v rh[RL][NPL], ry[RL][NPL];
    const size_t hps = (size_t)g.np * g.np, yps = (size_t)g.np * g.ncp;
    const uint16_t* hbase[RL];
    const uint16_t* ybase[RL];
#pragma unroll
    for (int q = 0; q < RL; ++q) {
        const int gi = min(i0 + lrow + 64 * q, g.np - 1), gj = min(j0 + lrow + 64 * q, g.ncp - 1);
        hbase[q] = g.Hp + (size_t)gi * g.np + lch * 8;
        ybase[q] = g.Ys + (size_t)gj * g.np + lch * 8;
    }
    auto gload = [&](int k0) {
#pragma unroll
        for (int q = 0; q < RL; ++q)
#pragma unroll
            for (int p = 0; p < NPL; ++p) {
                rh[q][p] = *(const u4v*)(hbase[q] + (size_t)p * hps + k0);
                ry[q][p] = *(const u4v*)(ybase[q] + (size_t)p * yps + k0);
            }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < RL; ++q)
#pragma unroll
            for (int p = 0; p < NPL; ++p) {
                const int r = lrow + 64 * q, c = (lch ^ swz(r)) * 8;
                *(u4v*)&Hs[buf][p][r * RS + c] = rh[q][p];
                *(u4v*)&Ys[buf][p][r * RS + c] = ry[q][p];
            }
    };
    auto compute = [&](int buf) {
        const int fr = lane & 15, fc = lane >> 4;
        u4v hf[WT][NPL], yf[WT][NPL];
#pragma unroll
        for (int b = 0; b < WT; ++b) {
            const int rh = wr + b * 16 + fr, ry = wc + b * 16 + fr;
            const int oh = rh * RS + ((fc ^ swz(rh)) << 3), oy = ry * RS + ((fc ^ swz(ry)) << 3);
#pragma unroll
            for (int p = 0; p < NPL; ++p) {
                hf[b][p] = *(const u4v*)&Hs[buf][p][oh];
                yf[b][p] = *(const u4v*)&Ys[buf][p][oy];
            }
        }
#pragma unroll
        for (int s = 0; s < NT; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if (s + t >= NT) continue;
#pragma unroll
                for (int bi = 0; bi < WT; ++bi)
#pragma unroll
                    for (int bj = 0; bj < WT; ++bj) {
                        const bf8 hre = __builtin_bit_cast(bf8, hf[bi][2 * s]);
                        const bf8 him = __builtin_bit_cast(bf8, hf[bi][2 * s + 1]);
                        const bf8 yre = __builtin_bit_cast(bf8, yf[bj][2 * t]);
                        const u4v ymi = yf[bj][2 * t + 1];
                        const bf8 yim = __builtin_bit_cast(bf8, ymi);
                        const bf8 nyim = __builtin_bit_cast(bf8, ymi ^ u4v{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u});
                        accr[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yre, hre, accr[bi][bj], 0, 0, 0);
                        acci[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yim, hre, acci[bi][bj], 0, 0, 0);
                        accr[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nyim, him, accr[bi][bj], 0, 0, 0);
                        acci[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yre, him, acci[bi][bj], 0, 0, 0);
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

    const size_t slab = (size_t)g.n * g.ncols;
    if (SPLIT) {
#pragma unroll
        for (int bi = 0; bi < WT; ++bi)
#pragma unroll
            for (int bj = 0; bj < WT; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + wr + bi * 16 + (lane & 15);
                    const int j = j0 + wc + bj * 16 + (lane >> 4) * 4 + r;
                    if (i < g.n && j < g.ncols)
                        g.P[(size_t)ks * slab + (size_t)i + (size_t)j * g.n] =
                            make_float2(accr[bi][bj][r], acci[bi][bj][r]);
                }
        __threadfence();
        // the arrival flag lives in the (no longer read) LDS of the operands: the loop ended with a barrier
        int* s_last = (int*)&Hs[0][0][0];
        if (tid == 0) s_last[0] = (atomicAdd(&g.cnt[it * g.tiles_n + jt], 1) == g.ksplit - 1);
        __syncthreads();
        if (!s_last[0]) return;
        __threadfence();
    }
#pragma unroll
    for (int bi = 0; bi < WT; ++bi)
#pragma unroll
        for (int bj = 0; bj < WT; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wr + bi * 16 + (lane & 15);
                const int j = j0 + wc + bj * 16 + (lane >> 4) * 4 + r;
                if (i >= g.n || j >= g.ncols) continue;
                float vr = accr[bi][bj][r], vi = acci[bi][bj][r];
                if (SPLIT) {
                    vr = 0.f;
                    vi = 0.f;
                    for (int s2 = 0; s2 < g.ksplit; ++s2) {
                        const zf p = g.P[(size_t)s2 * slab + (size_t)i + (size_t)j * g.n];
                        vr += p.x;
                        vi += p.y;
                    }
                }
                const zf yk = g.Yk[(size_t)i + (size_t)j * g.ldyk];
                const zf yp = g.Yp[(size_t)i + (size_t)j * g.ldyp];
                g.Yo[(size_t)i + (size_t)j * g.ldyo] = make_float2(g.alpha * (vr - g.shift * yk.x) + g.beta * yp.x,
                                                                 g.alpha * (vi - g.shift * yk.y) + g.beta * yp.y);
            }
    if (SPLIT && tid == 0) g.cnt[it * g.tiles_n + jt] = 0;
}


// Two-term split, 128 x 128 tiles, software-pipelined.  Each of the 4 waves owns a 64 x 64 block of
// outputs (4 x 4 MFMA blocks of 16 x 16) and moves one bf16 plane of each operand per k-stage
// straight from global memory into LDS (global_load_lds_dwordx4: no staging registers, no LDS
// store instructions).  Per k-stage of 32:
//   row blocks 0..2: read the H fragment of the next row block, then the 48 products of this one;
//   barrier (the next stage's tiles have landed, every wave is done with this stage's buffer);
//   start the stage after next into the buffer just released, read the next stage's Y fragments
//   and first H fragment, and run the 48 products of row block 3 meanwhile.
// So the matrix cores always have independent products queued while LDS and memory traffic for
// the next stage is in flight; one barrier per stage.
template <bool SPLIT>
__global__ __launch_bounds__(256) void k_filter_bf16_p(BArgs g)
{
    constexpr int NPL = 4, BM = 128, BK = 32;
    // one array per buffer: the compiler then knows which buffer a load into LDS targets and waits
    // for it only before reads of that buffer
    __shared__ __attribute__((aligned(1024))) uint16_t Hs0[NPL][BM * BK];
    __shared__ __attribute__((aligned(1024))) uint16_t Hs1[NPL][BM * BK];
    __shared__ __attribute__((aligned(1024))) uint16_t Ys0[NPL][BM * BK];
    __shared__ __attribute__((aligned(1024))) uint16_t Ys1[NPL][BM * BK];

    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nt = g.tiles_m * g.tiles_n * g.ksplit;
    const int tile = xcd_remap(blockIdx.x, nt);
    const int jt = tile % g.tiles_n;
    const int r1 = tile / g.tiles_n;
    const int ks = r1 % g.ksplit;
    const int it = r1 / g.ksplit;
    const int i0 = it * BM, j0 = jt * BM;
    const int kb = ks * g.kchunk;
    const int ke = min(g.np, kb + g.kchunk);
    const int nst = ke > kb ? (ke - kb) / BK : 0;
    const int wr = (wave & 1) * 64, wc = (wave >> 1) * 64;

    f4 accr[4][4], acci[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) { accr[a][b][r] = 0.f; acci[a][b][r] = 0.f; }

    // global -> LDS: wave w moves plane w of H and of Y, 8 instructions of 16 rows x 64 bytes each;
    // lane l serves row 16 i + l/4 at chunk position l%4.  Rows beyond the padded order / width are
    // clamped to the last one (they reach only outputs that are never stored)
    const int q = lane >> 2, pos = lane & 3;
    uint32_t ho[8], yo[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int r = 16 * i + q, c = pos ^ swz(r);
        ho[i] = (uint32_t)((min(i0 + r, g.np - 1) - i0) * g.np + c * 8) * 2u;
        yo[i] = (uint32_t)((min(j0 + r, g.ncp - 1) - j0) * g.np + c * 8) * 2u;
    }
    const char* hplane = (const char*)(g.Hp + (size_t)wave * g.np * g.np + (size_t)i0 * g.np);
    const char* yplane = (const char*)(g.Ys + (size_t)wave * g.np * g.ncp + (size_t)j0 * g.np);
    auto dma = [&](uint16_t (&hs)[NPL][BM * BK], uint16_t (&ys)[NPL][BM * BK], int k0) {
        const char* hb = hplane + 2 * (size_t)k0;
        const char* yb = yplane + 2 * (size_t)k0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            __builtin_amdgcn_global_load_lds((const void*)(hb + ho[i]), &hs[wave][16 * i * BK], 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void*)(yb + yo[i]), &ys[wave][16 * i * BK], 16, 0, 0);
        }
    };

    // fragment offsets (elements) of the four 16-row blocks of this wave, lane row l%16, chunk l/16
    const int fr = lane & 15, fc = lane >> 4;
    int hoff[4], yoff[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int rh = wr + 16 * b + fr, ry = wc + 16 * b + fr;
        hoff[b] = rh * BK + ((fc ^ swz(rh)) << 3);
        yoff[b] = ry * BK + ((fc ^ swz(ry)) << 3);
    }
    auto hread = [&](const uint16_t (&hs)[NPL][BM * BK], int b, u4v (&h)[NPL]) {
#pragma unroll
        for (int p = 0; p < NPL; ++p) h[p] = *(const u4v*)&hs[p][hoff[b]];
    };
    auto yread = [&](const uint16_t (&ys)[NPL][BM * BK], u4v (&y)[4][NPL]) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int p = 0; p < NPL; ++p) y[b][p] = *(const u4v*)&ys[p][yoff[b]];
    };
    // the 48 products of one 16-row block: term pairs (0,0), (0,1), (1,0), four real products each
    auto mblock = [&](int bi, const u4v (&h)[NPL], const u4v (&y)[4][NPL]) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                if (s + t >= 2) continue;
                const bf8 hre = __builtin_bit_cast(bf8, h[2 * s]);
                const bf8 him = __builtin_bit_cast(bf8, h[2 * s + 1]);
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) {
                    const bf8 yre = __builtin_bit_cast(bf8, y[bj][2 * t]);
                    const u4v ymi = y[bj][2 * t + 1];
                    const bf8 yim = __builtin_bit_cast(bf8, ymi);
                    const bf8 nyim = __builtin_bit_cast(bf8, ymi ^ u4v{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u});
                    accr[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yre, hre, accr[bi][bj], 0, 0, 0);
                    acci[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yim, hre, acci[bi][bj], 0, 0, 0);
                    accr[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nyim, him, accr[bi][bj], 0, 0, 0);
                    acci[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yre, him, acci[bi][bj], 0, 0, 0);
                }
            }
    };

    // Stage s lives in buffer s % 2.  A stage is split at its barrier into a front (row blocks 0..2)
    // and a back (loads two stages ahead, next stage's fragments, row block 3); the loop runs
    // back(s), front(s+1), back(s+1), front(s+2), so its trips start right after a barrier, when no
    // load into LDS is in flight, and every buffer is static.  Scheduling barriers keep each
    // fragment read one row block ahead of its products; the next stage's fragments are always read
    // (on the last stage from the idle buffer, unused) so that no branch joins in-flight reads.
    u4v yf[4][NPL], h0[NPL], h1[NPL], h2[NPL], h3[NPL];
    // products of one row block with the next block's H fragment read after its first four
    auto phase = [&](const uint16_t (&hs)[NPL][BM * BK], int b, const u4v (&h)[NPL], u4v (&hnext)[NPL]) {
        mblock(b, h, yf);
        hread(hs, b + 1, hnext);
        __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 44, 0);
        __builtin_amdgcn_sched_barrier(0);
    };
    auto front = [&](const uint16_t (&hs)[NPL][BM * BK]) {
        phase(hs, 0, h0, h1);
        phase(hs, 1, h1, h2);
        phase(hs, 2, h2, h3);
        // this thread's loads of the next stage have landed and its reads of this one are done;
        // then every wave's
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };
    auto back = [&](int s, uint16_t (&hs)[NPL][BM * BK], uint16_t (&ys)[NPL][BM * BK],
                    const uint16_t (&hs_next)[NPL][BM * BK], const uint16_t (&ys_next)[NPL][BM * BK]) {
        if (s + 2 < nst) dma(hs, ys, kb + (s + 2) * BK);
        __builtin_amdgcn_sched_barrier(0);
        u4v yn[4][NPL];
        yread(ys_next, yn);
        hread(hs_next, 0, h0);
        mblock(3, h3, yf);
        // one fragment read per two products of row block 3
#pragma unroll
        for (int r = 0; r < 20; ++r) {
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int p = 0; p < NPL; ++p) yf[b][p] = yn[b][p];
    };
    if (nst > 0) {
        dma(Hs0, Ys0, kb);
        if (nst > 1) dma(Hs1, Ys1, kb + BK);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        yread(Ys0, yf);
        hread(Hs0, 0, h0);
        front(Hs0);
        for (int s = 0; s < nst; s += 2) {
            back(s, Hs0, Ys0, Hs1, Ys1);
            if (s + 1 < nst) {
                front(Hs1);
                back(s + 1, Hs1, Ys1, Hs0, Ys0);
                if (s + 2 < nst) front(Hs0);
            }
        }
    }

    const size_t slab = (size_t)g.n * g.ncols;
    if (SPLIT) {
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + wr + bi * 16 + fr;
                    const int j = j0 + wc + bj * 16 + fc * 4 + r;
                    if (i < g.n && j < g.ncols)
                        g.P[(size_t)ks * slab + (size_t)i + (size_t)j * g.n] =
                            make_float2(accr[bi][bj][r], acci[bi][bj][r]);
                }
        __threadfence();
        // arrival flag in the operands' LDS: no wave touches it after the last stage's barrier
        int* s_last = (int*)&Hs0[0][0];
        __syncthreads();
        if (tid == 0) s_last[0] = (atomicAdd(&g.cnt[it * g.tiles_n + jt], 1) == g.ksplit - 1);
        __syncthreads();
        if (!s_last[0]) return;
        __threadfence();
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wr + bi * 16 + fr;
                const int j = j0 + wc + bj * 16 + fc * 4 + r;
                if (i >= g.n || j >= g.ncols) continue;
                float vr = accr[bi][bj][r], vi = acci[bi][bj][r];
                if (SPLIT) {
                    vr = 0.f;
                    vi = 0.f;
                    for (int s2 = 0; s2 < g.ksplit; ++s2) {
                        const zf p = g.P[(size_t)s2 * slab + (size_t)i + (size_t)j * g.n];
                        vr += p.x;
                        vi += p.y;
                    }
                }
                const zf yk = g.Yk[(size_t)i + (size_t)j * g.ldyk];
                const zf yp = g.Yp[(size_t)i + (size_t)j * g.ldyp];
                g.Yo[(size_t)i + (size_t)j * g.ldyo] = make_float2(g.alpha * (vr - g.shift * yk.x) + g.beta * yp.x,
                                                                 g.alpha * (vi - g.shift * yk.y) + g.beta * yp.y);
            }
    if (SPLIT && tid == 0) g.cnt[it * g.tiles_n + jt] = 0;
}

inline int grid_for(size_t total)
{
    size_t b = (total + 255) / 256;
    return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

}  // namespace

size_t bf16_ysplit_bytes(int n, int ncols, int nterms)
{
    const size_t np = (size_t)pad32(n), ncp = (size_t)(ncols + 63) / 64 * 64;
    return 2 * (size_t)nterms * np * ncp * sizeof(uint16_t);
}

size_t bf16_hplanes_elems(int n, int nterms)
{
    const size_t np = (size_t)pad32(n);
    return 2 * (size_t)nterms * np * np;
}

int launch_split_h_bf16(hipStream_t s, int n, const zd* H, int ldh, uint16_t* planes, int /*ldp*/, int nterms)
{
    const int np = pad32(n);
    hipLaunchKernelGGL(k_split_h, dim3(grid_for((size_t)np * np)), dim3(256), 0, s, n, np, H, ldh, planes, nterms);
    return (int)hipGetLastError();
}

int launch_filter_step_bf16(hipStream_t s, int n, int ncols, const uint16_t* Hplanes, int /*ldp*/, int nterms,
                            const zf* Yk, int ldyk, const zf* Yprev, int ldyp, zf* Yout, int ldyo, FilterStep fs,
                            uint16_t* ysplit, const GemmWs& gw)
{
    if (n <= 0 || ncols <= 0) return 0;
    if (nterms != 2 && nterms != 3) return (int)hipErrorInvalidValue;
    const int np = pad32(n), ncp = (ncols + 63) / 64 * 64;
    const bool timed = gw.ev_start && gw.ev_main && gw.ev_end;
    launch_timed(k_split_y, dim3(grid_for((size_t)np * ncp)), dim3(256), s, timed ? gw.ev_start : nullptr, nullptr, n,
                 np, ncols, ncp, Yk, ldyk, ysplit, nterms);
    BArgs g;
    g.n = n; g.np = np; g.ncols = ncols; g.ncp = ncp; g.nterms = nterms;
    g.Hp = Hplanes; g.Ys = ysplit; g.Yk = Yk; g.ldyk = ldyk; g.Yp = Yprev; g.ldyp = ldyp; g.Yo = Yout; g.ldyo = ldyo;
    g.alpha = (float)fs.alpha; g.beta = (float)fs.beta; g.shift = (float)fs.shift;
    g.P = (zf*)gw.ws;
    g.cnt = gw.cnt;
    // A forced plan (tuned table or caller): tile plan_bm (64, or 128 for the two-term split) and
    // K split plan_ksplit.  Otherwise 128 x 128 tiles (one workgroup per CU) for the two-term split
    // when they still give a workgroup per CU, else 64 x 64 tiles (two per CU; the three-term
    // split's planes do not fit the LDS at 128 x 128), and the K split that fills the CUs.
    const bool forced = gw.plan_bm == 64 || (gw.plan_bm == 128 && nterms == 2);
    const long t128 = (long)((n + 127) / 128) * ((ncols + 127) / 128);
    const int tile = forced ? gw.plan_bm : ((nterms == 2 && t128 >= 192) ? 128 : 64);
    const long per_cu = tile == 128 ? 256 : 512;
    g.tiles_m = (n + tile - 1) / tile;
    g.tiles_n = (ncols + tile - 1) / tile;
    const long tiles = (long)g.tiles_m * g.tiles_n;
    int ksp = 1;
    if (forced) {
        ksp = std::max(1, std::min(gw.plan_ksplit, np / 32));
    } else {
        while (tiles * ksp < per_cu && np / (2 * ksp) >= 512) ksp *= 2;
    }
    if (!gw.ws || !gw.cnt || tiles > gw.ncnt) ksp = 1;
    while (ksp > 1 && (size_t)ksp * n * ncols * sizeof(zf) > gw.bytes) ksp /= 2;
    int kc = (np + ksp - 1) / ksp;
    kc = (kc + 31) / 32 * 32;
    g.kchunk = kc;
    g.ksplit = (np + kc - 1) / kc;
    const int nt = g.tiles_m * g.tiles_n * g.ksplit;
    const bool split = g.ksplit > 1;
    const hipEvent_t e1 = timed ? gw.ev_main : nullptr;
    if (nterms == 2 && tile == 128) {
        if (split) launch_timed(k_filter_bf16_p<true>, dim3(nt), dim3(256), s, nullptr, e1, g);
        else launch_timed(k_filter_bf16_p<false>, dim3(nt), dim3(256), s, nullptr, e1, g);
    } else if (nterms == 2) {
        if (split) launch_timed(k_filter_bf16<2, true, 2>, dim3(nt), dim3(256), s, nullptr, e1, g);
        else launch_timed(k_filter_bf16<2, false, 2>, dim3(nt), dim3(256), s, nullptr, e1, g);
    } else {
        if (split) launch_timed(k_filter_bf16<3, true, 2>, dim3(nt), dim3(256), s, nullptr, e1, g);
        else launch_timed(k_filter_bf16<3, false, 2>, dim3(nt), dim3(256), s, nullptr, e1, g);
    }
    if (gw.plan_used) {
        gw.plan_used[0] = tile; gw.plan_used[1] = tile; gw.plan_used[2] = g.ksplit; gw.plan_used[3] = split ? 2 : 0;
    }
    if (timed) (void)hipEventRecord(gw.ev_end, s);
    return (int)hipGetLastError();
}

// Filter in BF16-split arithmetic; same sequencing as the FP64/FP32 filters (degrees sorted
// non-increasing, columns finishing on odd steps copied back from T at the end).
chfsi_status filter_bf16(chfsi_handle h, int n, const uint16_t* Hb, int ldh, int nterms, int ma, zf* Yf, int ldy,
                         zf* Tf, uint16_t* ysplit, const std::vector<int>& deg, double a, double b, double mu1,
                         int* flag_dev, const GemmWs& gw, double& flops, long long& matvecs, const zd* hy0)
{
    hipStream_t st = h->stream;
    if (ma <= 0 || deg[0] <= 0) return CHFSI_SUCCESS;
    const int dmax = deg[0];
    std::vector<FilterStep> steps;
    filter_coefficients(dmax, a, b, mu1, steps);
    for (int k = 1; k <= dmax; ++k) {
        int w = 0;
        while (w < ma && deg[w] >= k) ++w;
        const zf* yk = (k % 2 == 1) ? Yf : Tf;
        const int ldk = (k % 2 == 1) ? ldy : n;
        zf* yo = (k % 2 == 1) ? Tf : Yf;
        const int ldo = (k % 2 == 1) ? n : ldy;
        const zf* yp = (k == 1) ? yk : yo;
        const int ldp = (k == 1) ? ldk : ldo;
        if (k == 1 && hy0) {   // H Y_0 known (hy0, ld n): step 1 without a product
            if (launch_first_step(st, n, w, steps[0].alpha, steps[0].shift, hy0, n, yk, ldk, yo, ldo))
                return CHFSI_ERR_DEVICE;
            matvecs += w;        // the degree count; filter_flops counts the products performed
            continue;
        }
        GemmWs gs = gw;
        const int pr = nterms == 2 ? CHFSI_BF16X3 : CHFSI_BF16X6;
        apply_tuned_plan(h, pr, n, w, gs);
        h->ktimer.begin(n, w, pr, gs);
        if (launch_filter_step_bf16(st, n, w, Hb, ldh, nterms, yk, ldk, yp, ldp, yo, ldo, steps[k - 1], ysplit, gs))
            return CHFSI_ERR_DEVICE;
        h->ktimer.end(gs);
        flops += 8.0 * (double)n * (double)n * (double)w;
        matvecs += w;
    }
    std::vector<int> odd(ma);
    bool any = false;
    for (int j = 0; j < ma; ++j) { odd[j] = deg[j] % 2; any |= odd[j] != 0; }
    if (any) {
        if (hipMemcpyAsync(flag_dev, odd.data(), sizeof(int) * ma, hipMemcpyHostToDevice, st) != hipSuccess)
            return CHFSI_ERR_DEVICE;
        if (launch_copy_cols_flag_c(st, n, ma, Tf, n, Yf, ldy, flag_dev)) return CHFSI_ERR_DEVICE;
        if (hipStreamSynchronize(st) != hipSuccess) return CHFSI_ERR_DEVICE;
    }
    return CHFSI_SUCCESS;
}
