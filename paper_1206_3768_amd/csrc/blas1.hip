// Memory-bound helper kernels of the ChFSI path: residual norms (Algorithm 1, residual test),
// Lanczos vector operations (spectral upper bound), column dot products, copies and conversions,
// the Philox4x64-10 random fill, phase normalisation of eigenvectors and column permutations.
// All are column-major with one wave (64 lanes) or one workgroup per column so that every global
// access walks a contiguous column.
#include "common.h"

namespace {

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// sum over a 256-thread block; result valid in thread 0
__device__ inline double block_sum256(double v, double* sm)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sm[w] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0) r = sm[0] + sm[1] + sm[2] + sm[3];
    __syncthreads();
    return r;
}

__global__ void k_zlacpy(int M, int N, const zd* A, int lda, zd* B, int ldb)
{
    const size_t total = (size_t)M * N;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % M), j = (int)(e / M);
        B[(size_t)i + (size_t)j * ldb] = A[(size_t)i + (size_t)j * lda];
    }
}

__global__ void k_z2c(int M, int N, const zd* A, int lda, zf* B, int ldb)
{
    const size_t total = (size_t)M * N;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % M), j = (int)(e / M);
        zd v = A[(size_t)i + (size_t)j * lda];
        B[(size_t)i + (size_t)j * ldb] = make_float2((float)v.x, (float)v.y);
    }
}

__global__ void k_c2z(int M, int N, const zf* A, int lda, zd* B, int ldb)
{
    const size_t total = (size_t)M * N;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % M), j = (int)(e / M);
        zf v = A[(size_t)i + (size_t)j * lda];
        B[(size_t)i + (size_t)j * ldb] = make_double2((double)v.x, (double)v.y);
    }
}

// H <- (H + H^H)/2, one thread per lower-triangle entry (diagonal: imaginary part dropped)
// 32 x 32 tiles: tile (bi, bj), bi >= bj, is read (coalesced) into LDS and written conjugate
// transposed to tile (bj, bi)
__global__ __launch_bounds__(256) void k_mirror_lower(int n, zd* H, int ldh)
{
    __shared__ zd T[32][33];
    const int bi = blockIdx.x, bj = blockIdx.y;
    if (bi < bj) return;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {   // T[c][rr] = H(bi*32 + rr, bj*32 + c)
        const int i = bi * 32 + tx, j = bj * 32 + r;
        if (i < n && j < n) T[r][tx] = H[(size_t)i + (size_t)j * ldh];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {   // H(i, j) = conj(H(j, i)) for i = bj*32 + tx < j = bi*32 + r
        const int i = bj * 32 + tx, j = bi * 32 + r;
        if (i >= n || j >= n || i > j) continue;
        const zd v = T[tx][r];
        H[(size_t)i + (size_t)j * ldh] = make_double2(v.x, i == j ? 0.0 : -v.y);
    }
}


// Philox4x64-10 (Salmon et al., SC'11): ten rounds with the published multipliers and Weyl
// constants.  Element e of stream `stream` uses counter (e/2, stream, 0, 0) and key (seed, 0);
// its parity picks words (0,1) or (2,3); each word w gives (w >> 11) 2^-53 in [0,1), mapped to
// [-1, 1) for the real and imaginary parts.
__device__ inline void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t y0 = hi1 ^ c[1] ^ k0, y2 = hi0 ^ c[3] ^ k1;
        c[0] = y0; c[1] = lo1; c[2] = y2; c[3] = lo0;
    }
}

__global__ void k_philox_block(uint64_t seed, uint64_t stream, int n, int m, zd* Y, int ldy)
{
    const size_t total = (size_t)n * m;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        uint64_t c[4] = {(uint64_t)e >> 1, stream, 0, 0};
        philox4x64(c, seed, 0);
        const int w = (int)(e & 1) * 2;
        const double re = 2.0 * ((double)(c[w] >> 11) * 0x1.0p-53) - 1.0;
        const double im = 2.0 * ((double)(c[w + 1] >> 11) * 0x1.0p-53) - 1.0;
        const int i = (int)(e % n), j = (int)(e / n);
        Y[(size_t)i + (size_t)j * ldy] = make_double2(re, im);
    }
}

// y[j] = sum_i conj(V[i, j]) x[i], one wave per column (4 columns per 256-thread block); U
// independent partial sums per lane keep U loads in flight.  For the HEMV of Lanczos (16 n^2
// bytes) U = 4 measured best at n = 2048 (5.8 TB/s) and U = 8 at n = 4096 and 8192 (6.7 and
// 6.1 TB/s, against 6.0 and 5.6 with U = 4).
template <int U>
__global__ __launch_bounds__(256) void k_coldots(int n, int ncols, const zd* V, int ldv, const zd* x, zd* y)
{
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= ncols) return;
    const zd* v = V + (size_t)j * ldv;
    double sr[U], si[U];
#pragma unroll
    for (int u = 0; u < U; ++u) { sr[u] = 0.0; si[u] = 0.0; }
    int i = lane;
    for (; i + 64 * (U - 1) < n; i += 64 * U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const zd a = v[i + 64 * u], b = x[i + 64 * u];
            sr[u] += a.x * b.x + a.y * b.y;
            si[u] += a.x * b.y - a.y * b.x;
        }
    }
    for (; i < n; i += 64) {
        const zd a = v[i], b = x[i];
        sr[0] += a.x * b.x + a.y * b.y;
        si[0] += a.x * b.y - a.y * b.x;
    }
    double tr = 0.0, ti = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        tr += sr[u];
        ti += si[u];
    }
    tr = wave_sum(tr);
    ti = wave_sum(ti);
    if (lane == 0) y[j] = make_double2(tr, ti);
}

// the same for a few columns: one 256-thread block per column
__global__ __launch_bounds__(256) void k_coldots_block(int n, const zd* V, int ldv, const zd* x, zd* y)
{
    __shared__ double sm[8];
    const int j = blockIdx.x;
    const zd* v = V + (size_t)j * ldv;
    double sr[2] = {0, 0}, si[2] = {0, 0};
    int i = threadIdx.x;
    for (; i + 256 < n; i += 512) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const zd a = v[i + 256 * u], b = x[i + 256 * u];
            sr[u] += a.x * b.x + a.y * b.y;
            si[u] += a.x * b.y - a.y * b.x;
        }
    }
    for (; i < n; i += 256) {
        const zd a = v[i], b = x[i];
        sr[0] += a.x * b.x + a.y * b.y;
        si[0] += a.x * b.y - a.y * b.x;
    }
    double tr = wave_sum(sr[0] + sr[1]), ti = wave_sum(si[0] + si[1]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sm[w] = tr;
        sm[4 + w] = ti;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        y[j] = make_double2((sm[0] + sm[1]) + (sm[2] + sm[3]), (sm[4] + sm[5]) + (sm[6] + sm[7]));
}

// x[i] += alpha sum_j V[i, j] c[j]
__global__ __launch_bounds__(256) void k_gemv_n(int n, int ncols, const zd* V, int ldv, const zd* c, double alpha, zd* x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double sr = 0, si = 0;
    for (int j = 0; j < ncols; ++j) {
        const zd a = V[(size_t)i + (size_t)j * ldv], b = c[j];
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
    }
    zd o = x[i];
    o.x += alpha * sr;
    o.y += alpha * si;
    x[i] = o;
}

// r[j] = || HY[:, j] - theta[j] Y[:, j] ||_2, one 256-thread block per column
__global__ __launch_bounds__(256) void k_residual_norms(int n, const zd* HY, int ldhy, const zd* Y, int ldy,
                                                        const double* theta, double* r)
{
    __shared__ double sm[4];
    const int j = blockIdx.x;
    const double th = theta[j];
    const zd* hy = HY + (size_t)j * ldhy;
    const zd* y = Y + (size_t)j * ldy;
    double s = 0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const zd a = hy[i], b = y[i];
        const double dr = a.x - th * b.x, di = a.y - th * b.y;
        s += dr * dr + di * di;
    }
    s = block_sum256(s, sm);
    if (threadIdx.x == 0) r[j] = sqrt(s);
}

// *flag |= 1 if A and B (n x n) differ in any bit
__global__ void k_any_diff(int n, const zd* __restrict__ A, int lda, const zd* __restrict__ B, int ldb, int* flag)
{
    const size_t total = (size_t)n * n;
    int diff = 0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        const zd a = A[(size_t)i + (size_t)j * lda], b = B[(size_t)i + (size_t)j * ldb];
        diff |= (__double_as_longlong(a.x) != __double_as_longlong(b.x)) |
                (__double_as_longlong(a.y) != __double_as_longlong(b.y));
    }
    if (__any(diff) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// d[j] = Re(A[:, j]^H B[:, j]), one 256-thread block per column
__global__ __launch_bounds__(256) void k_pair_dots(int n, const zd* A, int lda, const zd* B, int ldb, double* d)
{
    __shared__ double sm[4];
    const zd* a = A + (size_t)blockIdx.x * lda;
    const zd* b = B + (size_t)blockIdx.x * ldb;
    double s = 0;
    for (int i = threadIdx.x; i < n; i += 256) s += a[i].x * b[i].x + a[i].y * b[i].y;
    s = block_sum256(s, sm);
    if (threadIdx.x == 0) d[blockIdx.x] = s;
}

// D[:, j] = Xc[:, j] - O_jj Xp[:, j]  (the part of each new vector off its predecessor)
__global__ void k_sub_diag_scaled(int n, int m, const zd* Xc, int ldc, const zd* Xp, int ldp, const zd* O, int ldo,
                                  zd* D, int ldd)
{
    const size_t total = (size_t)n * m;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        const zd o = O[(size_t)j * ldo + j], p = Xp[(size_t)j * ldp + i], c = Xc[(size_t)j * ldc + i];
        D[(size_t)j * ldd + i] = make_double2(c.x - (o.x * p.x - o.y * p.y), c.y - (o.x * p.y + o.y * p.x));
    }
}

__global__ __launch_bounds__(256) void k_colnorms(int n, const zd* Y, int ldy, double* r)
{
    __shared__ double sm[4];
    const zd* y = Y + (size_t)blockIdx.x * ldy;
    double s = 0;
    for (int i = threadIdx.x; i < n; i += 256) s += zabs2(y[i]);
    s = block_sum256(s, sm);
    if (threadIdx.x == 0) r[blockIdx.x] = sqrt(s);
}

// column sums of |A_ij| (for Hermitian A these are the row sums)
__global__ __launch_bounds__(256) void k_colabssum(int n, const zd* A, int lda, double* r)
{
    __shared__ double sm[4];
    const zd* a = A + (size_t)blockIdx.x * lda;
    double s = 0;
    for (int i = threadIdx.x; i < n; i += 256) s += sqrt(zabs2(a[i]));
    s = block_sum256(s, sm);
    if (threadIdx.x == 0) r[blockIdx.x] = s;
}

// r[j] = sum_i |A_ij - delta_ij|, one block per column
__global__ __launch_bounds__(256) void k_colabssum_off_identity(int n, const zd* A, int lda, double* r)
{
    __shared__ double sm[4];
    const int j = blockIdx.x;
    const zd* a = A + (size_t)j * lda;
    double s = 0;
    for (int i = threadIdx.x; i < n; i += 256) {
        zd v = a[i];
        if (i == j) v.x -= 1.0;
        s += sqrt(zabs2(v));
    }
    s = block_sum256(s, sm);
    if (threadIdx.x == 0) r[j] = s;
}

// G (m x m) <- F: the strict upper triangle of G, (G_jj - 1) / 2 on the diagonal, zero below
__global__ void k_first_order_factor(int m, zd* G, int ldg)
{
    const size_t total = (size_t)m * m;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % m), j = (int)(e / m);
        zd* g = G + (size_t)i + (size_t)j * ldg;
        if (i > j) *g = make_double2(0.0, 0.0);
        else if (i == j) *g = make_double2(0.5 * (g->x - 1.0), 0.0);
    }
}

// maximum that keeps a NaN once seen (fmax would drop it): a non-finite entry of the input must
// reach the host checks instead of vanishing from the norm
__device__ __forceinline__ double max_keep_nan(double x, double y) { return (y > x || y != y) ? y : x; }

__global__ __launch_bounds__(256) void k_max_reduce(int n, const double* v, double* out)
{
    __shared__ double sm[256];
    double m = 0;
    for (int i = threadIdx.x; i < n; i += 256) m = max_keep_nan(m, v[i]);
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sm[threadIdx.x] = max_keep_nan(sm[threadIdx.x], sm[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sm[0];
}

__global__ void k_scale_cols_inv(int n, int m, zd* Y, int ldy, const double* nrm)
{
    const size_t total = (size_t)n * m;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        const double s = nrm[j] > 0 ? 1.0 / nrm[j] : 0.0;
        zd v = Y[(size_t)i + (size_t)j * ldy];
        Y[(size_t)i + (size_t)j * ldy] = make_double2(v.x * s, v.y * s);
    }
}

// Y[:, j] *= 1/sqrt(d[j]) (0 when d[j] <= 0): columns scaled to unit norm from their squared norms
__global__ void k_scale_cols_rsqrt(int n, int m, zd* Y, int ldy, const double* d)
{
    const size_t total = (size_t)n * m;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        const double s = d[j] > 0 ? 1.0 / sqrt(d[j]) : 0.0;
        zd v = Y[(size_t)i + (size_t)j * ldy];
        Y[(size_t)i + (size_t)j * ldy] = make_double2(v.x * s, v.y * s);
    }
}

// W[:, c] = AX[:, idx[c]] - theta[idx[c]] BX[:, idx[c]]: the residuals of the selected columns
__global__ void k_residual_gather(int n, int na, const zd* AX, int lda, const zd* BX, int ldb, const double* theta,
                                  const int* idx, zd* W, int ldw)
{
    const size_t total = (size_t)n * na;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), c = (int)(e / n);
        const int j = idx[c];
        const double t = theta[j];
        const zd a = AX[(size_t)i + (size_t)j * lda], b = BX[(size_t)i + (size_t)j * ldb];
        W[(size_t)i + (size_t)c * ldw] = make_double2(a.x - t * b.x, a.y - t * b.y);
    }
}

// T[:, c] = U[:, k-1-c] / sqrt(g[k-1-c]) for c < kept (g ascending): the kept eigenvectors of a
// Gram matrix, largest first, scaled so that Y T has orthonormal columns
__global__ void k_orth_factor(int k, int kept, const zd* U, int ldu, const double* g, zd* T, int ldt)
{
    const size_t total = (size_t)k * kept;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % k), c = (int)(e / k);
        const int src = k - 1 - c;
        const double s = 1.0 / sqrt(g[src]);
        const zd u = U[(size_t)i + (size_t)src * ldu];
        T[(size_t)i + (size_t)c * ldt] = make_double2(u.x * s, u.y * s);
    }
}

__global__ void k_add_diag(int m, zd* G, int ldg, const double* shift, double factor)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) G[(size_t)i + (size_t)i * ldg].x += factor * shift[0];
}

__global__ __launch_bounds__(256) void k_fro2(int n, int m, const zd* Y, int ldy, double* out)
{
    __shared__ double sm[4];
    double s = 0;
    for (int j = 0; j < m; ++j)
        for (int i = threadIdx.x; i < n; i += 256) s += zabs2(Y[(size_t)i + (size_t)j * ldy]);
    s = block_sum256(s, sm);
    if (threadIdx.x == 0) out[0] = s;
}

// Lanczos: alpha = Re(v^H w) (given as dots[0]); w <- w - alpha v - beta_prev v_prev
__global__ void k_lanczos_update(int n, const zd* v, zd* w, const zd* vprev, const zd* dot, double* alpha_out,
                                 const double* beta_prev)
{
    const double al = dot[0].x;
    const double be = beta_prev ? beta_prev[0] : 0.0;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) alpha_out[0] = al;
    if (i >= n) return;
    zd o = w[i];
    const zd a = v[i];
    o.x -= al * a.x; o.y -= al * a.y;
    if (vprev) { const zd b = vprev[i]; o.x -= be * b.x; o.y -= be * b.y; }
    w[i] = o;
}

// beta = ||w||, vnext = w / beta  (single block computes the norm, grid then scales)
__global__ __launch_bounds__(256) void k_norm_to(int n, const zd* w, double* beta_out)
{
    __shared__ double sm[4];
    double s = 0;
    for (int i = threadIdx.x; i < n; i += 256) s += zabs2(w[i]);
    s = block_sum256(s, sm);
    if (threadIdx.x == 0) beta_out[0] = sqrt(s);
}

__global__ void k_scale_to(int n, const zd* w, zd* v, const double* beta)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double b = beta[0];
    const double s = b > 1e-300 ? 1.0 / b : 0.0;
    const zd a = w[i];
    v[i] = make_double2(a.x * s, a.y * s);
}

// each column: its largest-magnitude entry (first on ties) made real positive
__global__ __launch_bounds__(256) void k_phase_normalize(int m, zd* W, int ldw)
{
    __shared__ double sv[256];
    __shared__ int si[256];
    zd* w = W + (size_t)blockIdx.x * ldw;
    // start from index 0 so that a column of NaNs still yields an in-range index
    double best = -1;
    int bi = 0;
    for (int i = threadIdx.x; i < m; i += 256) {
        const double a = zabs2(w[i]);
        if (a > best) { best = a; bi = i; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double a = sv[threadIdx.x + o];
            const int ia = si[threadIdx.x + o];
            if (a > sv[threadIdx.x] || (a == sv[threadIdx.x] && ia < si[threadIdx.x])) {
                sv[threadIdx.x] = a;
                si[threadIdx.x] = ia;
            }
        }
        __syncthreads();
    }
    const int imax = si[0];
    const zd p = w[imax];
    const double ap = sqrt(zabs2(p));
    __syncthreads();
    if (!(ap > 0)) return;
    const zd ph = make_double2(p.x / ap, -p.y / ap);   // conj(phase)
    for (int i = threadIdx.x; i < m; i += 256) {
        if (i == imax) continue;
        w[i] = zmul(w[i], ph);
    }
    __syncthreads();
    if (threadIdx.x == 0) w[imax] = make_double2(ap, 0.0);
}

__global__ void k_any_nonfinite(int n, const double* v, int* flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(v[i])) atomicOr(flag, 1);
}

__global__ void k_permute_cols(int n, int m, const zd* src, int lds, zd* dst, int ldd, const int* perm)
{
    const size_t total = (size_t)n * m;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        dst[(size_t)i + (size_t)j * ldd] = src[(size_t)i + (size_t)perm[j] * lds];
    }
}

template <typename C2>
__global__ void k_copy_cols_flag(int n, int m, const C2* src, int lds, C2* dst, int ldd, const int* flag)
{
    const size_t total = (size_t)n * m;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        if (flag[j]) dst[(size_t)i + (size_t)j * ldd] = src[(size_t)i + (size_t)j * lds];
    }
}

__global__ void k_zero_upper(int n, zd* L, int ldl)
{
    const size_t total = (size_t)n * n;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        if (i < j) L[(size_t)i + (size_t)j * ldl] = make_double2(0.0, 0.0);
    }
}

__global__ void k_add_diag_const(int m, zd* G, int ldg, double shift)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) G[(size_t)i + (size_t)i * ldg].x += shift;
}

// Y1 = alpha (HY - shift Y0) on columns [0, w): the first step of the scaled recurrence
// (beta = 0) when the block's image H Y0 is already known (the previous Rayleigh-Ritz step's)
template <typename T2>
__global__ __launch_bounds__(256) void k_first_step(int n, int w, double alpha, double shift, const zd* __restrict__ HY,
                                                    int ldhy, const T2* __restrict__ Y0, int ldy0, T2* __restrict__ Y1,
                                                    int ldy1)
{
    const size_t total = (size_t)n * w;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        const zd hy = HY[(size_t)i + (size_t)j * ldhy];
        const T2 y = Y0[(size_t)i + (size_t)j * ldy0];
        T2 o;
        o.x = alpha * (hy.x - shift * (double)y.x);
        o.y = alpha * (hy.y - shift * (double)y.y);
        Y1[(size_t)i + (size_t)j * ldy1] = o;
    }
}

inline int grid_for(size_t total)
{
    size_t b = (total + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

int launch_zlacpy(hipStream_t s, int M, int N, const zd* A, int lda, zd* B, int ldb)
{
    if (M <= 0 || N <= 0) return 0;
    hipLaunchKernelGGL(k_zlacpy, dim3(grid_for((size_t)M * N)), dim3(256), 0, s, M, N, A, lda, B, ldb);
    return (int)hipGetLastError();
}

int launch_z2c(hipStream_t s, int M, int N, const zd* A, int lda, zf* B, int ldb)
{
    if (M <= 0 || N <= 0) return 0;
    hipLaunchKernelGGL(k_z2c, dim3(grid_for((size_t)M * N)), dim3(256), 0, s, M, N, A, lda, B, ldb);
    return (int)hipGetLastError();
}

int launch_c2z(hipStream_t s, int M, int N, const zf* A, int lda, zd* B, int ldb)
{
    if (M <= 0 || N <= 0) return 0;
    hipLaunchKernelGGL(k_c2z, dim3(grid_for((size_t)M * N)), dim3(256), 0, s, M, N, A, lda, B, ldb);
    return (int)hipGetLastError();
}


int launch_mirror_lower(hipStream_t s, int n, zd* H, int ldh)
{
    if (n <= 0) return 0;
    const int t = (n + 31) / 32;
    hipLaunchKernelGGL(k_mirror_lower, dim3(t, t), dim3(256), 0, s, n, H, ldh);
    return (int)hipGetLastError();
}

int launch_philox_block(hipStream_t s, unsigned long long seed, unsigned long long stream, int n, int m, zd* Y, int ldy)
{
    if (n <= 0 || m <= 0) return 0;
    hipLaunchKernelGGL(k_philox_block, dim3(grid_for((size_t)n * m)), dim3(256), 0, s, (uint64_t)seed,
                       (uint64_t)stream, n, m, Y, ldy);
    return (int)hipGetLastError();
}

int launch_coldots(hipStream_t s, int n, int ncols, const zd* V, int ldv, const zd* x, zd* y)
{
    if (ncols <= 0) return 0;
    if (ncols <= 256)   // too few columns to fill the device one wave each
        hipLaunchKernelGGL(k_coldots_block, dim3(ncols), dim3(256), 0, s, n, V, ldv, x, y);
    else if (n <= 3072)
        hipLaunchKernelGGL(k_coldots<4>, dim3((ncols + 3) / 4), dim3(256), 0, s, n, ncols, V, ldv, x, y);
    else
        hipLaunchKernelGGL(k_coldots<8>, dim3((ncols + 3) / 4), dim3(256), 0, s, n, ncols, V, ldv, x, y);
    return (int)hipGetLastError();
}

int launch_gemv_n(hipStream_t s, int n, int ncols, const zd* V, int ldv, const zd* c, double alpha, zd* x)
{
    if (n <= 0 || ncols <= 0) return 0;
    hipLaunchKernelGGL(k_gemv_n, dim3((n + 255) / 256), dim3(256), 0, s, n, ncols, V, ldv, c, alpha, x);
    return (int)hipGetLastError();
}

int launch_residual_norms(hipStream_t s, int n, int m, const zd* HY, int ldhy, const zd* Y, int ldy,
                          const double* theta, double* r)
{
    if (m <= 0) return 0;
    hipLaunchKernelGGL(k_residual_norms, dim3(m), dim3(256), 0, s, n, HY, ldhy, Y, ldy, theta, r);
    return (int)hipGetLastError();
}

int launch_any_diff(hipStream_t s, int n, const zd* A, int lda, const zd* B, int ldb, int* flag)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_any_diff, dim3(grid_for((size_t)n * n)), dim3(256), 0, s, n, A, lda, B, ldb, flag);
    return (int)hipGetLastError();
}

int launch_scale_cols_rsqrt(hipStream_t s, int n, int m, zd* Y, int ldy, const double* d)
{
    if (n <= 0 || m <= 0) return 0;
    hipLaunchKernelGGL(k_scale_cols_rsqrt, dim3(grid_for((size_t)n * m)), dim3(256), 0, s, n, m, Y, ldy, d);
    return (int)hipGetLastError();
}

int launch_residual_gather(hipStream_t s, int n, int na, const zd* AX, int lda, const zd* BX, int ldb,
                           const double* theta, const int* idx, zd* W, int ldw)
{
    if (n <= 0 || na <= 0) return 0;
    hipLaunchKernelGGL(k_residual_gather, dim3(grid_for((size_t)n * na)), dim3(256), 0, s, n, na, AX, lda, BX, ldb,
                       theta, idx, W, ldw);
    return (int)hipGetLastError();
}

int launch_orth_factor(hipStream_t s, int k, int kept, const zd* U, int ldu, const double* g, zd* T, int ldt)
{
    if (k <= 0 || kept <= 0) return 0;
    hipLaunchKernelGGL(k_orth_factor, dim3(grid_for((size_t)k * kept)), dim3(256), 0, s, k, kept, U, ldu, g, T, ldt);
    return (int)hipGetLastError();
}

int launch_pair_dots(hipStream_t s, int n, int m, const zd* A, int lda, const zd* B, int ldb, double* d)
{
    if (m <= 0) return 0;
    hipLaunchKernelGGL(k_pair_dots, dim3(m), dim3(256), 0, s, n, A, lda, B, ldb, d);
    return (int)hipGetLastError();
}

int launch_sub_diag_scaled(hipStream_t s, int n, int m, const zd* Xc, int ldc, const zd* Xp, int ldp, const zd* O,
                           int ldo, zd* D, int ldd)
{
    if (n <= 0 || m <= 0) return 0;
    hipLaunchKernelGGL(k_sub_diag_scaled, dim3(grid_for((size_t)n * m)), dim3(256), 0, s, n, m, Xc, ldc, Xp, ldp, O,
                       ldo, D, ldd);
    return (int)hipGetLastError();
}

int launch_colnorms(hipStream_t s, int n, int m, const zd* Y, int ldy, double* r)
{
    if (m <= 0) return 0;
    hipLaunchKernelGGL(k_colnorms, dim3(m), dim3(256), 0, s, n, Y, ldy, r);
    return (int)hipGetLastError();
}

int launch_scale_cols_inv(hipStream_t s, int n, int m, zd* Y, int ldy, const double* nrm)
{
    if (n <= 0 || m <= 0) return 0;
    hipLaunchKernelGGL(k_scale_cols_inv, dim3(grid_for((size_t)n * m)), dim3(256), 0, s, n, m, Y, ldy, nrm);
    return (int)hipGetLastError();
}

// out[0] = max_j ||A[:, j]||; uses out[1 .. n] as scratch
int launch_max_colnorm(hipStream_t s, int n, const zd* A, int lda, double* out)
{
    hipLaunchKernelGGL(k_colnorms, dim3(n), dim3(256), 0, s, n, A, lda, out + 1);
    hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, n, out + 1, out);
    return (int)hipGetLastError();
}

// out[0] = ||A||_inf for Hermitian A (max column abs-sum); uses out[1 .. n] as scratch
int launch_max_rowsum_abs(hipStream_t s, int n, const zd* A, int lda, double* out)
{
    hipLaunchKernelGGL(k_colabssum, dim3(n), dim3(256), 0, s, n, A, lda, out + 1);
    hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, n, out + 1, out);
    return (int)hipGetLastError();
}

int launch_max_rowsum_off_identity(hipStream_t s, int n, const zd* A, int lda, double* out)
{
    hipLaunchKernelGGL(k_colabssum_off_identity, dim3(n), dim3(256), 0, s, n, A, lda, out + 1);
    hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, n, out + 1, out);
    return (int)hipGetLastError();
}

int launch_first_order_factor(hipStream_t s, int m, zd* G, int ldg)
{
    if (m <= 0) return 0;
    hipLaunchKernelGGL(k_first_order_factor, dim3(grid_for((size_t)m * m)), dim3(256), 0, s, m, G, ldg);
    return (int)hipGetLastError();
}

int launch_add_diag(hipStream_t s, int m, zd* G, int ldg, const double* shift_dev, double factor)
{
    hipLaunchKernelGGL(k_add_diag, dim3((m + 255) / 256), dim3(256), 0, s, m, G, ldg, shift_dev, factor);
    return (int)hipGetLastError();
}

int launch_fro2(hipStream_t s, int n, int m, const zd* Y, int ldy, double* out)
{
    hipLaunchKernelGGL(k_fro2, dim3(1), dim3(256), 0, s, n, m, Y, ldy, out);
    return (int)hipGetLastError();
}

// dot scratch: alpha_out[1..2] holds the complex dot product v^H w
int launch_lanczos_alpha(hipStream_t s, int n, const zd* v, zd* w, const zd* vprev, double* alpha_out,
                         const double* beta_prev, zd* dot)
{
    hipLaunchKernelGGL(k_coldots_block, dim3(1), dim3(256), 0, s, n, v, n, w, dot);
    hipLaunchKernelGGL(k_lanczos_update, dim3((n + 255) / 256), dim3(256), 0, s, n, v, w, vprev, dot, alpha_out,
                       beta_prev);
    return (int)hipGetLastError();
}

int launch_lanczos_normalize(hipStream_t s, int n, const zd* w, zd* vnext, double* beta_out)
{
    hipLaunchKernelGGL(k_norm_to, dim3(1), dim3(256), 0, s, n, w, beta_out);
    hipLaunchKernelGGL(k_scale_to, dim3((n + 255) / 256), dim3(256), 0, s, n, w, vnext, beta_out);
    return (int)hipGetLastError();
}

int launch_phase_normalize(hipStream_t s, int m, int ncols, zd* W, int ldw)
{
    if (ncols <= 0) return 0;
    hipLaunchKernelGGL(k_phase_normalize, dim3(ncols), dim3(256), 0, s, m, W, ldw);
    return (int)hipGetLastError();
}

int launch_any_nonfinite(hipStream_t s, int n, const double* v, int* flag)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_any_nonfinite, dim3((n + 255) / 256), dim3(256), 0, s, n, v, flag);
    return (int)hipGetLastError();
}

int launch_permute_cols(hipStream_t s, int n, int m, const zd* src, int lds, zd* dst, int ldd, const int* perm)
{
    if (n <= 0 || m <= 0) return 0;
    hipLaunchKernelGGL(k_permute_cols, dim3(grid_for((size_t)n * m)), dim3(256), 0, s, n, m, src, lds, dst, ldd, perm);
    return (int)hipGetLastError();
}

int launch_copy_cols_flag(hipStream_t s, int n, int m, const zd* src, int lds, zd* dst, int ldd, const int* flag)
{
    if (n <= 0 || m <= 0) return 0;
    hipLaunchKernelGGL(k_copy_cols_flag<zd>, dim3(grid_for((size_t)n * m)), dim3(256), 0, s, n, m, src, lds, dst,
                       ldd, flag);
    return (int)hipGetLastError();
}

int launch_copy_cols_flag_c(hipStream_t s, int n, int m, const zf* src, int lds, zf* dst, int ldd, const int* flag)
{
    if (n <= 0 || m <= 0) return 0;
    hipLaunchKernelGGL(k_copy_cols_flag<zf>, dim3(grid_for((size_t)n * m)), dim3(256), 0, s, n, m, src, lds, dst,
                       ldd, flag);
    return (int)hipGetLastError();
}

int launch_zero_upper(hipStream_t s, int n, zd* L, int ldl)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_zero_upper, dim3(grid_for((size_t)n * n)), dim3(256), 0, s, n, L, ldl);
    return (int)hipGetLastError();
}

int launch_add_diag_const(hipStream_t s, int m, zd* G, int ldg, double shift)
{
    if (m <= 0) return 0;
    hipLaunchKernelGGL(k_add_diag_const, dim3((m + 255) / 256), dim3(256), 0, s, m, G, ldg, shift);
    return (int)hipGetLastError();
}

int launch_first_step(hipStream_t s, int n, int w, double alpha, double shift, const zd* HY, int ldhy, const zd* Y0,
                      int ldy0, zd* Y1, int ldy1)
{
    if (n <= 0 || w <= 0) return 0;
    hipLaunchKernelGGL(k_first_step<zd>, dim3(grid_for((size_t)n * w)), dim3(256), 0, s, n, w, alpha, shift, HY, ldhy,
                       Y0, ldy0, Y1, ldy1);
    return (int)hipGetLastError();
}

int launch_first_step(hipStream_t s, int n, int w, double alpha, double shift, const zd* HY, int ldhy, const zf* Y0,
                      int ldy0, zf* Y1, int ldy1)
{
    if (n <= 0 || w <= 0) return 0;
    hipLaunchKernelGGL(k_first_step<zf>, dim3(grid_for((size_t)n * w)), dim3(256), 0, s, n, w, alpha, shift, HY, ldhy,
                       Y0, ldy0, Y1, ldy1);
    return (int)hipGetLastError();
}
