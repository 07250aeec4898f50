// Hermitian eigensolver for the Rayleigh quotient G = Y^H H Y of the Rayleigh-Ritz step
// (Algorithm 1), sized for blocks of a few hundred columns: parallel two-sided block Jacobi.
//
// G (m x m) is embedded in an M x M matrix, M = m rounded up to a multiple of 32, with the padded
// diagonal set to 1e30 and zero coupling (padded indices are never rotated and sort last).  The
// M / 16 blocks of 16 indices meet in round-robin order: a sweep has nb - 1 rounds (nb = M / 16),
// and in each round every pair of blocks forms a 32 x 32 Hermitian subproblem.
//   k_eig_inner  one workgroup per block pair runs one cyclic Jacobi sweep on its subproblem in
//                LDS (complex 2 x 2 rotations, round-robin over the 32 indices; a round in which
//                no pair exceeds the threshold is skipped) and writes the accumulated rotation J.
//                A single inner sweep per round costs at most one extra outer sweep and halves or
//                better the inner work.
//   k_eig_apply  G <- J^H G J and W <- W J, one workgroup per 32 x 32 tile (products on the FP64
//                MFMA); J is block diagonal in block-pair order, so every tile is touched by
//                exactly one workgroup.
// After each sweep the largest off-diagonal modulus and the diagonal are copied to the host, which
// stops once the off-diagonal is below 5e-14 of the matrix scale or below the caller's level
// (rotations are skipped below a fifth of that level).  A
// Rayleigh quotient of nearly converged Ritz vectors is nearly diagonal (its off-diagonal entries
// are bounded by the residual norms), so the later loops of a solve need two or three sweeps.
//
// Complex rotation of the pair (p, q) with a = G_pp, b = G_qq (real) and g = G_pq = |g| e^{i phi}:
// the real symmetric Schur rotation of [[a, |g|], [|g|, b]] (zeta = (b - a) / (2 |g|),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2), s = t c; Golub and Van
// Loan, Matrix Computations, section 8.5) conjugated by diag(1, e^{-i phi}):
//   R = [[c, s e^{i phi}], [-s e^{-i phi}, c]],   R^H G R diagonal.
// With d = (b - a) / 2 and rho = sqrt(d^2 + |g|^2): c^2 = (1 + |d| / rho) / 2 and
// s e^{i phi} = sign(d) g / (2 rho c), so two reciprocal square roots suffice and |g| itself is never
// needed (the threshold test compares |g|^2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.h"
#include "gemm_tile.h"

namespace {

constexpr int EB = 16;        // indices per block
constexpr int ES = 2 * EB;    // order of a block-pair subproblem
constexpr int EP = ES + 1;    // LDS row pitch
constexpr double PAD = 1e30;  // diagonal of the padded indices

// round-robin pair i of round r among n (even) players: player n-1 meets r, the others rotate
__host__ __device__ inline void rr_pair(int n, int r, int i, int& a, int& b)
{
    if (i == 0) {
        a = r;
        b = n - 1;
    } else {
        a = (r + i) % (n - 1);
        b = (r - i + (n - 1)) % (n - 1);
    }
}

__device__ inline zd zconjd(zd a) { return make_double2(a.x, -a.y); }
__device__ inline zd zaxpy(double c, zd x, zd s, zd y) { zd p = zmul(s, y); return make_double2(c * x.x + p.x, c * x.y + p.y); }

// global index of subproblem index u for the block pair (P, Q)
__device__ inline int sub_index(int P, int Q, int u) { return u < EB ? P * EB + u : Q * EB + (u - EB); }

// per column j < m of the Hermitian G: stat[j] = max_{i != j} |G_ij|, stat[m + j] = Re G_jj
__global__ __launch_bounds__(256) void k_eig_rowstat(int m, const zd* __restrict__ G, int ldg, double* __restrict__ stat)
{
    __shared__ double sm[256];
    const int j = blockIdx.x;
    double o = 0;
    for (int i = threadIdx.x; i < m; i += 256) {
        if (i == j) continue;
        const zd g = G[(size_t)i + (size_t)j * ldg];
        o = fmax(o, sqrt(g.x * g.x + g.y * g.y));
    }
    sm[threadIdx.x] = o;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        stat[j] = sm[0];
        stat[m + j] = G[(size_t)j + (size_t)j * ldg].x;
    }
}

// Gp (M x M) = [G(act, act) 0; 0 PAD I] for the k active indices act[0 .. k); Wp = I
__global__ __launch_bounds__(256) void k_eig_compress(int k, int M, const zd* __restrict__ G, int ldg,
                                                      const int* __restrict__ act, zd* __restrict__ Gp,
                                                      zd* __restrict__ Wp)
{
    const size_t total = (size_t)M * M;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % M), j = (int)(e / M);
        zd g = make_double2(0.0, 0.0);
        if (i < k && j < k) {
            // the Hermitian part (G + G^H) / 2: a Gram or Rayleigh quotient whose factors were
            // updated rather than recomputed is Hermitian only up to their drift, and an
            // anti-Hermitian remainder above the stopping level would never be rotated away
            const zd a = G[(size_t)act[i] + (size_t)act[j] * ldg], b = G[(size_t)act[j] + (size_t)act[i] * ldg];
            g = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
        } else if (i == j) {
            g.x = PAD;
        }
        if (i == j) g.y = 0.0;
        Gp[e] = g;
        Wp[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
}

// Kernel A: workgroup w diagonalises the subproblem of block pair w of round `round` (512 threads:
// two per 2 x 2 block, so that two waves per SIMD hide the latency of the rotation updates).
__global__ __launch_bounds__(512) void k_eig_inner(int M, int nb, int round, const zd* __restrict__ Gp,
                                                   zd* __restrict__ J, const double* __restrict__ scale)
{
    __shared__ zd A2[2][ES * EP];
    __shared__ zd V[ES * EP];
    __shared__ double rc[ES / 2];
    __shared__ zd rs[ES / 2];
    __shared__ int rot[ES];
    const int tid = threadIdx.x;
    int P, Q;
    rr_pair(nb, round, blockIdx.x, P, Q);
    #pragma unroll
    for (int e = tid; e < ES * ES; e += 512) {
        const int u = e % ES, v = e / ES;
        A2[0][u * EP + v] = Gp[(size_t)sub_index(P, Q, u) + (size_t)sub_index(P, Q, v) * M];
        V[u * EP + v] = make_double2(u == v ? 1.0 : 0.0, 0.0);
    }
    if (tid < ES) rot[tid] = 0;
    const double tol2 = scale[1];   // squared rotation threshold
    // this thread's 2 x 2 block (pair bi, pair bj), its row `half` (pi or qi) and row bi + 16 half
    // of V (pair bj); the subproblem is double-buffered, since both rows of a block read all four
    // of its entries
    const int bi = (tid & 255) / (ES / 2), bj = tid % (ES / 2), half = tid >> 8;
    int cur = 0;
    __syncthreads();
    for (int r = 0; r < ES - 1; ++r) {
        const zd* A = A2[cur];
        if (tid < ES / 2) {
            int p, q;
            rr_pair(ES, r, tid, p, q);
            const zd g = A[p * EP + q];
            const double g2 = g.x * g.x + g.y * g.y;
            double c = 1.0;
            zd se = make_double2(0.0, 0.0);
            if (g2 > tol2) {
                // cos^2 = (1 + |d| / rho) / 2, s e^{i phi} = sign(d) g / (2 rho cos), rho = sqrt(d^2 + |g|^2):
                // two reciprocal square roots, no cancellation (|d| / rho >= 0)
                const double d = 0.5 * (A[q * EP + q].x - A[p * EP + p].x);
                const double irho = rsqrt_nr(d * d + g2);
                const double w = 0.5 + 0.5 * fabs(d) * irho;
                const double ic = rsqrt_nr(w);
                c = w * ic;
                const double f = (d >= 0 ? 0.5 : -0.5) * irho * ic;
                se = make_double2(f * g.x, f * g.y);
                rot[r] = 1;
            }
            rc[tid] = c;
            rs[tid] = se;
        }
        __syncthreads();
        if (rot[r]) {
            zd* An = A2[cur ^ 1];
            int pi, qi, pj, qj;
            rr_pair(ES, r, bi, pi, qi);
            rr_pair(ES, r, bj, pj, qj);
            const double ci = rc[bi], cj = rc[bj];
            const zd si = rs[bi], sj = rs[bj];
            const zd b00 = A[pi * EP + pj], b01 = A[pi * EP + qj], b10 = A[qi * EP + pj], b11 = A[qi * EP + qj];
            // T = B R_j,  R = [[c, s], [-conj(s), c]];  B' = R_i^H T,  R^H = [[c, -s], [conj(s), c]]
            const zd nsj = make_double2(-sj.x, sj.y);   // -conj(s_j)
            const zd t00 = zaxpy(cj, b00, nsj, b01), t01 = zaxpy(cj, b01, sj, b00);
            const zd t10 = zaxpy(cj, b10, nsj, b11), t11 = zaxpy(cj, b11, sj, b10);
            const zd msi = make_double2(-si.x, -si.y), csi = zconjd(si);
            if (half == 0) {   // row pi
                zd o00 = zaxpy(ci, t00, msi, t10), o01 = zaxpy(ci, t01, msi, t11);
                if (bi == bj) { o01 = make_double2(0.0, 0.0); o00.y = 0.0; }   // the rotated diagonal block is real diagonal
                An[pi * EP + pj] = o00;
                An[pi * EP + qj] = o01;
            } else {           // row qi
                zd o10 = zaxpy(ci, t10, csi, t00), o11 = zaxpy(ci, t11, csi, t01);
                if (bi == bj) { o10 = make_double2(0.0, 0.0); o11.y = 0.0; }
                An[qi * EP + pj] = o10;
                An[qi * EP + qj] = o11;
            }
            const int u = bi + half * (ES / 2);   // V <- V R on row u
            const zd vp = V[u * EP + pj], vq = V[u * EP + qj];
            V[u * EP + pj] = zaxpy(cj, vp, nsj, vq);
            V[u * EP + qj] = zaxpy(cj, vq, sj, vp);
            cur ^= 1;
        }
        __syncthreads();
    }
    zd* Jw = J + (size_t)blockIdx.x * ES * ES;
    #pragma unroll
    for (int e = tid; e < ES * ES; e += 512) {
        const int u = e % ES, v = e / ES;
        Jw[e] = V[u * EP + v];
    }
}

// 32 x 32 complex product op(A) B on the FP64 MFMA (v_mfma_f64_16x16x4f64, four real products per
// complex one), A and B in LDS with pitch EP, op(A) = A or (CONJ_A) A^H.  Each of the 4 waves forms
// one 16 x 16 output tile: register r of lane l holds row 16 (wave & 1) + (l & 15) and column
// 16 (wave >> 1) + 4 r + (l >> 4).
template <bool CONJ_A>
__device__ inline void cgemm32(const zd* A, const zd* B, d4& cr, d4& ci)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = 16 * (wave & 1) + (lane & 15), col = 16 * (wave >> 1) + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) { cr[r] = 0.0; ci[r] = 0.0; }
#pragma unroll
    for (int kk = 0; kk < ES / 4; ++kk) {
        const int k = 4 * kk + (lane >> 4);
        const zd a = CONJ_A ? zconjd(A[k * EP + row]) : A[row * EP + k];
        const zd b = B[k * EP + col];
        cr = chfsi_tile::mfma16(b.x, a.x, cr);
        ci = chfsi_tile::mfma16(b.y, a.x, ci);
        cr = chfsi_tile::mfma16(-b.y, a.y, cr);
        ci = chfsi_tile::mfma16(b.x, a.y, ci);
    }
}

// Kernel B: G <- J^H G J on the (pair p, pair q) tiles, W <- W J on (32-row slab, pair q) tiles.
__global__ __launch_bounds__(256) void k_eig_apply(int M, int nb, int round, zd* __restrict__ Gp, zd* __restrict__ Wp,
                                                   const zd* __restrict__ J)
{
    __shared__ zd X[ES * EP];
    __shared__ zd Jq[ES * EP];
    __shared__ zd Jp[ES * EP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int npair = nb / 2;
    const int b = blockIdx.x;
    const bool gpart = b < npair * npair;
    int p = 0, q, slab = 0;
    if (gpart) {
        p = b / npair;
        q = b % npair;
    } else {
        slab = (b - npair * npair) / npair;
        q = (b - npair * npair) % npair;
    }
    int Pp, Qp, Pq, Qq;
    rr_pair(nb, round, p, Pp, Qp);
    rr_pair(nb, round, q, Pq, Qq);
    #pragma unroll
    for (int e = tid; e < ES * ES; e += 256) {
        const int u = e % ES, v = e / ES;
        const size_t col = (size_t)sub_index(Pq, Qq, v) * M;
        X[u * EP + v] = gpart ? Gp[(size_t)sub_index(Pp, Qp, u) + col] : Wp[(size_t)slab * ES + u + col];
        Jq[u * EP + v] = J[(size_t)q * ES * ES + e];
        if (gpart) Jp[u * EP + v] = J[(size_t)p * ES * ES + e];
    }
    __syncthreads();
    d4 tr, ti;
    cgemm32<false>(X, Jq, tr, ti);   // T = X Jq
    const int row = 16 * (wave & 1) + (lane & 15);
    if (!gpart) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int col = 16 * (wave >> 1) + 4 * r + (lane >> 4);
            Wp[(size_t)slab * ES + row + (size_t)sub_index(Pq, Qq, col) * M] = make_double2(tr[r], ti[r]);
        }
        return;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) X[row * EP + 16 * (wave >> 1) + 4 * r + (lane >> 4)] = make_double2(tr[r], ti[r]);
    __syncthreads();
    d4 gr, gi;
    cgemm32<true>(Jp, X, gr, gi);    // G' = Jp^H T
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int col = 16 * (wave >> 1) + 4 * r + (lane >> 4);
        Gp[(size_t)sub_index(Pp, Qp, row) + (size_t)sub_index(Pq, Qq, col) * M] = make_double2(gr[r], gi[r]);
    }
}

// out[0] = max |G_ij| over i != j < m (real indices); out[1 + i] = Re G_ii for i < M
__global__ __launch_bounds__(256) void k_eig_colmax(int m, int M, const zd* __restrict__ Gp, double* __restrict__ colmax,
                                                    double* __restrict__ out)
{
    __shared__ double sm[256];
    const int j = blockIdx.x;
    double o = 0;
    if (j < m)
        for (int i = threadIdx.x; i < m; i += 256) {
            if (i == j) continue;
            const zd g = Gp[(size_t)i + (size_t)j * M];
            o = fmax(o, sqrt(g.x * g.x + g.y * g.y));
        }
    sm[threadIdx.x] = o;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        colmax[j] = sm[0];
        out[1 + j] = Gp[(size_t)j + (size_t)j * M].x;
    }
}

__global__ __launch_bounds__(256) void k_eig_maxreduce(int M, const double* __restrict__ colmax, double* __restrict__ out)
{
    __shared__ double sm[256];
    double o = 0;
    for (int i = threadIdx.x; i < M; i += 256) o = fmax(o, colmax[i]);
    sm[threadIdx.x] = o;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sm[0];
}

// Eigenvectors of G in ascending order: column c of W is e_{-src[c]-1} when src[c] < 0 (a
// deflated index) and otherwise column src[c] of Wp scattered to the rows act[0 .. k); theta[c] =
// val[c].  pos[i] = position of row i in act, or -1.
__global__ __launch_bounds__(256) void k_eig_expand(int m, int M, const zd* __restrict__ Wp, const int* __restrict__ src,
                                                    const int* __restrict__ pos, const double* __restrict__ val,
                                                    zd* __restrict__ W, int ldw, double* __restrict__ theta)
{
    const size_t total = (size_t)m * m;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % m), c = (int)(e / m);
        const int sc = src[c];
        zd w = make_double2(0.0, 0.0);
        if (sc < 0) w.x = (i == -sc - 1) ? 1.0 : 0.0;
        else if (pos[i] >= 0) w = Wp[(size_t)pos[i] + (size_t)sc * M];
        W[(size_t)i + (size_t)c * ldw] = w;
        if (i == 0) theta[c] = val[c];
    }
}

int grid_for(size_t n)
{
    size_t g = (n + 255) / 256;
    return (int)std::min<size_t>(std::max<size_t>(g, 1), 4096);
}

}  // namespace

int eig_padded_order(int m) { return ((m + ES - 1) / ES) * ES; }

size_t eig_host_doubles(int m) { return 3 * (size_t)eig_padded_order(m) + 8; }

size_t eig_work_bytes(int m)
{
    const size_t M = (size_t)eig_padded_order(m);
    return (2 * M * M + (M / ES) * ES * ES) * sizeof(zd) + (4 * M + 16) * sizeof(double) + 4 * M * sizeof(int) + 1024;
}

// Eigen-decomposition G = W diag(theta) W^H of the Hermitian m x m matrix G (device, leading
// dimension ldg; its Hermitian part (G + G^H) / 2 is decomposed): on return G holds W (columns
// ascending in theta), theta[m] (device) the eigenvalues.  Indices whose whole off-diagonal row is below the stopping threshold are already
// eigenpairs of G to that accuracy (deflated): block Jacobi runs on the remaining k x k part only,
// which in the late loops of a solve is a small fraction of m.  work: eig_work_bytes(m) bytes of
// device memory; host: eig_host_doubles(m) doubles of host memory (pinned for speed).
// *sweeps receives the sweeps taken.  Returns a hipError_t as int, or -1 when 40 sweeps did not
// reach the threshold.
int eig_jacobi(hipStream_t s, int m, zd* G, int ldg, double* theta, void* work, double* host, int* sweeps,
               double stop_abs)
{
    if (sweeps) *sweeps = 0;
    if (m <= 0) return 0;
    const int Mm = eig_padded_order(m);
    char* w = (char*)work;
    zd* Gp = (zd*)w;
    zd* Wp = Gp + (size_t)Mm * Mm;
    zd* J = Wp + (size_t)Mm * Mm;
    double* dbuf = (double*)(J + (size_t)(Mm / ES) * ES * ES);
    double* stat = dbuf;                  // [2 m]: row off-diagonal maxima, diagonal
    double* colmax = dbuf + 2 * Mm;       // [Mm]
    double* outd = colmax + Mm;           // [Mm + 1]: off max, diagonal of Gp
    double* scl = outd + Mm + 1;          // [4]: scale, threshold^2
    int* iw = (int*)(scl + 4);            // act [Mm], src [Mm], pos [Mm]
    hipLaunchKernelGGL(k_eig_rowstat, dim3(m), dim3(256), 0, s, m, (const zd*)G, ldg, stat);
    int rc = (int)hipMemcpyAsync(host, stat, sizeof(double) * 2 * m, hipMemcpyDeviceToHost, s);
    if (rc == 0) rc = (int)hipStreamSynchronize(s);
    if (rc != 0) return rc;
    double sc = 0;
    for (int j = 0; j < m; ++j) sc = std::max(sc, std::max(host[j], std::fabs(host[m + j])));
    const double stop = std::max(5e-14 * sc, stop_abs);   // off-diagonal target
    const double rot = 0.2 * stop;                         // rotations below this are skipped
    std::vector<int> act, pos(m, -1);
    std::vector<double> dval(m);
    for (int j = 0; j < m; ++j) {
        dval[j] = host[m + j];
        if (host[j] > stop) { pos[j] = (int)act.size(); act.push_back(j); }
    }
    const int k = (int)act.size();
    std::vector<double> aval;              // eigenvalues of the active part (compressed order)
    int sw = 0;
    if (k > 0) {
        const int M = eig_padded_order(k), nb = M / EB, npair = nb / 2;
        // staged through the (pinned) host buffer; the first sweep's synchronisation retires the
        // copies before that part of the buffer is written again
        int* hact = (int*)(host + Mm + 8);
        double* hs = host + 2 * Mm + 8;
        std::memcpy(hact, act.data(), sizeof(int) * k);
        hs[0] = sc;
        hs[1] = rot * rot;
        rc = (int)hipMemcpyAsync(iw, hact, sizeof(int) * k, hipMemcpyHostToDevice, s);
        if (rc == 0) rc = (int)hipMemcpyAsync(scl, hs, sizeof(double) * 2, hipMemcpyHostToDevice, s);
        if (rc != 0) return rc;
        hipLaunchKernelGGL(k_eig_compress, dim3(grid_for((size_t)M * M)), dim3(256), 0, s, k, M, (const zd*)G, ldg,
                           (const int*)iw, Gp, Wp);
        bool done = false;
        while (!done && sw < 40) {
            for (int r = 0; r < nb - 1; ++r) {
                hipLaunchKernelGGL(k_eig_inner, dim3(npair), dim3(512), 0, s, M, nb, r, (const zd*)Gp, J,
                                   (const double*)scl);
                hipLaunchKernelGGL(k_eig_apply, dim3(npair * npair + (M / ES) * npair), dim3(256), 0, s, M, nb, r,
                                   Gp, Wp, (const zd*)J);
            }
            ++sw;
            hipLaunchKernelGGL(k_eig_colmax, dim3(M), dim3(256), 0, s, k, M, (const zd*)Gp, colmax, outd);
            hipLaunchKernelGGL(k_eig_maxreduce, dim3(1), dim3(256), 0, s, M, (const double*)colmax, outd);
            rc = (int)hipMemcpyAsync(host, outd, sizeof(double) * (M + 1), hipMemcpyDeviceToHost, s);
            if (rc == 0) rc = (int)hipStreamSynchronize(s);
            if (rc != 0) return rc;
            done = host[0] <= stop;
        }
        if (sweeps) *sweeps = sw;
        if (!done) return -1;
        aval.assign(host + 1, host + 1 + k);
    }
    // ascending order over deflated and active eigenvalues
    std::vector<int> ord(m);
    std::iota(ord.begin(), ord.end(), 0);
    std::vector<int> defl;                 // deflated indices in increasing order
    for (int j = 0; j < m; ++j)
        if (pos[j] < 0) defl.push_back(j);
    // candidate c < k: active eigenpair c; c >= k: deflated index defl[c - k]
    auto value = [&](int c) { return c < k ? aval[c] : dval[defl[c - k]]; };
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return value(a) < value(b); });
    // host staging: src [m], pos [m] as ints, values [m] as doubles
    int* hsrc = (int*)(host + Mm + 8);
    int* hpos = hsrc + m;
    double* hval = host + 2 * Mm + 8;
    for (int c = 0; c < m; ++c) {
        const int o = ord[c];
        hsrc[c] = o < k ? o : -(defl[o - k] + 1);
        hval[c] = value(o);
    }
    std::memcpy(hpos, pos.data(), sizeof(int) * m);
    int* dsrc = iw + Mm;                   // src [m] then pos [m], one copy
    int* dpos = dsrc + m;
    double* dval_d = colmax;               // reused: [m] values in output order
    rc = (int)hipMemcpyAsync(dsrc, hsrc, sizeof(int) * 2 * m, hipMemcpyHostToDevice, s);
    if (rc == 0) rc = (int)hipMemcpyAsync(dval_d, hval, sizeof(double) * m, hipMemcpyHostToDevice, s);
    if (rc != 0) return rc;
    const int Mk = eig_padded_order(std::max(k, 1));
    hipLaunchKernelGGL(k_eig_expand, dim3(grid_for((size_t)m * m)), dim3(256), 0, s, m, Mk, (const zd*)Wp,
                       (const int*)dsrc, (const int*)dpos, (const double*)dval_d, G, ldg, theta);
    rc = (int)hipGetLastError();
    if (rc == 0) rc = (int)hipStreamSynchronize(s);   // the host staging must outlive the copies
    return rc;
}
