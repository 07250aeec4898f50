// Per-vector filter-degree network: 5 -> 64 -> 64 -> 64 -> 1, ReLU hidden layers,
// d = dmin + (dmax - dmin) sigmoid(z).  FP32 forward, hand-written backward (mean squared error
// against a degree label) and Adam.  Parameter layout (row-major W[out][in]):
//   W1[64][5] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[1][64] b4[1]  (8769 floats)
//
// The paper uses one fixed degree for every vector (Section 3.1, Table 3); the network replaces
// it with a per-vector prediction learned from the solver's own traces.
#include "common.h"
#include "driver.h"

#include <cmath>
#include <functional>
#include <vector>

namespace {

constexpr int NF = MLP_NF, NH = MLP_NH;
constexpr int OW1 = 0, OB1 = OW1 + NH * NF, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH * NH, OW4 = OB3 + NH, OB4 = OW4 + NH, NP = OB4 + 1;
static_assert(NP == MLP_NPARAM, "parameter count");

__device__ inline float sigmoidf_(float z) { return 1.0f / (1.0f + __expf(-z)); }

// One thread per sample; weights staged in LDS (35 KB).  Optionally stores the pre-activations
// (for the backward pass) and the output-layer delta of the squared-error loss.
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ P, int N, const float* __restrict__ X,
                                                     float dmin, float dmax, float* __restrict__ out,
                                                     float* __restrict__ Z, const float* __restrict__ y,
                                                     float* __restrict__ delta4, float* __restrict__ sqerr)
{
    __shared__ float w[NP];
    for (int i = threadIdx.x; i < NP; i += blockDim.x) w[i] = P[i];
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= N) return;
    float x[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) x[i] = X[(size_t)b * NF + i];
    float h[NH], g[NH];
#pragma unroll
    for (int o = 0; o < NH; ++o) {
        float s = w[OB1 + o];
#pragma unroll
        for (int i = 0; i < NF; ++i) s += w[OW1 + o * NF + i] * x[i];
        if (Z) Z[(size_t)b * 3 * NH + o] = s;
        h[o] = s > 0.f ? s : 0.f;
    }
#pragma unroll
    for (int o = 0; o < NH; ++o) {
        float s = w[OB2 + o];
#pragma unroll
        for (int i = 0; i < NH; ++i) s += w[OW2 + o * NH + i] * h[i];
        if (Z) Z[(size_t)b * 3 * NH + NH + o] = s;
        g[o] = s > 0.f ? s : 0.f;
    }
#pragma unroll
    for (int o = 0; o < NH; ++o) {
        float s = w[OB3 + o];
#pragma unroll
        for (int i = 0; i < NH; ++i) s += w[OW3 + o * NH + i] * g[i];
        if (Z) Z[(size_t)b * 3 * NH + 2 * NH + o] = s;
        h[o] = s > 0.f ? s : 0.f;
    }
    float z4 = w[OB4];
#pragma unroll
    for (int i = 0; i < NH; ++i) z4 += w[OW4 + i] * h[i];
    const float sg = sigmoidf_(z4);
    const float d = dmin + (dmax - dmin) * sg;
    if (out) out[b] = d;
    if (y) {
        const float err = d - y[b];
        delta4[b] = (2.0f * err / (float)N) * (dmax - dmin) * sg * (1.0f - sg);
        sqerr[b] = err * err;
    }
}

// delta of hidden layer l (0-based: 0..2) from the layer above.
//  l == 2: delta3[b][o] = relu'(z3) W4[o] delta4[b]
//  l <  2: delta_l[b][i] = relu'(z_l) sum_o W_{l+2}[o][i] delta_{l+1}[b][o]
__global__ void k_mlp_delta(const float* __restrict__ P, int N, const float* __restrict__ Z,
                            const float* __restrict__ delta4, float* __restrict__ D, int l)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N * NH) return;
    const int b = e / NH, i = e % NH;
    const float z = Z[(size_t)b * 3 * NH + l * NH + i];
    float v = 0.f;
    if (z > 0.f) {
        if (l == 2) {
            v = P[OW4 + i] * delta4[b];
        } else {
            const int ow = (l == 1) ? OW3 : OW2;
            const float* dn = D + (size_t)b * 3 * NH + (l + 1) * NH;
            for (int o = 0; o < NH; ++o) v += P[ow + o * NH + i] * dn[o];
        }
    }
    D[(size_t)b * 3 * NH + l * NH + i] = v;
}

// weight/bias gradients of layer L (1..4): gW[o][i] = sum_b delta_L[b][o] in_L[b][i], gb[o] = sum_b delta_L[b][o]
__global__ void k_mlp_wgrad(int N, const float* __restrict__ X, const float* __restrict__ Z,
                            const float* __restrict__ D, const float* __restrict__ delta4, float* __restrict__ grad,
                            int L)
{
    const int nin = (L == 1) ? NF : NH, nout = (L == 4) ? 1 : NH;
    const int ow = L == 1 ? OW1 : L == 2 ? OW2 : L == 3 ? OW3 : OW4;
    const int ob = L == 1 ? OB1 : L == 2 ? OB2 : L == 3 ? OB3 : OB4;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = nout * nin;
    if (e >= nw + nout) return;
    const bool bias = e >= nw;
    const int o = bias ? e - nw : e / nin, i = bias ? 0 : e % nin;
    float s = 0.f;
    for (int b = 0; b < N; ++b) {
        const float d = (L == 4) ? delta4[b] : D[(size_t)b * 3 * NH + (L - 1) * NH + o];
        if (bias) { s += d; continue; }
        float in;
        if (L == 1) in = X[(size_t)b * NF + i];
        else {
            const float z = Z[(size_t)b * 3 * NH + (L - 2) * NH + i];
            in = z > 0.f ? z : 0.f;
        }
        s += d * in;
    }
    grad[bias ? ob + o : ow + o * nin + i] = s;
}

__global__ void k_sum(int N, const float* __restrict__ v, float* __restrict__ out)
{
    __shared__ float sm[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < N; i += 256) s += v[i];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sm[0] / (float)N;
}

__global__ void k_adam(int np, float* __restrict__ P, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_gather_rows5(int nb, const float* __restrict__ X, const float* __restrict__ y,
                               const int* __restrict__ idx, float* __restrict__ Xb, float* __restrict__ yb)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int s = idx[b];
#pragma unroll
    for (int i = 0; i < NF; ++i) Xb[(size_t)b * NF + i] = X[(size_t)s * NF + i];
    yb[b] = y[s];
}

// features of active column j for the next filter: t = (theta - c)/e, log10(r/thr), position of a
// in [mu1, b], relative width of [mu1, b], previous degree; then (f - mean) / std
__global__ void k_degree_features(int m, const double* __restrict__ theta, const double* __restrict__ r, double a,
                                  double b, double mu1, double thr, const int* __restrict__ dprev,
                                  const float* __restrict__ norm, float* __restrict__ feat)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const double c = 0.5 * (a + b), e = 0.5 * (b - a);
    double f[NF];
    f[0] = (theta[j] - c) / e;
    f[1] = log10(fmax(r[j], 1e-300) / thr);
    f[2] = (a - mu1) / (b - mu1);
    f[3] = (b - mu1) / (fabs(mu1) + fabs(b));
    f[4] = (double)dprev[j];
#pragma unroll
    for (int i = 0; i < NF; ++i) feat[(size_t)j * NF + i] = (float)((f[i] - (double)norm[i]) / (double)norm[NF + i]);
}

}  // namespace

size_t mlp_scratch_floats(int N) { return (size_t)N * (6 * NH + 4) + 64; }

int launch_mlp_forward(hipStream_t s, const float* P, int N, const float* X, float dmin, float dmax, float* out)
{
    if (N <= 0) return 0;
    hipLaunchKernelGGL(k_mlp_forward, dim3((N + 255) / 256), dim3(256), 0, s, P, N, X, dmin, dmax, out, nullptr,
                       nullptr, nullptr, nullptr);
    return (int)hipGetLastError();
}

// scratch: Z [N][3][64], D [N][3][64], delta4 [N], sqerr [N]
int launch_mlp_loss_grad(hipStream_t s, const float* P, int N, const float* X, const float* y, float dmin, float dmax,
                         float* grad, float* loss_dev, float* scratch)
{
    if (N <= 0) return 0;
    float* Z = scratch;
    float* D = Z + (size_t)N * 3 * NH;
    float* d4 = D + (size_t)N * 3 * NH;
    float* se = d4 + N;
    hipLaunchKernelGGL(k_mlp_forward, dim3((N + 255) / 256), dim3(256), 0, s, P, N, X, dmin, dmax, nullptr, Z, y, d4,
                       se);
    for (int l = 2; l >= 0; --l)
        hipLaunchKernelGGL(k_mlp_delta, dim3((N * NH + 255) / 256), dim3(256), 0, s, P, N, Z, d4, D, l);
    for (int L = 1; L <= 4; ++L) {
        const int nin = (L == 1) ? NF : NH, nout = (L == 4) ? 1 : NH;
        const int cnt = nout * nin + nout;
        hipLaunchKernelGGL(k_mlp_wgrad, dim3((cnt + 255) / 256), dim3(256), 0, s, N, X, Z, D, d4, grad, L);
    }
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, N, se, loss_dev);
    // k_sum divides by N: mean squared error
    return (int)hipGetLastError();
}

int launch_mlp_adam(hipStream_t s, int np, float* P, const float* g, float* m, float* v, int t, float lr, float b1,
                    float b2, float eps)
{
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, s, np, P, g, m, v, lr, b1, b2, eps, c1, c2);
    return (int)hipGetLastError();
}

int launch_gather_rows5(hipStream_t s, int nb, const float* X, const float* y, const int* idx, float* Xb, float* yb)
{
    if (nb <= 0) return 0;
    hipLaunchKernelGGL(k_gather_rows5, dim3((nb + 255) / 256), dim3(256), 0, s, nb, X, y, idx, Xb, yb);
    return (int)hipGetLastError();
}

int launch_degree_features_ext(hipStream_t s, int m, const double* theta, const double* r, double a, double b,
                               double mu1, double thr, const int* dprev, const float* norm, float* feat)
{
    if (m <= 0) return 0;
    hipLaunchKernelGGL(k_degree_features, dim3((m + 255) / 256), dim3(256), 0, s, m, theta, r, a, b, mu1, thr, dprev,
                       norm, feat);
    return (int)hipGetLastError();
}

// Predicted degree per active column; non-finite or out-of-range predictions fall back to
// `fallback(j)` (the analytic degree).
chfsi_status learned_degrees(chfsi_handle h, int ma, const double* theta_dev, const double* r_dev, double a,
                             double b, double mu1, double thr, const std::vector<int>& dprev, float* feat,
                             float* dpred, int* iscr, int dmin, int dmax, int* out,
                             const std::function<int(int)>& fallback)
{
    if (ma <= 0) return CHFSI_SUCCESS;
    hipStream_t st = h->stream;
    if (hipMemcpyAsync(iscr, dprev.data(), sizeof(int) * ma, hipMemcpyHostToDevice, st) != hipSuccess)
        return CHFSI_ERR_DEVICE;
    if (launch_degree_features_ext(st, ma, theta_dev, r_dev, a, b, mu1, thr, iscr, h->model + MLP_NPARAM, feat))
        return CHFSI_ERR_DEVICE;
    if (launch_mlp_forward(st, h->model, ma, feat, (float)dmin, (float)dmax, dpred)) return CHFSI_ERR_DEVICE;
    std::vector<float> hp(ma);
    if (hipMemcpyAsync(hp.data(), dpred, sizeof(float) * ma, hipMemcpyDeviceToHost, st) != hipSuccess)
        return CHFSI_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return CHFSI_ERR_DEVICE;
    for (int j = 0; j < ma; ++j) {
        const float v = hp[j];
        if (!std::isfinite(v) || v < (float)dmin - 0.5f || v > (float)dmax + 0.5f) out[j] = fallback(j);
        else out[j] = std::min(dmax, std::max(dmin, (int)std::lround(v)));
    }
    return CHFSI_SUCCESS;
}

// ---------------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------------

namespace {
// host-side Philox4x64-10 for the minibatch shuffle
void philox_host(uint64_t c[4], uint64_t k0, uint64_t k1)
{
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
}

chfsi_status ensure_ws(chfsi_handle h, size_t bytes)
{
    if (bytes > h->ws.cap) {
        (void)hipStreamSynchronize(h->stream);
        h->ws.grow(bytes);
        if (h->ws.cap < bytes) return CHFSI_ERR_ALLOC;
    }
    h->ws.begin(false);
    return CHFSI_SUCCESS;
}
}  // namespace

extern "C" {

chfsi_status chfsi_set_degree_model(chfsi_handle h, const void* blob, size_t nbytes)
{
    if (!h) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    if (!blob) { h->has_model = false; return CHFSI_SUCCESS; }
    const size_t need = sizeof(float) * (MLP_NPARAM + 2 * MLP_NF);
    if (nbytes != need) return CHFSI_ERR_ARG;
    const float* f = (const float*)blob;
    for (size_t i = 0; i < need / sizeof(float); ++i)
        if (!std::isfinite(f[i])) return CHFSI_ERR_ARG;
    for (int i = 0; i < MLP_NF; ++i)
        if (!(f[MLP_NPARAM + MLP_NF + i] > 0)) return CHFSI_ERR_ARG;
    if (!h->model && hipMalloc((void**)&h->model, need) != hipSuccess) { h->model = nullptr; return CHFSI_ERR_ALLOC; }
    if (hipMemcpyAsync(h->model, blob, need, hipMemcpyHostToDevice, h->stream) != hipSuccess) return CHFSI_ERR_DEVICE;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return CHFSI_ERR_DEVICE;
    h->has_model = true;
    return CHFSI_SUCCESS;
}

chfsi_status chfsi_mlp_forward(chfsi_handle h, const float* P, int N, const float* X, float dmin, float dmax, float* out)
{
    if (!h || !P || !X || !out || N < 0 || !(dmax > dmin)) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    if (launch_mlp_forward(h->stream, P, N, X, dmin, dmax, out)) return CHFSI_ERR_DEVICE;
    return hipStreamSynchronize(h->stream) == hipSuccess ? CHFSI_SUCCESS : CHFSI_ERR_DEVICE;
}

chfsi_status chfsi_mlp_loss_grad(chfsi_handle h, const float* P, int N, const float* X, const float* y, float dmin,
                                 float dmax, float* grad, float* loss)
{
    if (!h || !P || !X || !y || !grad || !loss || N <= 0 || !(dmax > dmin)) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    const size_t nf = mlp_scratch_floats(N) + 64;
    if (ensure_ws(h, nf * sizeof(float)) != CHFSI_SUCCESS) return CHFSI_ERR_ALLOC;
    float* scr = h->ws.take<float>(nf);
    float* ld = scr + mlp_scratch_floats(N);
    if (launch_mlp_loss_grad(h->stream, P, N, X, y, dmin, dmax, grad, ld, scr)) return CHFSI_ERR_DEVICE;
    if (hipMemcpyAsync(loss, ld, sizeof(float), hipMemcpyDeviceToHost, h->stream) != hipSuccess) return CHFSI_ERR_DEVICE;
    return hipStreamSynchronize(h->stream) == hipSuccess ? CHFSI_SUCCESS : CHFSI_ERR_DEVICE;
}

chfsi_status chfsi_mlp_adam(chfsi_handle h, float* P, const float* grad, float* m, float* v, int t, float lr,
                            float beta1, float beta2, float eps)
{
    if (!h || !P || !grad || !m || !v || t < 1) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    if (launch_mlp_adam(h->stream, MLP_NPARAM, P, grad, m, v, t, lr, beta1, beta2, eps)) return CHFSI_ERR_DEVICE;
    return hipStreamSynchronize(h->stream) == hipSuccess ? CHFSI_SUCCESS : CHFSI_ERR_DEVICE;
}

chfsi_status chfsi_mlp_train(chfsi_handle h, float* P, int N, const float* X, const float* y, float dmin, float dmax,
                             int epochs, int batch, float lr, unsigned long long seed, float* loss_hist)
{
    if (!h || !P || !X || !y || N <= 0 || epochs < 0 || batch <= 0 || !(dmax > dmin) || !(lr > 0)) return CHFSI_ERR_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return CHFSI_ERR_DEVICE;
    hipStream_t st = h->stream;
    const int B = std::min(batch, N);
    const size_t nscr = mlp_scratch_floats(B);
    const size_t floats = nscr + (size_t)B * (NF + 1) + 3 * (size_t)MLP_NPARAM + 64;
    if (ensure_ws(h, floats * sizeof(float) + (size_t)N * sizeof(int) + 1024) != CHFSI_SUCCESS) return CHFSI_ERR_ALLOC;
    float* scr = h->ws.take<float>(nscr);
    float* Xb = h->ws.take<float>((size_t)B * NF);
    float* yb = h->ws.take<float>(B);
    float* g = h->ws.take<float>(MLP_NPARAM);
    float* mom = h->ws.take<float>(MLP_NPARAM);
    float* vel = h->ws.take<float>(MLP_NPARAM);
    float* ld = h->ws.take<float>(64);
    int* idx = h->ws.take<int>(N);
    if (hipMemsetAsync(mom, 0, sizeof(float) * MLP_NPARAM, st) != hipSuccess) return CHFSI_ERR_DEVICE;
    if (hipMemsetAsync(vel, 0, sizeof(float) * MLP_NPARAM, st) != hipSuccess) return CHFSI_ERR_DEVICE;
    std::vector<int> perm(N);
    int t = 0;
    const int nbatches = N / B;
    std::vector<float> losses(std::max(nbatches, 1));
    for (int ep = 0; ep < epochs; ++ep) {
        for (int i = 0; i < N; ++i) perm[i] = i;
        for (int i = N - 1; i > 0; --i) {   // Fisher-Yates with Philox words
            uint64_t c[4] = {(uint64_t)i, (uint64_t)ep, 7, 0};
            philox_host(c, seed, 1);
            const int j = (int)(c[0] % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        if (hipMemcpyAsync(idx, perm.data(), sizeof(int) * N, hipMemcpyHostToDevice, st) != hipSuccess)
            return CHFSI_ERR_DEVICE;
        for (int bi = 0; bi < nbatches; ++bi) {
            if (launch_gather_rows5(st, B, X, y, idx + (size_t)bi * B, Xb, yb)) return CHFSI_ERR_DEVICE;
            if (launch_mlp_loss_grad(st, P, B, Xb, yb, dmin, dmax, g, ld + (bi % 32), scr)) return CHFSI_ERR_DEVICE;
            if (launch_mlp_adam(st, MLP_NPARAM, P, g, mom, vel, ++t, lr, 0.9f, 0.999f, 1e-8f)) return CHFSI_ERR_DEVICE;
            if (bi % 32 == 31 || bi == nbatches - 1) {
                const int cnt = bi % 32 + 1;
                if (hipMemcpyAsync(losses.data() + (bi - cnt + 1), ld, sizeof(float) * cnt, hipMemcpyDeviceToHost,
                                   st) != hipSuccess)
                    return CHFSI_ERR_DEVICE;
                if (hipStreamSynchronize(st) != hipSuccess) return CHFSI_ERR_DEVICE;
            }
        }
        if (loss_hist) {
            double s = 0;
            for (int bi = 0; bi < nbatches; ++bi) s += losses[bi];
            loss_hist[ep] = (float)(s / std::max(nbatches, 1));
        }
    }
    return hipStreamSynchronize(st) == hipSuccess ? CHFSI_SUCCESS : CHFSI_ERR_DEVICE;
}

}  // extern "C"
