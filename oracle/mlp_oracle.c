/*
 * FP64 reference for the per-vector filter-degree network.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline); the product never calls it.
 *
 * The paper fixes one filter degree for all vectors (Section 3.1: the degree does not matter much
 * as long as it is high enough; Table 3 uses 25).  The learned policy predicts a degree per vector
 * from five features with a fully connected network 5 -> 64 -> 64 -> 64 -> 1, ReLU on the hidden
 * layers and d = dmin + (dmax - dmin) * sigmoid(z) on the output, trained with the mean squared
 * error against a degree label and Adam (Kingma & Ba 2015).
 *
 * Parameter vector layout (row-major weights W[out][in]):
 *   W1[64][5] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[1][64] b4[1]   -> 8769 values.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NF 5
#define NH 64
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NH * NF)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NH * NH)
#define OFF_W4 (OFF_B3 + NH)
#define OFF_B4 (OFF_W4 + NH)
#define NPARAM (OFF_B4 + 1)

int orc_mlp_nparams(void) { return NPARAM; }

static double sigm(double z) { return 1.0 / (1.0 + exp(-z)); }

/* dense layer: out[o] = b[o] + sum_i W[o][i] in[i] */
static void dense(const double* W, const double* b, int nin, int nout, const double* in, double* out)
{
    for (int o = 0; o < nout; ++o) {
        double s = b[o];
        for (int i = 0; i < nin; ++i) s += W[o * nin + i] * in[i];
        out[o] = s;
    }
}

/* Forward pass of one sample; keeps pre-activations for the backward pass. */
static double forward1(const double* P, const double* x, double dmin, double dmax,
                       double* z1, double* h1, double* z2, double* h2, double* z3, double* h3, double* z4)
{
    dense(P + OFF_W1, P + OFF_B1, NF, NH, x, z1);
    for (int i = 0; i < NH; ++i) h1[i] = z1[i] > 0 ? z1[i] : 0;
    dense(P + OFF_W2, P + OFF_B2, NH, NH, h1, z2);
    for (int i = 0; i < NH; ++i) h2[i] = z2[i] > 0 ? z2[i] : 0;
    dense(P + OFF_W3, P + OFF_B3, NH, NH, h2, z3);
    for (int i = 0; i < NH; ++i) h3[i] = z3[i] > 0 ? z3[i] : 0;
    dense(P + OFF_W4, P + OFF_B4, NH, 1, h3, z4);
    return dmin + (dmax - dmin) * sigm(z4[0]);
}

void orc_mlp_forward(const double* P, int N, const double* X, double dmin, double dmax, double* out)
{
    double z1[NH], h1[NH], z2[NH], h2[NH], z3[NH], h3[NH], z4[1];
    for (int k = 0; k < N; ++k) out[k] = forward1(P, X + (size_t)k * NF, dmin, dmax, z1, h1, z2, h2, z3, h3, z4);
}

/* Loss L = (1/N) sum_k (d_k - y_k)^2 and its gradient with respect to every parameter. */
double orc_mlp_loss_grad(const double* P, int N, const double* X, const double* y, double dmin,
                         double dmax, double* grad)
{
    memset(grad, 0, sizeof(double) * NPARAM);
    double z1[NH], h1[NH], z2[NH], h2[NH], z3[NH], h3[NH], z4[1];
    double d1[NH], d2[NH], d3[NH];
    double loss = 0;
    for (int k = 0; k < N; ++k) {
        const double* x = X + (size_t)k * NF;
        double d = forward1(P, x, dmin, dmax, z1, h1, z2, h2, z3, h3, z4);
        double err = d - y[k];
        loss += err * err;
        double s = sigm(z4[0]);
        double delta4 = (2.0 * err / N) * (dmax - dmin) * s * (1.0 - s);
        for (int i = 0; i < NH; ++i) grad[OFF_W4 + i] += delta4 * h3[i];
        grad[OFF_B4] += delta4;
        for (int i = 0; i < NH; ++i) d3[i] = z3[i] > 0 ? P[OFF_W4 + i] * delta4 : 0;
        for (int o = 0; o < NH; ++o) {
            for (int i = 0; i < NH; ++i) grad[OFF_W3 + o * NH + i] += d3[o] * h2[i];
            grad[OFF_B3 + o] += d3[o];
        }
        for (int i = 0; i < NH; ++i) {
            double s2 = 0;
            for (int o = 0; o < NH; ++o) s2 += P[OFF_W3 + o * NH + i] * d3[o];
            d2[i] = z2[i] > 0 ? s2 : 0;
        }
        for (int o = 0; o < NH; ++o) {
            for (int i = 0; i < NH; ++i) grad[OFF_W2 + o * NH + i] += d2[o] * h1[i];
            grad[OFF_B2 + o] += d2[o];
        }
        for (int i = 0; i < NH; ++i) {
            double s1 = 0;
            for (int o = 0; o < NH; ++o) s1 += P[OFF_W2 + o * NH + i] * d2[o];
            d1[i] = z1[i] > 0 ? s1 : 0;
        }
        for (int o = 0; o < NH; ++o) {
            for (int i = 0; i < NF; ++i) grad[OFF_W1 + o * NF + i] += d1[o] * x[i];
            grad[OFF_B1 + o] += d1[o];
        }
    }
    return loss / N;
}

/* One Adam step (bias-corrected moments), t >= 1. */
void orc_adam_step(int np, double* P, const double* g, double* m, double* v, int t, double lr,
                   double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int i = 0; i < np; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        P[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
