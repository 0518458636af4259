/*
 * CPU oracle for the learned heuristic (a project addition beside the paper's
 * method): k-nearest-neighbour edge features, a 8 -> 128 -> 128 -> 1 GELU
 * edge-scoring MLP (forward, backward of binary cross-entropy with logits,
 * Adam), and the installation of eta = (1/d) * 2 sigmoid(s) on the kNN edges
 * (eta = 1/d elsewhere, the paper's heuristic of Sec. 2.1).
 *
 * TEST INFRASTRUCTURE ONLY; the product never loads it.
 *
 * The MLP runs in float64 with libm's erf for GELU(z) = z (1 + erf(z/sqrt2))/2.
 * With `quantize` set it rounds, where the GPU keeps bfloat16 values, to the
 * nearest bfloat16 (ties to even): the inputs, the weights, the activations
 * H1 and H2 and the back-propagated dZ1 and dZ2; everything else stays in
 * float64. With `quantize` clear it is the plain float64 network (used for the
 * finite-difference check of the backward pass).
 */
#include "mmas_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define H 128 /* hidden width */
#define IN 16 /* input width: 8 features padded to 16 */

static float f32_bits(uint32_t b) {
    float f;
    memcpy(&f, &b, 4);
    return f;
}
static uint32_t bits_f32(float f) {
    uint32_t b;
    memcpy(&b, &f, 4);
    return b;
}

float orc_bf16_round(float x) {
    uint32_t b = bits_f32(x);
    b = b + 0x7FFFu + ((b >> 16) & 1u);
    return f32_bits(b & 0xFFFF0000u);
}

static double q(double x, int quantize) { return quantize ? (double)orc_bf16_round((float)x) : x; }

/* ---- features --------------------------------------------------------- */

/* Per directed edge i -> j, j the r-th of the 16 nearest cities of i (by
 * (distance, index)), in FP32 with this order of operations:
 *   dbar_i = (sum over r of d(i, knn[i][r]), accumulated left to right) / 16
 *   f0 = d_ij / dbar_i            f1 = r / 15
 *   f2 = (rank of i among the 16 nearest of j, or 16) / 16
 *   f3 = (x_j - x_i) / dbar_i     f4 = (y_j - y_i) / dbar_i
 *   f5 = indeg(j) / 16            f6 = indeg(i) / 16
 *   f7 = dbar_j / dbar_i
 * where indeg(v) counts the cities that have v among their 16 nearest.
 * knn: n*16; feat: (n*16)*8 row-major by edge e = 16 i + r. */
void orc_knn_features(int n, const int32_t* dist, const float* xy, uint16_t* knn, float* feat) {
    const int K = 16;
    orc_nearest(n, dist, K, knn);
    float* dbar = (float*)malloc(sizeof(float) * (size_t)n);
    int* indeg = (int*)calloc((size_t)n, sizeof(int));
    for (int i = 0; i < n; ++i) {
        float s = 0.0f;
        for (int r = 0; r < K; ++r) s = s + (float)dist[(size_t)i * n + knn[i * K + r]];
        dbar[i] = s / 16.0f;
        for (int r = 0; r < K; ++r) indeg[knn[i * K + r]] += 1;
    }
    for (int i = 0; i < n; ++i) {
        for (int r = 0; r < K; ++r) {
            const int j = knn[i * K + r];
            int back = 16;
            for (int t = 0; t < K; ++t)
                if (knn[j * K + t] == i) {
                    back = t;
                    break;
                }
            float* f = feat + ((size_t)i * K + r) * 8;
            f[0] = (float)dist[(size_t)i * n + j] / dbar[i];
            f[1] = (float)r / 15.0f;
            f[2] = (float)back / 16.0f;
            f[3] = (xy[2 * j] - xy[2 * i]) / dbar[i];
            f[4] = (xy[2 * j + 1] - xy[2 * i + 1]) / dbar[i];
            f[5] = (float)indeg[j] / 16.0f;
            f[6] = (float)indeg[i] / 16.0f;
            f[7] = dbar[j] / dbar[i];
        }
    }
    free(dbar);
    free(indeg);
}

/* ---- MLP ---------------------------------------------------------------- */

static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }
static double gelu_d(double z) {
    const double Phi = 0.5 * (1.0 + erf(z / sqrt(2.0)));
    const double phi = exp(-0.5 * z * z) / sqrt(2.0 * M_PI);
    return Phi + z * phi;
}
static double sigmoid(double s) { return 1.0 / (1.0 + exp(-s)); }

/* Parameters: W1 IN x H (row k = input k), b1 H, W2 H x H (row = input),
 * b2 H, w3 H, b3 1. X: E x IN. */
void orc_mlp_forward(int64_t E, const float* X, const float* W1, const float* b1, const float* W2, const float* b2,
                     const float* w3, float b3, int quantize, float* s_out) {
    double* h1 = (double*)malloc(sizeof(double) * H);
    double* h2 = (double*)malloc(sizeof(double) * H);
    for (int64_t e = 0; e < E; ++e) {
        const float* x = X + e * IN;
        for (int c = 0; c < H; ++c) {
            double z = 0.0;
            for (int k = 0; k < IN; ++k) z += q(x[k], quantize) * q(W1[k * H + c], quantize);
            z += b1[c];
            h1[c] = q(gelu(z), quantize);
        }
        for (int c = 0; c < H; ++c) {
            double z = 0.0;
            for (int k = 0; k < H; ++k) z += h1[k] * q(W2[k * H + c], quantize);
            z += b2[c];
            h2[c] = q(gelu(z), quantize);
        }
        double s = 0.0;
        for (int k = 0; k < H; ++k) s += h2[k] * q(w3[k], quantize);
        s_out[e] = (float)(s + b3);
    }
    free(h1);
    free(h2);
}

/* Loss = mean over edges of softplus(s) - f s (binary cross-entropy with
 * logits against the target frequency f in [0,1]); gradients of it. Returns
 * the loss. Gradient arrays have the parameters' shapes. */
double orc_mlp_backward(int64_t E, const float* X, const float* f, const float* W1, const float* b1, const float* W2,
                        const float* b2, const float* w3, float b3, int quantize, float* gW1, float* gb1, float* gW2,
                        float* gb2, float* gw3, float* gb3) {
    double* z1 = (double*)malloc(sizeof(double) * H);
    double* h1 = (double*)malloc(sizeof(double) * H);
    double* z2 = (double*)malloc(sizeof(double) * H);
    double* h2 = (double*)malloc(sizeof(double) * H);
    double* dz2 = (double*)malloc(sizeof(double) * H);
    double* dz1 = (double*)malloc(sizeof(double) * H);
    double* GW1 = (double*)calloc(IN * H, sizeof(double));
    double* GB1 = (double*)calloc(H, sizeof(double));
    double* GW2 = (double*)calloc(H * H, sizeof(double));
    double* GB2 = (double*)calloc(H, sizeof(double));
    double* GW3 = (double*)calloc(H, sizeof(double));
    double GB3 = 0.0, loss = 0.0;
    for (int64_t e = 0; e < E; ++e) {
        const float* x = X + e * IN;
        for (int c = 0; c < H; ++c) {
            double z = 0.0;
            for (int k = 0; k < IN; ++k) z += q(x[k], quantize) * q(W1[k * H + c], quantize);
            z1[c] = z + b1[c];
            h1[c] = q(gelu(z1[c]), quantize);
        }
        for (int c = 0; c < H; ++c) {
            double z = 0.0;
            for (int k = 0; k < H; ++k) z += h1[k] * q(W2[k * H + c], quantize);
            z2[c] = z + b2[c];
            h2[c] = q(gelu(z2[c]), quantize);
        }
        double s = b3;
        for (int k = 0; k < H; ++k) s += h2[k] * q(w3[k], quantize);
        /* softplus(s) - f s, computed stably */
        loss += (s > 0 ? s + log1p(exp(-s)) : log1p(exp(s))) - (double)f[e] * s;
        const double g = (sigmoid(s) - (double)f[e]) / (double)E;
        GB3 += g;
        for (int k = 0; k < H; ++k) {
            GW3[k] += h2[k] * g;
            dz2[k] = q(g * q(w3[k], quantize) * gelu_d(z2[k]), quantize);
            GB2[k] += dz2[k];
        }
        for (int k = 0; k < H; ++k)
            for (int c = 0; c < H; ++c) GW2[k * H + c] += h1[k] * dz2[c];
        for (int k = 0; k < H; ++k) {
            double dh = 0.0;
            for (int c = 0; c < H; ++c) dh += dz2[c] * q(W2[k * H + c], quantize);
            dz1[k] = q(dh * gelu_d(z1[k]), quantize);
            GB1[k] += dz1[k];
        }
        for (int k = 0; k < IN; ++k)
            for (int c = 0; c < H; ++c) GW1[k * H + c] += q(x[k], quantize) * dz1[c];
    }
    for (int i = 0; i < IN * H; ++i) gW1[i] = (float)GW1[i];
    for (int i = 0; i < H * H; ++i) gW2[i] = (float)GW2[i];
    for (int i = 0; i < H; ++i) {
        gb1[i] = (float)GB1[i];
        gb2[i] = (float)GB2[i];
        gw3[i] = (float)GW3[i];
    }
    *gb3 = (float)GB3;
    free(z1);
    free(h1);
    free(z2);
    free(h2);
    free(dz2);
    free(dz1);
    free(GW1);
    free(GB1);
    free(GW2);
    free(GB2);
    free(GW3);
    return loss / (double)E;
}

/* Adam (Kingma and Ba) in FP32, one step t >= 1:
 *   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g g
 *   p = p - lr (m / c1) / (sqrt(v / c2) + eps),  c1 = 1 - b1^t, c2 = 1 - b2^t
 * with c1, c2 given (computed in FP64 by the caller and rounded). */
void orc_adam(int64_t count, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
              float c1, float c2) {
    const float o1 = 1.0f - b1, o2 = 1.0f - b2;
    for (int64_t i = 0; i < count; ++i) {
        m[i] = b1 * m[i] + o1 * g[i];
        v[i] = b2 * v[i] + o2 * (g[i] * g[i]);
        p[i] = p[i] - lr * (m[i] / c1) / (sqrtf(v[i] / c2) + eps);
    }
}

/* ---- install ------------------------------------------------------------ */

/* exp in FP32 for the sigmoid of the install: x is clamped to [-104, 89]
 * (exp underflows to 0 or overflows beyond), k = nearest integer to
 * x log2(e), r = x - k ln2 (ln2 in a 15-bit head and a tail, so k * head is
 * exact), exp(r) from its Taylor series through r^8 (|r| <= ln2/2) by
 * Horner, then scaled by 2^k. */
float orc_expf(float x) {
    const float LOG2E = f32_bits(0x3FB8AA3Bu);
    const float LN2_HI = f32_bits(0x3F317200u); /* 0.693145751953125 */
    const float LN2_LO = f32_bits(0x35BFBE8Eu); /* ln2 - LN2_HI, nearest FP32 */
    if (x > 89.0f) x = 89.0f;
    if (x < -104.0f) x = -104.0f;
    const float kf = rintf(x * LOG2E);
    const float r = (x - kf * LN2_HI) - kf * LN2_LO;
    float p = 1.0f / 40320.0f;
    p = 1.0f / 5040.0f + r * p;
    p = 1.0f / 720.0f + r * p;
    p = 1.0f / 120.0f + r * p;
    p = 1.0f / 24.0f + r * p;
    p = 1.0f / 6.0f + r * p;
    p = 0.5f + r * p;
    p = 1.0f + r * p;
    p = 1.0f + r * p;
    return ldexpf(p, (int)kf);
}

/* eta_ij = fl(fl(1/d_ij) * fl(2 * sigma(s_ij))) on the 16 nearest of i;
 * every other edge of i takes the multiplier of i's lowest-scored edge,
 * fl(2 * sigma(min_r s_ir)) (an unscored edge counts as no better than the
 * worst scored one); sigma(s) = 1 / (1 + orc_expf(-s)); heur = eta^beta
 * (left-to-right products); heur_ii = 0. s: n*16 by edge 16 i + r. With
 * all scores 0 every multiplier is 1 and heur is the plain eta^beta. */
void orc_install_eta(int n, const int32_t* dist, const uint16_t* knn, const float* s, int beta, float* heur) {
    for (int i = 0; i < n; ++i) {
        float smin = s[i * 16];
        for (int r = 1; r < 16; ++r)
            if (s[i * 16 + r] < smin) smin = s[i * 16 + r];
        for (int j = 0; j < n; ++j) {
            float h = 0.0f;
            if (i != j) {
                const float eta = 1.0f / (float)dist[(size_t)i * n + j];
                float sc = smin;
                for (int r = 0; r < 16; ++r)
                    if (knn[i * 16 + r] == j) {
                        sc = s[i * 16 + r];
                        break;
                    }
                const float sg = 1.0f / (1.0f + orc_expf(-sc));
                const float x = eta * (2.0f * sg);
                h = 1.0f;
                for (int b = 0; b < beta; ++b) h = h * x;
            }
            heur[(size_t)i * n + j] = h;
        }
    }
}
