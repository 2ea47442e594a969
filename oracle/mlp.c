/*
 * mlp.c -- oracle: the opacity surrogate network, its mean-squared-error
 * gradient and the Adam update.  Test infrastructure only.
 *
 * Network: x (2) -> tanh(W1 x + b1) (64) -> tanh(W2 h1 + b2) (64)
 *          -> y = W3 h2 + b3 + Ws x (2).
 * Parameters are one flat vector in the order W1 b1 W2 b2 W3 b3 Ws, matrices
 * row-major (output index first).
 *
 * With bf16 = 1 the 64x64 layer is evaluated the way a bfloat16 matrix core
 * sees it: each operand is split into a bfloat16 "hi" part and a bfloat16
 * "lo" remainder and the product keeps hi*hi + hi*lo + lo*hi; every other
 * operation stays in double precision.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "m1_oracle.h"

#define NI 2
#define NH 64
#define NO 2
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NH * NI)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NO * NH)
#define OFF_WS (OFF_B3 + NO)
#define NPARAM (OFF_WS + NO * NI)

int m1o_mlp_nparam(void) { return NPARAM; }

/* Round to bfloat16 (8-bit significand) with round-to-nearest-even, after
 * rounding to binary32. */
double m1o_bf16_round(double x)
{
    float f = (float)x;
    unsigned int u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return x; /* inf / nan untouched */
    unsigned int lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* product a*b of two scalars as split-bfloat16 operands (see header) */
static double split_mul(double a, double b)
{
    double ah = m1o_bf16_round(a), al = m1o_bf16_round(a - ah);
    double bh = m1o_bf16_round(b), bl = m1o_bf16_round(b - bh);
    return ah * bh + ah * bl + al * bh;
}

typedef struct { double z1[NH], h1[NH], z2[NH], h2[NH], y[NO]; } fwd_t;

static void forward_one(const double *th, int bf16, const double *x, fwd_t *s)
{
    const double *W1 = th + OFF_W1, *b1 = th + OFF_B1, *W2 = th + OFF_W2, *b2 = th + OFF_B2;
    const double *W3 = th + OFF_W3, *b3 = th + OFF_B3, *Ws = th + OFF_WS;
    for (int j = 0; j < NH; ++j) {
        s->z1[j] = W1[j * NI] * x[0] + W1[j * NI + 1] * x[1] + b1[j];
        s->h1[j] = tanh(s->z1[j]);
    }
    for (int j = 0; j < NH; ++j) {
        double acc = 0.0;
        for (int k = 0; k < NH; ++k)
            acc += bf16 ? split_mul(W2[j * NH + k], s->h1[k]) : W2[j * NH + k] * s->h1[k];
        s->z2[j] = acc + b2[j];
        s->h2[j] = tanh(s->z2[j]);
    }
    for (int o = 0; o < NO; ++o) {
        double acc = b3[o] + Ws[o * NI] * x[0] + Ws[o * NI + 1] * x[1];
        for (int j = 0; j < NH; ++j) acc += W3[o * NH + j] * s->h2[j];
        s->y[o] = acc;
    }
}

/* y[n][2] = net(x[n][2]) */
void m1o_mlp_forward(const double *theta, int bf16, long n, const double *x, double *y)
{
#pragma omp parallel for schedule(static) if (n > 1024)
    for (long b = 0; b < n; ++b) {
        fwd_t s;
        forward_one(theta, bf16, x + 2 * b, &s);
        y[2 * b] = s.y[0];
        y[2 * b + 1] = s.y[1];
    }
}

/* L = (1/n) sum_b sum_o (y_bo - t_bo)^2 / 2 and its gradient (back-propagation;
 * in bf16 mode the split products of the 64x64 layer are differentiated as
 * if the rounding were the identity, the same points the matrix core sees). */
double m1o_mlp_loss_grad(const double *th, int bf16, long n, const double *x,
                         const double *t, double *grad)
{
    const double *W2 = th + OFF_W2, *W3 = th + OFF_W3;
    memset(grad, 0, NPARAM * sizeof(double));
    double loss = 0.0;
    for (long b = 0; b < n; ++b) {
        fwd_t s;
        const double *xb = x + 2 * b;
        forward_one(th, bf16, xb, &s);
        double dy[NO], dz2[NH], dz1[NH];
        for (int o = 0; o < NO; ++o) {
            double r = s.y[o] - t[2 * b + o];
            loss += 0.5 * r * r / n;
            dy[o] = r / n;
        }
        for (int o = 0; o < NO; ++o) {
            for (int j = 0; j < NH; ++j) grad[OFF_W3 + o * NH + j] += dy[o] * s.h2[j];
            grad[OFF_B3 + o] += dy[o];
            grad[OFF_WS + o * NI] += dy[o] * xb[0];
            grad[OFF_WS + o * NI + 1] += dy[o] * xb[1];
        }
        for (int j = 0; j < NH; ++j) {
            double dh = W3[j] * dy[0] + W3[NH + j] * dy[1];
            dz2[j] = dh * (1.0 - s.h2[j] * s.h2[j]);
            grad[OFF_B2 + j] += dz2[j];
        }
        for (int j = 0; j < NH; ++j)
            for (int k = 0; k < NH; ++k)
                grad[OFF_W2 + j * NH + k] += bf16 ? split_mul(dz2[j], s.h1[k]) : dz2[j] * s.h1[k];
        for (int k = 0; k < NH; ++k) {
            double dh = 0.0;
            for (int j = 0; j < NH; ++j)
                dh += bf16 ? split_mul(W2[j * NH + k], dz2[j]) : W2[j * NH + k] * dz2[j];
            dz1[k] = dh * (1.0 - s.h1[k] * s.h1[k]);
            grad[OFF_B1 + k] += dz1[k];
            grad[OFF_W1 + k * NI] += dz1[k] * xb[0];
            grad[OFF_W1 + k * NI + 1] += dz1[k] * xb[1];
        }
    }
    return loss;
}

/* Adam (Kingma & Ba 2015) with bias correction; step counts from 1. */
void m1o_adam(long np, double *theta, const double *g, double *m, double *v, long step,
              double lr, double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    for (long i = 0; i < np; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        theta[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
