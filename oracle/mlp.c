/*
 * mlp.c -- FP64 reference of the bubbly-glass surrogate network (test
 * infrastructure, part of the CPU oracle).  Plain loops, no blocking.
 *
 * Network (a reading; the paper only names volume scattering as future work,
 * Sec. 6): input x = (cos(theta), (lambda - 580) / 200, (d - 3.5) / 1.5,
 * rho_b / 34, e[pane] (8 learned values)); three hidden layers of 64 with
 * ReLU; output o (3 values); heads R = exp(o0) / (exp(o0) + exp(o1) + 1),
 * T = exp(o1) / (same), w = softplus(o2); loss = mean over the batch of
 * (R - R*)^2 + (T - T*)^2 + (w - w*)^2.
 *
 * Parameter vector layout (float64 here, the same order everywhere):
 *   W1[64][12] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3]
 *   E[n_panes][8]
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "sdm_oracle.h"

#define NIN 12
#define NH 64
#define NOUT 3
#define NEMB 8

int64_t orc_mlp_nparams(int32_t n_panes)
{
    return (int64_t)NH * NIN + NH + NH * NH + NH + NH * NH + NH + NOUT * NH + NOUT + (int64_t)NEMB * n_panes;
}

typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4, *E;
} view;

static view make_view(const double *p)
{
    view v;
    v.W1 = p; p += NH * NIN;
    v.b1 = p; p += NH;
    v.W2 = p; p += NH * NH;
    v.b2 = p; p += NH;
    v.W3 = p; p += NH * NH;
    v.b3 = p; p += NH;
    v.W4 = p; p += NOUT * NH;
    v.b4 = p; p += NOUT;
    v.E = p;
    return v;
}

static void features(const double *tup, int pane, const view *v, double *x)
{
    x[0] = tup[0];
    x[1] = (tup[1] - 580.0) / 200.0;
    x[2] = (tup[2] - 3.5) / 1.5;
    x[3] = tup[3] / 34.0;
    for (int e = 0; e < NEMB; ++e) x[4 + e] = v->E[pane * NEMB + e];
}

static void dense(const double *W, const double *b, const double *x, int nin, int nout, double *y)
{
    for (int o = 0; o < nout; ++o) {
        double s = b[o];
        for (int i = 0; i < nin; ++i) s += W[o * nin + i] * x[i];
        y[o] = s;
    }
}

static void relu(double *z, int n, double *h)
{
    for (int i = 0; i < n; ++i) h[i] = z[i] > 0.0 ? z[i] : 0.0;
}

static double softplus(double x) { return x > 30.0 ? x : log1p(exp(x)); }

static void heads(const double *o, double *out)
{
    double m = fmax(fmax(o[0], o[1]), 0.0);
    double a = exp(o[0] - m), b = exp(o[1] - m), c = exp(-m);
    double s = a + b + c;
    out[0] = a / s;
    out[1] = b / s;
    out[2] = softplus(o[2]);
}

/* Round to the nearest bfloat16 (8 significant bits), ties to even, directly
 * from the double: x = f 2^e with f in [0.5, 1) becomes nearbyint(f 2^8)
 * 2^(e-8) under the default round-to-nearest-even mode.  Values below the
 * smallest normal bfloat16 (2^-126) keep 8 bits as well (no gradual
 * underflow; no such values occur in the network); inf and nan pass. */
double orc_bf16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    const double f = frexp(x, &e);
    return ldexp(nearbyint(ldexp(f, 8)), e - 8);
}

/* Layer with BF16 operands: y = b + sum bf16(W) bf16(x).  Only the operands
 * are rounded; the products, the sum and the bias are FP64, so this
 * is the plain definition of a dense layer on bfloat16 inputs (the matrix
 * cores' FP32 accumulation differs from it by FP32 rounding only). */
static void dense_bf16(const double *W, const double *b, const double *xb, int nin, int nout, double *y)
{
    for (int o = 0; o < nout; ++o) {
        double s = b[o];
        for (int i = 0; i < nin; ++i) s += orc_bf16(W[o * nin + i]) * xb[i];
        y[o] = s;
    }
}

/* Network evaluated with BF16 operands: the features, the weights and the
 * hidden activations are rounded to bfloat16 where they enter a product;
 * everything else (feature scaling, sums, biases, heads) is FP64. */
void orc_mlp_forward_bf16(const double *params, int32_t n_panes, int64_t m, const double *tuples,
                          const int32_t *panes, double *out)
{
    (void)n_panes;
    view v = make_view(params);
    for (int64_t s = 0; s < m; ++s) {
        double x[NIN], z1[NH], h1[NH], z2[NH], h2[NH], z3[NH], h3[NH], o[NOUT];
        features(tuples + 4 * s, panes[s], &v, x);
        for (int i = 0; i < NIN; ++i) x[i] = orc_bf16(x[i]);
        dense_bf16(v.W1, v.b1, x, NIN, NH, z1); relu(z1, NH, h1);
        for (int i = 0; i < NH; ++i) h1[i] = orc_bf16(h1[i]);
        dense_bf16(v.W2, v.b2, h1, NH, NH, z2); relu(z2, NH, h2);
        for (int i = 0; i < NH; ++i) h2[i] = orc_bf16(h2[i]);
        dense_bf16(v.W3, v.b3, h2, NH, NH, z3); relu(z3, NH, h3);
        for (int i = 0; i < NH; ++i) h3[i] = orc_bf16(h3[i]);
        dense_bf16(v.W4, v.b4, h3, NH, NOUT, o);
        heads(o, out + 3 * s);
    }
}

/* Test instrument: the BF16-operand network of one tuple (as
 * orc_mlp_forward_bf16) and a bound on how far an evaluation that sums the
 * same BF16 products in FP32 can lie from it, when its cos and thickness
 * inputs may also be off by e_cos and e_d (absolute).  A layer's
 * pre-activation z moves by at most E = |W| D + gamma (|b| + |W| (|h| + D)),
 * gamma = 65 u / (1 - 65 u), u = 2^-24 (an FP32 sum of at most 65 terms),
 * D bounding how far the layer's inputs h already differ.  The ReLU output
 * is rounded to BF16 again, and rounding is monotone, so the next layer's D
 * is the width of [bf16(max(z - E, 0)), bf16(max(z + E, 0))]: zero unless a
 * BF16 rounding boundary lies within E of z.  The scaled features start
 * within 4 u of their exact values.  The output bound is carried through
 * the heads by their derivatives (R(1 - R), RT, T(1 - T); the softplus
 * slope), with 5 % for second-order terms and 2e-6 for the heads' own FP32
 * rounding. */
static void layer_bound(const double *W, const double *b, const double *h, const double *D, int nin, int nout,
                        double gam, double *z, double *E)
{
    for (int o = 0; o < nout; ++o) {
        double s = b[o], a = fabs(b[o]), dd = 0.0;
        for (int i = 0; i < nin; ++i) {
            double wb = orc_bf16(W[o * nin + i]);
            s += wb * h[i];
            a += fabs(wb) * (fabs(h[i]) + D[i]);
            dd += fabs(wb) * D[i];
        }
        z[o] = s;
        E[o] = dd + gam * a;
    }
}

static void relu_bf16_interval(const double *z, const double *E, int n, double *h, double *D)
{
    for (int i = 0; i < n; ++i) {
        h[i] = orc_bf16(z[i] > 0.0 ? z[i] : 0.0);
        double hi = z[i] + E[i], lo = z[i] - E[i];
        D[i] = orc_bf16(hi > 0.0 ? hi : 0.0) - orc_bf16(lo > 0.0 ? lo : 0.0);
    }
}

void orc_mlp_bf16_bound(const double *params, const double *tup, int32_t pane, double e_cos, double e_d,
                        double out[3], double bound[3])
{
    view v = make_view(params);
    const double u = ldexp(1.0, -24), gam = 65.0 * u / (1.0 - 65.0 * u);
    double x[NIN], h0[NIN], D0[NIN], z[NH], E[NH], h[NH], D[NH], o[NOUT], eo[NOUT];
    features(tup, pane, &v, x);
    for (int i = 0; i < NIN; ++i) {
        double ex = 0.0;
        if (i == 0) ex = e_cos;
        else if (i == 1 || i == 3) ex = 4.0 * u * fabs(x[i]);
        else if (i == 2) ex = e_d / 1.5 + 4.0 * u * fabs(x[i]);
        h0[i] = orc_bf16(x[i]);
        D0[i] = orc_bf16(x[i] + ex) - orc_bf16(x[i] - ex);
    }
    layer_bound(v.W1, v.b1, h0, D0, NIN, NH, gam, z, E);
    relu_bf16_interval(z, E, NH, h, D);
    layer_bound(v.W2, v.b2, h, D, NH, NH, gam, z, E);
    relu_bf16_interval(z, E, NH, h, D);
    layer_bound(v.W3, v.b3, h, D, NH, NH, gam, z, E);
    relu_bf16_interval(z, E, NH, h, D);
    layer_bound(v.W4, v.b4, h, D, NH, NOUT, gam, o, eo);
    heads(o, out);
    double R = out[0], T = out[1];
    bound[0] = 1.05 * (R * (1.0 - R) * eo[0] + R * T * eo[1]) + 2e-6;
    bound[1] = 1.05 * (R * T * eo[0] + T * (1.0 - T) * eo[1]) + 2e-6;
    bound[2] = 1.05 * eo[2] / (1.0 + exp(-o[2])) + 2e-6;
}

/* tuples: m x 4 (cos, lambda_nm, d_mm, rho_b); panes: m; out: m x 3 (R, T, w) */
void orc_mlp_forward(const double *params, int32_t n_panes, int64_t m, const double *tuples,
                     const int32_t *panes, double *out)
{
    (void)n_panes;
    view v = make_view(params);
    for (int64_t s = 0; s < m; ++s) {
        double x[NIN], z1[NH], h1[NH], z2[NH], h2[NH], z3[NH], h3[NH], o[NOUT];
        features(tuples + 4 * s, panes[s], &v, x);
        dense(v.W1, v.b1, x, NIN, NH, z1); relu(z1, NH, h1);
        dense(v.W2, v.b2, h1, NH, NH, z2); relu(z2, NH, h2);
        dense(v.W3, v.b3, h2, NH, NH, z3); relu(z3, NH, h3);
        dense(v.W4, v.b4, h3, NH, NOUT, o);
        heads(o, out + 3 * s);
    }
}

/* Mean loss over m samples and its gradient with respect to every parameter. */
double orc_mlp_loss_grad(const double *params, int32_t n_panes, int64_t m, const double *tuples,
                         const int32_t *panes, const double *target, double *grad)
{
    view v = make_view(params);
    int64_t P = orc_mlp_nparams(n_panes);
    memset(grad, 0, sizeof(double) * (size_t)P);
    double *gW1 = grad, *gb1 = gW1 + NH * NIN, *gW2 = gb1 + NH, *gb2 = gW2 + NH * NH, *gW3 = gb2 + NH,
           *gb3 = gW3 + NH * NH, *gW4 = gb3 + NH, *gb4 = gW4 + NOUT * NH, *gE = gb4 + NOUT;
    double loss = 0.0;
    for (int64_t s = 0; s < m; ++s) {
        double x[NIN], z1[NH], h1[NH], z2[NH], h2[NH], z3[NH], h3[NH], o[NOUT], y[NOUT];
        features(tuples + 4 * s, panes[s], &v, x);
        dense(v.W1, v.b1, x, NIN, NH, z1); relu(z1, NH, h1);
        dense(v.W2, v.b2, h1, NH, NH, z2); relu(z2, NH, h2);
        dense(v.W3, v.b3, h2, NH, NH, z3); relu(z3, NH, h3);
        dense(v.W4, v.b4, h3, NH, NOUT, o);
        heads(o, y);
        const double *t = target + 3 * s;
        double e0 = y[0] - t[0], e1 = y[1] - t[1], e2 = y[2] - t[2];
        loss += e0 * e0 + e1 * e1 + e2 * e2;
        /* d loss / d (R, T, w), then through the heads */
        double gR = 2.0 * e0 / m, gT = 2.0 * e1 / m, gw = 2.0 * e2 / m;
        double R = y[0], T = y[1];
        double go[NOUT];
        go[0] = gR * R * (1.0 - R) + gT * (-T * R);
        go[1] = gR * (-R * T) + gT * T * (1.0 - T);
        go[2] = gw / (1.0 + exp(-o[2]));
        /* output layer */
        double gh3[NH] = {0}, gz3[NH], gh2[NH] = {0}, gz2[NH], gh1[NH] = {0}, gz1[NH], gx[NIN] = {0};
        for (int q = 0; q < NOUT; ++q) {
            gb4[q] += go[q];
            for (int i = 0; i < NH; ++i) {
                gW4[q * NH + i] += go[q] * h3[i];
                gh3[i] += go[q] * v.W4[q * NH + i];
            }
        }
        for (int i = 0; i < NH; ++i) gz3[i] = z3[i] > 0.0 ? gh3[i] : 0.0;
        for (int q = 0; q < NH; ++q) {
            gb3[q] += gz3[q];
            for (int i = 0; i < NH; ++i) {
                gW3[q * NH + i] += gz3[q] * h2[i];
                gh2[i] += gz3[q] * v.W3[q * NH + i];
            }
        }
        for (int i = 0; i < NH; ++i) gz2[i] = z2[i] > 0.0 ? gh2[i] : 0.0;
        for (int q = 0; q < NH; ++q) {
            gb2[q] += gz2[q];
            for (int i = 0; i < NH; ++i) {
                gW2[q * NH + i] += gz2[q] * h1[i];
                gh1[i] += gz2[q] * v.W2[q * NH + i];
            }
        }
        for (int i = 0; i < NH; ++i) gz1[i] = z1[i] > 0.0 ? gh1[i] : 0.0;
        for (int q = 0; q < NH; ++q) {
            gb1[q] += gz1[q];
            for (int i = 0; i < NIN; ++i) {
                gW1[q * NIN + i] += gz1[q] * x[i];
                gx[i] += gz1[q] * v.W1[q * NIN + i];
            }
        }
        for (int e = 0; e < NEMB; ++e) gE[panes[s] * NEMB + e] += gx[4 + e];
    }
    return loss / m;
}
