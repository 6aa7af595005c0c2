/*
 * Reference checker for the learned form of the probe update (see learned.h).
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow binary64 code for the test-suite. It
 * shares no code with the GPU library.
 */
#include "learned.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

double orc_round_bf16(double v)
{
    if (v == 0.0 || !isfinite(v)) return v;
    /* bfloat16 keeps binary32's exponent range: 8 significant bits for normal
     * values (|v| >= 2^-126), a fixed quantum of 2^-133 below that */
    double a = fabs(v);
    double q;
    if (a < 0x1p-126) {
        q = 0x1p-133;
    } else {
        int e;
        frexp(a, &e);      /* a = m 2^e, m in [0.5, 1) */
        q = ldexp(1.0, e - 8);
    }
    double k = a / q;      /* exact: a scaled by a power of two */
    double fl = floor(k);
    double frac = k - fl;
    double r;
    if (frac > 0.5) r = fl + 1.0;
    else if (frac < 0.5) r = fl;
    else r = fmod(fl, 2.0) == 0.0 ? fl : fl + 1.0;
    double out = r * q;
    return v < 0 ? -out : out;
}

static double rnd(double v, int32_t mirror) { return mirror ? orc_round_bf16(v) : v; }

/* y[rows] = W[rows][cols] x[cols] (+ b) with optional bfloat16 rounding of W. */
static void affine(const double *W, const double *b, const double *x, int32_t rows,
                   int32_t cols, int32_t mirror, double *y)
{
    for (int32_t r = 0; r < rows; ++r) {
        double acc = b ? b[r] : 0.0;
        for (int32_t c = 0; c < cols; ++c) acc += rnd(W[(size_t)r * cols + c], mirror) * x[c];
        y[r] = acc;
    }
}

typedef struct {
    double x[ORC_FEATURES];                 /* network input (rounded in mirror mode) */
    double a[3][ORC_HIDDEN];                /* pre-activations of the hidden layers */
    double h[3][ORC_HIDDEN];                /* activations (rounded in mirror mode) */
    double o[ORC_OUTPUTS];
} fwd_state;

static void forward(const double *theta, const double *x, int32_t mirror, fwd_state *st)
{
    for (int k = 0; k < ORC_FEATURES; ++k) st->x[k] = rnd(x[k], mirror);
    affine(theta + ORC_OFF_W1, NULL, st->x, ORC_HIDDEN, ORC_FEATURES, mirror, st->a[0]);
    for (int k = 0; k < ORC_HIDDEN; ++k) st->h[0][k] = rnd(st->a[0][k] > 0 ? st->a[0][k] : 0, mirror);
    affine(theta + ORC_OFF_W2, theta + ORC_OFF_B2, st->h[0], ORC_HIDDEN, ORC_HIDDEN, mirror, st->a[1]);
    for (int k = 0; k < ORC_HIDDEN; ++k) st->h[1][k] = rnd(st->a[1][k] > 0 ? st->a[1][k] : 0, mirror);
    affine(theta + ORC_OFF_W3, theta + ORC_OFF_B3, st->h[1], ORC_HIDDEN, ORC_HIDDEN, mirror, st->a[2]);
    for (int k = 0; k < ORC_HIDDEN; ++k) st->h[2][k] = rnd(st->a[2][k] > 0 ? st->a[2][k] : 0, mirror);
    affine(theta + ORC_OFF_W4, theta + ORC_OFF_B4, st->h[2], ORC_OUTPUTS, ORC_HIDDEN, mirror, st->o);
}

void orc_mlp_forward(const double *theta, const double x[ORC_FEATURES], int32_t mirror,
                     double o[ORC_OUTPUTS], double act[3][ORC_HIDDEN])
{
    fwd_state st;
    forward(theta, x, mirror, &st);
    memcpy(o, st.o, sizeof st.o);
    if (act) memcpy(act, st.h, sizeof st.h);
}

void orc_mlp_forward_batch(const double *theta, const double *x, int64_t n, int32_t mirror,
                           double *o)
{
    for (int64_t s = 0; s < n; ++s) {
        fwd_state st;
        forward(theta, x + (size_t)s * ORC_FEATURES, mirror, &st);
        memcpy(o + (size_t)s * ORC_OUTPUTS, st.o, sizeof st.o);
    }
}

/* g_in[cols] = mask(a) * (W^T g_out) for one layer, rounded in mirror mode. */
static void back_hidden(const double *W, const double *g_out, int32_t rows, int32_t cols,
                        const double *a, int32_t mirror, double *g_in)
{
    for (int32_t c = 0; c < cols; ++c) {
        double acc = 0.0;
        for (int32_t r = 0; r < rows; ++r) acc += rnd(W[(size_t)r * cols + c], mirror) * g_out[r];
        g_in[c] = rnd(a[c] > 0 ? acc : 0.0, mirror);
    }
}

/* dW[rows][cols] += g[rows] in[cols]^T, db[rows] += g. */
static void outer_add(double *dW, double *db, const double *g, const double *in, int32_t rows,
                      int32_t cols)
{
    for (int32_t r = 0; r < rows; ++r) {
        for (int32_t c = 0; c < cols; ++c) dW[(size_t)r * cols + c] += g[r] * in[c];
        if (db) db[r] += g[r];
    }
}

double orc_mlp_loss_grad(const double *theta, const double *x, const double *targets, int32_t n,
                         const orc_loss_config *cfg, int32_t mirror, double *grad)
{
    if (grad) memset(grad, 0, sizeof(double) * ORC_MLP_PARAMS);
    if (n <= 0) return 0.0;
    double loss = 0.0;
    const double inv_n = 1.0 / (double)n;
    for (int32_t s = 0; s < n; ++s) {
        fwd_state st;
        forward(theta, x + (size_t)s * ORC_FEATURES, mirror, &st);
        const double *z = targets + (size_t)s * 4;
        double err = 0.0, sq = 0.0;
        for (int c = 0; c < 3; ++c) {
            double d = st.o[c] - z[c];
            sq += d * d;
            err += fabs(d);
        }
        double r = err / z[3];
        double lr = log(r > cfg->min_error ? r : cfg->min_error);
        double dh = st.o[3] - lr;
        loss += (sq + cfg->head_weight * dh * dh) * inv_n;
        if (!grad) continue;
        double go[ORC_OUTPUTS];
        for (int c = 0; c < 3; ++c) go[c] = rnd(2.0 * inv_n * (st.o[c] - z[c]), mirror);
        go[3] = rnd(2.0 * cfg->head_weight * inv_n * dh, mirror);
        double g3[ORC_HIDDEN], g2[ORC_HIDDEN], g1[ORC_HIDDEN];
        back_hidden(theta + ORC_OFF_W4, go, ORC_OUTPUTS, ORC_HIDDEN, st.a[2], mirror, g3);
        back_hidden(theta + ORC_OFF_W3, g3, ORC_HIDDEN, ORC_HIDDEN, st.a[1], mirror, g2);
        back_hidden(theta + ORC_OFF_W2, g2, ORC_HIDDEN, ORC_HIDDEN, st.a[0], mirror, g1);
        outer_add(grad + ORC_OFF_W4, grad + ORC_OFF_B4, go, st.h[2], ORC_OUTPUTS, ORC_HIDDEN);
        outer_add(grad + ORC_OFF_W3, grad + ORC_OFF_B3, g3, st.h[1], ORC_HIDDEN, ORC_HIDDEN);
        outer_add(grad + ORC_OFF_W2, grad + ORC_OFF_B2, g2, st.h[0], ORC_HIDDEN, ORC_HIDDEN);
        outer_add(grad + ORC_OFF_W1, NULL, g1, st.x, ORC_HIDDEN, ORC_FEATURES);
    }
    return loss;
}

void orc_adam_step(double *theta, double *m, double *v, const double *g, int32_t count,
                   int32_t t, double lr, double beta1, double beta2, double eps)
{
    const double c1 = 1.0 - pow(beta1, (double)t);
    const double c2 = 1.0 - pow(beta2, (double)t);
    for (int32_t k = 0; k < count; ++k) {
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
        const double mh = m[k] / c1, vh = v[k] / c2;
        theta[k] -= lr * mh / (sqrt(vh) + eps);
    }
}

int64_t orc_batch_index(uint64_t seed, int64_t i, int64_t count)
{
    uint64_t st = seed + (uint64_t)i;
    return (int64_t)(orc_splitmix64(&st) % (uint64_t)count);
}

double orc_probe_sdf(const orc_setup *s, int32_t p)
{
    double pos[3];
    orc_probe_position(s, p, pos);
    float x[3] = {(float)pos[0], (float)pos[1], (float)pos[2]};
    int32_t L = orc_level32(s, x);
    if (L < 0) return 1e30;
    return (double)orc_sdf32(s, L, x);
}

void orc_learned_features(const orc_setup *s, const double *u_irr_tile,
                          const double *prev_irr_tile, const double *prev_depth_tile,
                          double probe_sdf, int32_t t, double S, double D,
                          double x[ORC_FEATURES])
{
    const int32_t ri = s->irr_res, rd = s->depth_res;
    const int32_t i = t % ri, j = t / ri;
    const int32_t si = ri + 2, sd = rd + 2;
    const size_t at = ((size_t)(j + 1) * si + (size_t)(i + 1)) * 3;
    for (int c = 0; c < 3; ++c) {
        x[c] = u_irr_tile[at + c] / S;
        x[3 + c] = prev_irr_tile[at + c] / S;
    }
    /* the depth texels whose octahedral cells tile irradiance texel (i, j) */
    const int32_t k = rd / ri;
    double m1 = 0.0, m2 = 0.0;
    for (int32_t b = 0; b < k; ++b)
        for (int32_t a = 0; a < k; ++a) {
            const size_t d = ((size_t)(k * j + b + 1) * sd + (size_t)(k * i + a + 1)) * 2;
            m1 += prev_depth_tile[d];
            m2 += prev_depth_tile[d + 1];
        }
    m1 /= (double)(k * k);
    m2 /= (double)(k * k);
    x[6] = m1 / D;
    x[7] = sqrt(m2 > 0.0 ? m2 : 0.0) / D;
    double dir[3];
    orc_texel_direction(ri, i, j, dir);
    x[8] = dir[0];
    x[9] = dir[1];
    x[10] = dir[2];
    double q = probe_sdf / D;
    x[11] = q < -4.0 ? -4.0 : (q > 4.0 ? 4.0 : q);
    x[12] = 1.0;
    x[13] = x[14] = x[15] = 0.0;
}

void orc_learned_features_all(const orc_setup *s, const double *u_irr, const double *prev_irr,
                              const double *prev_depth, const int32_t *probes, int32_t count,
                              double S, double D, double *out)
{
    const size_t ti = (size_t)(s->irr_res + 2) * (s->irr_res + 2) * 3;
    const size_t td = (size_t)(s->depth_res + 2) * (s->depth_res + 2) * 2;
    const int32_t T = s->irr_res * s->irr_res;
    for (int32_t q = 0; q < count; ++q) {
        const int32_t p = probes[q];
        const double sdf = orc_probe_sdf(s, p);
        for (int32_t t = 0; t < T; ++t)
            orc_learned_features(s, u_irr + p * ti, prev_irr + p * ti, prev_depth + p * td, sdf, t,
                                 S, D, out + ((size_t)q * T + t) * ORC_FEATURES);
    }
}
