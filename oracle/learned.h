/*
 * Reference checker for the learned form of the probe update.
 *
 * TEST INFRASTRUCTURE ONLY (like oracle.h): plain, slow binary64 code used by
 * the test-suite to check the GPU library's denoiser kernels; the library never
 * links or calls it.
 *
 * The learned form is an extension beyond the paper. Each frame it traces a
 * small ray set per probe, forms the Eq. 3 estimate from it, and lets a small
 * per-texel network map that noisy estimate (with the probe's history) to the
 * update a many-ray set would give for the frame. A second output of the network predicts
 * its own relative error; probes whose mean predicted error exceeds a threshold
 * (and probes without history) take the plain update instead.
 *
 * Network (one irradiance texel; parameters theta, binary32 masters):
 *   x  in R^16  features (slot layout in orc_learned_features)
 *   h1 = relu(W1 x)                 W1 [64][16]  (slot 12 of x is 1: the bias)
 *   h2 = relu(W2 h1 + b2)           W2 [64][64], b2 [64]
 *   h3 = relu(W3 h2 + b3)           W3 [64][64], b3 [64]
 *   o  = W4 h3 + b4                 W4 [4][64],  b4 [4]
 * theta = W1 | W2 | b2 | W3 | b3 | W4 | b4  (ORC_MLP_PARAMS values, row-major).
 *
 * Mirror mode reproduces where the GPU kernels round to bfloat16 (8 significant
 * bits, round to nearest even): the weight matrices, the network input, each
 * hidden activation after the ReLU and, in the backward pass, the output
 * gradient and each hidden gradient after its ReLU mask. Biases stay binary32
 * values; everything else here is binary64. Exact mode rounds nothing.
 *
 * Output mapping: the update U = max(0, E_prev + S * o[0..2]) per channel,
 * mixed into the irradiance with the hysteresis like the plain update;
 * predicted relative error r = exp(o[3]).
 */
#ifndef SDFDDGI_ORACLE_LEARNED_H
#define SDFDDGI_ORACLE_LEARNED_H

#include <stdint.h>

#include "oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_FEATURES 16
#define ORC_HIDDEN 64
#define ORC_OUTPUTS 4
#define ORC_OFF_W1 0
#define ORC_OFF_W2 (ORC_OFF_W1 + ORC_HIDDEN * ORC_FEATURES)
#define ORC_OFF_B2 (ORC_OFF_W2 + ORC_HIDDEN * ORC_HIDDEN)
#define ORC_OFF_W3 (ORC_OFF_B2 + ORC_HIDDEN)
#define ORC_OFF_B3 (ORC_OFF_W3 + ORC_HIDDEN * ORC_HIDDEN)
#define ORC_OFF_W4 (ORC_OFF_B3 + ORC_HIDDEN)
#define ORC_OFF_B4 (ORC_OFF_W4 + ORC_OUTPUTS * ORC_HIDDEN)
#define ORC_MLP_PARAMS (ORC_OFF_B4 + ORC_OUTPUTS)

typedef struct {
    double head_weight;   /* lambda: weight of the error-head term            */
    double min_error;     /* floor of the realised relative error (log target) */
} orc_loss_config;

/* Round to bfloat16 (8 significant bits, nearest even); keeps 0, inf, NaN. */
double orc_round_bf16(double v);

/* Forward pass. act (may be NULL) receives the three hidden activations. */
void orc_mlp_forward(const double *theta, const double x[ORC_FEATURES], int32_t mirror,
                     double o[ORC_OUTPUTS], double act[3][ORC_HIDDEN]);

/* orc_mlp_forward for n samples: x [n][16] -> o [n][4]. */
void orc_mlp_forward_batch(const double *theta, const double *x, int64_t n, int32_t mirror,
                           double *o);

/* Mean loss over n samples and its gradient with respect to theta (grad may be
 * NULL). targets[n][4] = (z0, z1, z2, denom): z = (U* - E_prev) / S is the
 * residual the irradiance outputs aim at, denom the relative-error scale.
 *   loss_n = sum_c (o_c - z_c)^2 + lambda (o_3 - ln max(r_n, r_min))^2,
 *   r_n = sum_c |o_c - z_c| / denom_n   (held constant in the gradient). */
double orc_mlp_loss_grad(const double *theta, const double *x /* [n][16] */,
                         const double *targets /* [n][4] */, int32_t n,
                         const orc_loss_config *cfg, int32_t mirror, double *grad);

/* One Adam step (Kingma & Ba 2015, Algorithm 1) on count parameters; t >= 1 is
 * the step number used for the bias corrections. */
void orc_adam_step(double *theta, double *m, double *v, const double *g, int32_t count,
                   int32_t t, double lr, double beta1, double beta2, double eps);

/* Index of minibatch sample i of a step: the first SplitMix64 output of the
 * state seed + i, reduced modulo count. */
int64_t orc_batch_index(uint64_t seed, int64_t i, int64_t count);

/* Signed distance at probe p's position: the binary32 cascade sampler at the
 * level the point selects (1e30 when the probe lies outside every level). */
double orc_probe_sdf(const orc_setup *s, int32_t p);

/* Feature vector of interior irradiance texel t (= i + res*j) of one probe:
 *   0..2   U_low / S   (low-ray Eq. 3 irradiance, no hysteresis)
 *   3..5   E_prev / S  (previous irradiance)
 *   6      mean of E[t] over the k x k depth texels covering texel t, / D
 *   7      sqrt(max(0, mean of E[t^2] over them)) / D
 *   8..10  texel centre direction
 *   11     probe signed distance / D, clamped to [-4, 4]
 *   12     1
 *   13..15 0
 * with k = depth_res / irr_res. Tiles are padded ([res+2][res+2][comps]). */
void orc_learned_features(const orc_setup *s, const double *u_irr_tile,
                          const double *prev_irr_tile, const double *prev_depth_tile,
                          double probe_sdf, int32_t t, double S, double D,
                          double x[ORC_FEATURES]);

/* orc_learned_features for every interior irradiance texel of the listed
 * probes (atlases of all probes, padded tiles); out [count][Ti][16]. */
void orc_learned_features_all(const orc_setup *s, const double *u_irr, const double *prev_irr,
                              const double *prev_depth, const int32_t *probes, int32_t count,
                              double S, double D, double *out);

#ifdef __cplusplus
}
#endif
#endif
