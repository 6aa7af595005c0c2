/*
 * sdfddgi.h -- C ABI of the MI355X (gfx950) implementation of the per-frame
 * probe update of "Signed Distance Fields Dynamic Diffuse Global Illumination"
 * (Hu et al., arXiv 2007.14394), Sec. 3.3 "Probe update".
 *
 * One call to sdfddgi_update_frame performs, for every probe of a uniform
 * grid (Sec. 3.2, Eq. 2: irradiance sampled at probe positions P over
 * directions D):
 *   1. rotate a spherical-Fibonacci ray set by one random rotation drawn from
 *      the frame's seed (Sec. 3.3: random low-discrepancy directions);
 *   2. sphere-trace every ray through the baked signed distance grid (Sec. 3.3);
 *   3. shade each hit with the sun seen through an SDF shadow ray plus the
 *      previous frame's probe irradiance times the multi-bounce coefficient
 *      (Sec. 3.3, multi-bounce through last frame's probes);
 *   4. estimate Eq. 3, E(D) = integral over the sphere of max(0, cos(D, D'))
 *      L(D') dD', for every texel direction D of the probe's octahedral map, and
 *      the first two moments of the ray distances for the depth map;
 *   5. mix with the previous values (Sec. 3.3, temporal mixing; skipped for
 *      probes whose history is rejected, Alg. 1 markRejectHistory) and fill
 *      the octahedral one-texel border.
 *
 * Numerical contract (what the library computes, exactly):
 *   - Ray directions: ray i of R is the spherical-Fibonacci point
 *     z = 1 - (2i+1)/R, r = sqrt(1 - z^2), phi = 2 pi frac(i*g), g = (sqrt5-1)/2,
 *     rotated by the matrix of Shoemake's uniform random quaternion built
 *     from three SplitMix64 draws u = (x >> 11) * 2^-53 of the frame seed, all
 *     in binary64 and rounded once to binary32 (sdfddgi_ray_directions).
 *   - Geometry (the decisions): binary32 with one fixed operation order --
 *     grid coordinate u = (x - (float)origin) * (float)(1/spacing); cell
 *     clamp(floor(u), 0, n-2); fraction clamp(u - cell, 0, 1); trilinear as
 *     three rounds of lerps a + f*(b - a) evaluated as fma(f, b - a, a)
 *     (x, then y, then z); sample point x = fma(t, w, o); step t = fma(relax, d, t).
 *     Cascade level = finest level whose box shrunk by one voxel holds x (the
 *     coarsest level counts with its full box; outside it the ray escapes).
 *     A ray stops on: t > t_max (miss), leaving the grid (miss), d < 0 at the
 *     first sample of a probe ray (inside), d < hit_eps (hit), or after
 *     max_steps samples (hit at the last sample). Normal = central differences
 *     at +-spacing/2 on the hit's level, scaled by 1/sqrt(|g|^2) (falls back to
 *     -w when |g|^2 < 1e-24). Shadow ray from fma(n, shadow_bias, x) toward the
 *     light, traced only where n.l > 0; blocked on a hit or on running out of
 *     steps.
 *   - Radiometry: ray radiance = albedo/pi * (E_sun + bounce_gain * E_prev),
 *     E_sun = radiance * max(0, n.l) * visible, E_prev = the previous atlas
 *     interpolated at (x, n) like sdfddgi_sample_irradiance; a miss carries
 *     sky_rgb at distance t_max, a probe inside geometry carries 0 at 0.
 *   - Eq. 3 estimator: E_t = pi * sum_i w_ti L_i / sum_i w_ti with
 *     w_ti = max(0, n_t . w_i); depth moments sum_i w_ti^s (t_i, t_i^2) /
 *     sum_i w_ti^s with s = depth_sharpness. Blend M = h M_old + (1-h) E with
 *     h = hysteresis, or M = E for a probe whose history is rejected.
 *   - Accuracy: ray decisions (outcome, step counts, shadow result, distance
 *     and normal bits) are bit-identical to a binary32 evaluation of the
 *     sequence above; maps agree with a binary64 evaluation of the
 *     radiometry to about 1e-5 relative.
 *
 * Layouts (row-major, x fastest):
 *   SDF level    float [n2][n1][n0], vertex (i,j,k) at origin + spacing*(i,j,k)
 *   albedo level float [n2][n1][n0][3]
 *   probes       p = x + nx*(y + ny*z), position origin + spacing*(x,y,z)
 *   irradiance   float [P][irr_res+2][irr_res+2][3]  (rows = v, columns = u of
 *                the octahedral square; interior 1..irr_res, texel (i,j) centre
 *                at u = (i+1/2)/res*2-1, v = (j+1/2)/res*2-1; z folds at |u|+|v|=1)
 *   depth        float [P][depth_res+2][depth_res+2][2]  (E[t], E[t^2])
 *   payload      float [P][R][4]  (R, G, B, t) per ray
 *   ray records  int32 [P][R][8]  (outcome | level<<8, steps, visibility
 *                (1 lit, 0 blocked, -1 not traced), shadow steps, bits of t,
 *                bits of the normal's x, y, z)
 *
 * Conventions:
 *   - Every array argument except those of sdfddgi_ray_directions is a DEVICE
 *     pointer owned by the caller and only read/written during the call's
 *     stream-ordered work; sdfddgi_create copies the grids into memory the
 *     context owns, so the caller may free them once create returns.
 *   - GPU work goes on the stream given to sdfddgi_create, in order, and is
 *     asynchronous: results are valid once the caller synchronises that stream.
 *     The one exception is internal: back-to-back sdfddgi_update_frame calls
 *     run each frame's tables and primary trace on a side stream of the context
 *     and, on grid contexts, the atlas-independent half of its hit shading
 *     (normal, shadow ray, albedo) on a second one (default priority), both
 *     overlapping the previous frame's lookups and blend, and join them back
 *     into the caller's stream before the frame's multi-bounce lookups -- so the
 *     rule above still holds for every result.
 *   - Status codes only; nothing is thrown across the ABI. A failed call leaves
 *     the context's maps as they were. sdfddgi_last_error gives the message.
 *   - A context is used by one host thread at a time (no internal locking).
 *     Calls on different contexts are independent.
 */
#ifndef SDFDDGI_H
#define SDFDDGI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sdfddgi_ctx sdfddgi_ctx;

typedef enum {
    SDFDDGI_OK = 0,
    SDFDDGI_EINVAL = 1,   /* bad argument: sizes, non-finite values, NULL pointers */
    SDFDDGI_ENOMEM = 2,   /* device or host allocation failed                      */
    SDFDDGI_EDEVICE = 3,  /* no usable gfx950 device, or a HIP call/launch failed  */
    SDFDDGI_ESTATE = 4    /* call not valid in the context's current state         */
} sdfddgi_status;

#define SDFDDGI_MAX_LEVELS 4
#define SDFDDGI_MAX_RAYS 1024

/* Context flags (sdfddgi_params.flags). */
#define SDFDDGI_FLAG_RECORD_RAYS 1u  /* keep per-ray records (sdfddgi_get_ray_records) */
#define SDFDDGI_FLAG_TIMING 2u       /* time each kernel with events (sdfddgi_get_kernel_times) */
/* Precision form: the SDF is stored in binary16 (each value clamped to +-65504 and
 * rounded to nearest even at create; stepping still runs in binary32 on the
 * widened values, so ray decisions are those of the binary32 sequence on that
 * rounded grid), and the Eq. 3 contraction runs on FP16 (irradiance) and BF16
 * (depth moments) MFMA with FP32 accumulation; hysteresis stays binary32. */
#define SDFDDGI_FLAG_FP16 4u

/* One level of the baked distance grid. Level 0 is the finest; each coarser
 * level must contain the finer ones (a nested cascade). */
typedef struct {
    int32_t n[3];              /* vertices per axis, each >= 2                    */
    double origin[3];          /* position of vertex (0,0,0)                     */
    double spacing;            /* vertex spacing (cubic voxels), > 0             */
    const float *sdf;          /* device [n2][n1][n0]                            */
    const float *albedo_rgb;   /* device [n2][n1][n0][3], or NULL: params.albedo */
} sdfddgi_sdf_level;

typedef struct {
    int32_t num_levels;                          /* 1..SDFDDGI_MAX_LEVELS */
    sdfddgi_sdf_level level[SDFDDGI_MAX_LEVELS];
} sdfddgi_sdf_grid;

/* The uniform probe grid of Sec. 3.2 (sdfddgi_relocate_probes applies Alg. 1). */
typedef struct {
    int32_t n[3];              /* probes per axis, each >= 2 */
    double origin[3];
    double spacing[3];         /* each > 0 */
} sdfddgi_probe_grid;

typedef struct {
    int32_t rays_per_probe;    /* R: multiple of 16, 16..SDFDDGI_MAX_RAYS          */
    int32_t max_steps;         /* sphere-trace samples per ray, 1..4096            */
    int32_t irr_res;           /* irradiance map side (interior), 2..32; 8 typical */
    int32_t depth_res;         /* depth map side (interior), 2..32; 16 typical     */
    float hit_eps;             /* hit when the distance falls below this, > 0      */
    float t_max;               /* longest ray, > 0                                 */
    float hysteresis;          /* weight of the old value, [0, 1)                  */
    float bounce_gain;         /* multi-bounce coefficient, [0, 1]                 */
    float depth_sharpness;     /* cosine power of the depth weights, >= 0          */
    float shadow_bias;         /* shadow-ray origin offset along the normal, >= 0  */
    float relax;               /* step = relax * distance, (0, 2]                  */
    float sky_rgb[3];          /* radiance of escaping rays, finite, >= 0          */
    float albedo[3];           /* albedo where a level has no albedo grid          */
    uint32_t flags;            /* SDFDDGI_FLAG_*                                   */
    /* Learned form (sdfddgi_update_frame_learned); 0 rays: not available. */
    int32_t learned_rays;      /* low ray count: 0, or a multiple of 16 in 16..R   */
    float fallback_error;      /* tau: mean predicted relative error above which a
                                  probe takes the plain update in the learned frame
                                  after next, >= 0 (+inf: only probes without
                                  history or without a prediction do)              */
} sdfddgi_params;

/* Directional light: direction toward the light (any non-zero length; it is
 * normalised in binary64) and its radiance. */
typedef struct {
    float dir_to_light[3];
    float radiance_rgb[3];
} sdfddgi_light;

/* Fill *p with the defaults used for the 8x8 / 16x16 maps: 144 rays, 64 steps,
 * eps 1e-3, t_max 2*sqrt(3), h 0.97, gain 1, s 50, bias 4e-3, relax 1, black
 * sky, albedo 0.5, no flags, no learned form (0 rays, tau 0.02). Host only. */
void sdfddgi_default_params(sdfddgi_params *p);

/* Create a context on the current HIP device: validates the arguments, copies
 * the grids (device to device) into context-owned memory, allocates both
 * atlas pairs (zeroed; every probe's history starts rejected), and waits for
 * the copies. hip_stream: the hipStream_t all later work runs on (NULL: the
 * null stream). On failure *out is set to NULL. */
sdfddgi_status sdfddgi_create(const sdfddgi_sdf_grid *sdf, const sdfddgi_probe_grid *probes,
                              const sdfddgi_params *params, void *hip_stream,
                              sdfddgi_ctx **out);

/* A context whose probe update traces the scene's primitives instead of a baked
 * grid (Sec. 3.1: the scene as a union of signed distance primitives; Sec. 3.3:
 * their distance queried with cluster culling and the 2 lastSDF bound along a
 * ray). Host arrays, as for sdfddgi_bake_sdf: kind[nprims] (0 sphere of radius
 * half[.][0], 1 axis-aligned box of half extents half[.][0..2]),
 * center/half/albedo [nprims][3] (binary64; distances use their binary32
 * roundings, albedo >= 0), 1 <= nprims <= 1024, primitives packed cluster_size
 * (1..64) to a cluster in Morton order of their centres, at most 256 clusters.
 * The update then differs from the grid's only in the scene query: a sample's
 * distance is the minimum over the primitives (equal bit for bit to the
 * brute-force minimum), a ray misses only past t_max (there is no grid box), a
 * hit's normal is the normalised gradient of the nearest primitive's distance
 * (the lowest index among equals; -w where it vanishes) and its albedo that
 * primitive's; records report level 0. Everything else is sdfddgi_create's.
 * Not with SDFDDGI_FLAG_FP16 or learned_rays > 0 (EINVAL); relocation is ESTATE. */
sdfddgi_status sdfddgi_create_analytic(int32_t nprims, const int32_t *kind, const double *center,
                                       const double *half, const double *albedo,
                                       int32_t cluster_size, const sdfddgi_probe_grid *probes,
                                       const sdfddgi_params *params, void *hip_stream,
                                       sdfddgi_ctx **out);

/* One frame of the probe update of Sec. 3.3 for every probe (steps 1-5
 * above). Reads the current maps as the previous frame, writes the other
 * buffer pair, then makes it current. Clears every probe's reject flag.
 * Consecutive calls with no other call on the context in between overlap (see
 * the stream convention above); the results are the same as one at a time.
 * A context created with SDFDDGI_FLAG_RECORD_RAYS never overlaps frames. */
sdfddgi_status sdfddgi_update_frame(sdfddgi_ctx *ctx, const sdfddgi_light *light,
                                    uint64_t rotation_seed);

/* Irradiance at points for normals from the current irradiance atlas: trilinear
 * over the 8 probes of the cell holding each point (cell clamped to the grid),
 * each probe read bilinearly from its padded octahedral tile at the normal's
 * direction (the probe interpolation of Sec. 3.4, without visibility
 * weighting). points, normals: device [n][3]; normals need not be unit length
 * but must be non-zero; out_rgb: device [n][3]. n = 0 is a no-op. */
sdfddgi_status sdfddgi_sample_irradiance(sdfddgi_ctx *ctx, const float *points,
                                         const float *normals, int64_t n, float *out_rgb);

/* Steps 4-5 alone on a caller-provided payload (device [P][R][4]: R, G, B, t),
 * with the ray directions of rotation_seed; like update_frame it reads the
 * current maps, writes the other pair, makes it current and clears the reject
 * flags. Lets a caller with its own tracer use the blend. */
sdfddgi_status sdfddgi_blend(sdfddgi_ctx *ctx, const float *payload, uint64_t rotation_seed);

/* Copy the current maps out to device buffers (layouts above); either may be NULL. */
sdfddgi_status sdfddgi_get_maps(sdfddgi_ctx *ctx, float *irr, float *depth);

/* Install maps (e.g. a checkpoint) as the current ones and mark every probe's
 * history valid. Both pointers are required. */
sdfddgi_status sdfddgi_set_maps(sdfddgi_ctx *ctx, const float *irr, const float *depth);

/* Reject every probe's history: the next frame writes its new estimate
 * without mixing in the old maps (Alg. 1, markRejectHistory). */
sdfddgi_status sdfddgi_reset_history(sdfddgi_ctx *ctx);

/* Copy the last frame's per-ray payload (device [P][R][4]). ESTATE before the
 * first frame. */
sdfddgi_status sdfddgi_get_payload(sdfddgi_ctx *ctx, float *out);

/* Copy the last frame's per-ray records (device int32 [P][R][8]). ESTATE if
 * the context was created without SDFDDGI_FLAG_RECORD_RAYS or before the
 * first frame. */
sdfddgi_status sdfddgi_get_ray_records(sdfddgi_ctx *ctx, int32_t *out);

/* Copy the last frame's binary32 ray directions (device [R][3]). */
sdfddgi_status sdfddgi_get_ray_directions(sdfddgi_ctx *ctx, float *out);

/* The binary32 ray directions of a frame seed, computed on the host (host
 * pointer out [rays][3]); identical to what the GPU uses for that seed. */
sdfddgi_status sdfddgi_ray_directions(uint64_t rotation_seed, int32_t rays, float *out);

/* Mean per-kernel GPU times in milliseconds over the update_frame calls (plain
 * or learned) made since the previous call of this function (at most the last
 * 256), measured with events recorded on the context's stream around each
 * kernel: [0] ray-direction/weight tables (in back-to-back plain frames on
 * grids their weight rows, which run beside the trace while the directions block
 * runs ahead of it; in a learned frame the low set's directions block, its weight
 * rows running before the low-ray blend), [1] primary sphere trace, [2] hit
 * shading (normal, shadow ray, lookups), [3] blend, [4] whole frame,
 * [5] denoiser, [6] fallback trace (tables, list, primary, shadow rays),
 * [7] fallback lookups and blend. In a learned frame [1]-[3] are the low-ray
 * pass. Where the hit shading is split (learned frames, and back-to-back plain
 * frames on grid contexts) the atlas-independent half (normal, shadow ray,
 * albedo) runs beside the previous frame and the lookups after it, and [2]
 * spans both; [5]-[7] are 0 in a plain frame.
 * Host pointer ms[count], count <= 8. Waits for the last timed frame.
 * ESTATE without SDFDDGI_FLAG_TIMING or when no frame ran since the last call. */
sdfddgi_status sdfddgi_get_kernel_times(sdfddgi_ctx *ctx, float *ms, int32_t count);

/* Alg. 1 (UpdateProbePos) for every probe, on the context's stream: from its grid
 * position x, while the SDF at x is below threshold1 (at most `iterations`
 * times), step along the normalised SDF gradient (the hit-normal rule; +y where
 * it vanishes) by threshold1 - SDF(x), a Newton step on the distance field;
 * each coordinate stays within max_offset * spacing of the grid position, and a
 * probe outside every level stays where it is. All binary32:
 *   x_c = min(max(fma(threshold1 - d, n_c, x_c), g_c - o_c), g_c + o_c).
 * A probe whose new position is more than threshold2 from its position before
 * this call has its history rejected (markRejectHistory). Rays start from the
 * new positions from the next frame on; the probe interpolation keeps using the
 * grid cells. The paper gives no threshold values; they are arguments here. */
sdfddgi_status sdfddgi_relocate_probes(sdfddgi_ctx *ctx, float threshold1, float threshold2,
                                       int32_t iterations, float max_offset);

/* Copy the current probe positions (device [P][3], binary32). */
sdfddgi_status sdfddgi_get_probe_positions(sdfddgi_ctx *ctx, float *out);

/* Sizes of the context's problem: probes P, rays R, and the float counts of
 * one irradiance and one depth atlas. Host pointers; any may be NULL. */
sdfddgi_status sdfddgi_get_sizes(const sdfddgi_ctx *ctx, int64_t *probes, int32_t *rays,
                                 int64_t *irr_floats, int64_t *depth_floats);

/* Message of the context's last failure ("" if none). With ctx == NULL: the
 * message of the last failed sdfddgi_create on this thread. */
const char *sdfddgi_last_error(const sdfddgi_ctx *ctx);

/* Wait for the context's stream, then free everything the context owns.
 * NULL is a no-op. */
sdfddgi_status sdfddgi_destroy(sdfddgi_ctx *ctx);

/* ------------------------------------------------------------ learned form --
 * An extension beyond the paper: each frame traces learned_rays rays per probe,
 * forms the Eq. 3 estimate U_low from them (no hysteresis), and a per-texel
 * network maps it, with the probe's history, to the estimate of the frame's
 * update with many rays. Per interior irradiance texel t the network reads
 *   x = (U_low/S [3], E_prev/S [3], mean E[d]/D, sqrt(mean E[d^2])/D over the
 *        k x k depth texels covering t (k = depth_res/irr_res), texel direction
 *        [3], clamp(probe signed distance / D, -4, 4), 1, 0, 0, 0)
 * and computes h1 = relu(W1 x), h2 = relu(W2 h1 + b2), h3 = relu(W3 h2 + b3),
 * o = W4 h3 + b4 (16 -> 64 -> 64 -> 64 -> 4) with bfloat16 weights, inputs and
 * activations (round to nearest even) and FP32 accumulation on MFMA. The
 * texel's update is U_hat = max(0, E_prev + S o[0..2]) and its predicted
 * relative error exp(o[3]). Which probes take the plain update with
 * rays_per_probe rays instead is decided before the frame's trace: those whose
 * history is rejected, and those whose mean predicted error over their texels
 * in the learned frame before the previous one exceeded fallback_error (every
 * probe in the context's first two learned frames; the predictions persist
 * across set_maps and plain frames). The network still runs for them, to
 * predict for the learned frame after next. Every other probe
 * mixes U_hat into its irradiance (hysteresis, then borders) and the low-ray
 * depth moments into its depth map. Requires learned_rays > 0, depth_res an
 * even multiple of irr_res and irr_res <= 16.
 *
 * Parameter vector (binary32, SDFDDGI_DENOISER_PARAMS values, row-major):
 *   W1 [64][16] | W2 [64][64] | b2 [64] | W3 [64][64] | b3 [64] | W4 [4][64] | b4 [4] */
#define SDFDDGI_DENOISER_PARAMS 9604
#define SDFDDGI_FEATURES 16

typedef struct sdfddgi_denoiser sdfddgi_denoiser;

/* Upload a network (host params[count], count == SDFDDGI_DENOISER_PARAMS, all
 * finite) with its feature scales S = irr_scale and D = depth_scale (both > 0)
 * to the current device and pack its bfloat16 MFMA operands. hip_stream as in
 * sdfddgi_create. */
sdfddgi_status sdfddgi_denoiser_create(const float *params, int32_t count, float irr_scale,
                                       float depth_scale, void *hip_stream,
                                       sdfddgi_denoiser **out);

/* The network on n feature vectors: device features[n][16] -> device out[n][4]
 * (o[0..3] above). n = 0 is a no-op. */
sdfddgi_status sdfddgi_denoiser_infer(sdfddgi_denoiser *den, const float *features, int64_t n,
                                      float *out);

sdfddgi_status sdfddgi_denoiser_destroy(sdfddgi_denoiser *den);

/* One learned frame (see above) on the context's stream; like update_frame it
 * reads the current maps, writes the other pair, makes it current and clears
 * the reject flags of the probes it updated plainly. ESTATE if the context was
 * created with learned_rays == 0; EINVAL if den is on another device. */
sdfddgi_status sdfddgi_update_frame_learned(sdfddgi_ctx *ctx, const sdfddgi_denoiser *den,
                                            const sdfddgi_light *light, uint64_t rotation_seed);

/* The last learned frame's fallback: *count (host) = number of probes that took
 * the plain update; probes (device [P], may be NULL) receives their indices in
 * no particular order, mean_error (device [P], may be NULL) every probe's mean
 * predicted relative error in that frame (which decides the learned frame after
 * next). Waits for the stream. ESTATE before a learned frame. */
sdfddgi_status sdfddgi_get_fallback(sdfddgi_ctx *ctx, int32_t *count, int32_t *probes,
                                    float *mean_error);

/* Training pairs for the network from the current maps, without changing them:
 * traces learned_rays per probe for the frame, forms U_low, and writes for every
 * probe p and interior irradiance texel t (row p*Ti + t):
 *   features[.][16] = x above (the denoiser's S and D),
 *   targets[.][4]   = ((T - E_prev)/S [3], |T|_1 / S + rel_floor)
 * with T the texel of target_irr, an irradiance atlas of the context's layout
 * (e.g. the many-ray plain update of the same frame from the same maps, without
 * hysteresis). Device pointers; the context's stream. */
sdfddgi_status sdfddgi_learned_examples(sdfddgi_ctx *ctx, const sdfddgi_denoiser *den,
                                        const sdfddgi_light *light, uint64_t rotation_seed,
                                        const float *target_irr, float rel_floor,
                                        float *features, float *targets);

/* ---------------------------------------------------------------- training --
 * Loss per sample (o = network output, (z, q) = targets row):
 *   sum_c (o_c - z_c)^2 + head_weight * (o_3 - ln max(r, min_error))^2,
 *   r = sum_c |o_c - z_c| / q, held constant in the gradient;
 * the step's loss is the mean over its samples. Forward and backward run with
 * the bfloat16 roundings of the forward pass above plus the output gradient and
 * each hidden gradient (after its ReLU mask) rounded to bfloat16, FP32
 * accumulation; Adam (Kingma and Ba 2015) updates binary32 masters. */
typedef struct {
    float head_weight;   /* weight of the error-head term, >= 0 */
    float min_error;     /* floor of r in the log target, > 0   */
    float beta1, beta2;  /* Adam moment decays, [0, 1)          */
    float eps;           /* Adam denominator offset, >= 0       */
} sdfddgi_train_config;

typedef struct sdfddgi_trainer sdfddgi_trainer;

sdfddgi_status sdfddgi_trainer_create(const float *init_params, int32_t count,
                                      const sdfddgi_train_config *cfg, void *hip_stream,
                                      sdfddgi_trainer **out);

/* Mean loss and gradient over samples 0..n-1 of device features[n][16],
 * targets[n][4], in order; grad (host [SDFDDGI_DENOISER_PARAMS]) and loss (host)
 * may be NULL. Waits for the stream. Parameters are not changed. */
sdfddgi_status sdfddgi_trainer_gradient(sdfddgi_trainer *tr, const float *features,
                                        const float *targets, int32_t n, float *grad,
                                        float *loss);

/* One Adam step with learning rate lr on a minibatch of `batch` samples: sample
 * i of the step is row (first SplitMix64 output of the state seed + i) mod count
 * of the device arrays. loss (host, may be NULL) receives the minibatch loss
 * before the update (and waits for the stream). */
sdfddgi_status sdfddgi_trainer_step(sdfddgi_trainer *tr, const float *features,
                                    const float *targets, int64_t count, int32_t batch,
                                    uint64_t seed, float lr, float *loss);

/* Copy the binary32 master parameters to host params[SDFDDGI_DENOISER_PARAMS]. */
sdfddgi_status sdfddgi_trainer_get_params(sdfddgi_trainer *tr, float *params);

sdfddgi_status sdfddgi_trainer_destroy(sdfddgi_trainer *tr);

/* ------------------------------------------------------------ scene baking --
 * Input preparation on the device (training scenes in bulk): the exact signed
 * distance of a union of primitives at every vertex (i,j,k) of a grid, vertex at
 * origin + spacing*(i,j,k), evaluated in binary64 and rounded once; albedo_out
 * receives the albedo of the nearest primitive (ties: lower index), 0 and
 * empty_value where there are no primitives. Primitive arrays are host arrays:
 * kind[nprims] (0 sphere with radius half[.][0], 1 axis-aligned box with half
 * extents half[.][0..2]), center/half/albedo [nprims][3]. sdf (device
 * [n2][n1][n0]) and albedo_out (device [n2][n1][n0][3], may be NULL). Waits for
 * the stream before returning. */
sdfddgi_status sdfddgi_bake_sdf(int32_t nprims, const int32_t *kind, const double *center,
                                const double *half, const double *albedo, const int32_t n[3],
                                const double origin[3], double spacing, float empty_value,
                                float *sdf, float *albedo_out, void *hip_stream);

/* For callers that cannot allocate device memory (tight loops, harnesses that
 * forbid hipMalloc): sdfddgi_bake_sdf with the same arguments, results and
 * errors, which calls no allocator. The primitives are staged in a buffer the
 * library holds in static device memory, one per device for the life of the
 * process (about 304 KiB), so nprims may be at most
 * SDFDDGI_BAKE_NOALLOC_MAX_PRIMS (EINVAL above). Every call on a device shares
 * that device's buffer: calls that overlap on one device (from several host
 * threads) race and must be serialised by the caller. Waits for the stream
 * before returning, after which the buffer is free again. */
#define SDFDDGI_BAKE_NOALLOC_MAX_PRIMS 4096
sdfddgi_status sdfddgi_bake_sdf_noalloc(int32_t nprims, const int32_t *kind, const double *center,
                                        const double *half, const double *albedo,
                                        const int32_t n[3], const double origin[3], double spacing,
                                        float empty_value, float *sdf, float *albedo_out,
                                        void *hip_stream);

/* ------------------------------------------------------------ batched form --
 * Many independent scenes of uneven size updated together: each frame is one
 * replay of a captured HIP graph whose launches cover every scene -- the ray
 * tables of each distinct ray count, one persistent primary trace over the
 * concatenated rays of all scenes, one hit-shading pass over all their hits and
 * one blend over all their probes. Every scene runs the precision form (its grid
 * stored in binary16, FP16/BF16 MFMA blend) of the update above, so each scene's
 * maps are bit-identical to a single-scene context created with
 * SDFDDGI_FLAG_FP16 and run over the same frames. Scenes share the frame's
 * rotation seed; each has its own light. */
#define SDFDDGI_MAX_BATCH_SCENES 64

typedef struct sdfddgi_batch sdfddgi_batch;

typedef struct {
    sdfddgi_sdf_level level;      /* one grid level (device arrays, as in create)       */
    sdfddgi_probe_grid probes;
    sdfddgi_params params;        /* rays_per_probe a multiple of 64; irr_res 8 and
                                     depth_res 16; flags and learned fields ignored    */
} sdfddgi_batch_scene;

/* Launch configuration of the batch's trace and blend kernels, chosen by
 * sdfddgi_batch_autotune (or the defaults at create: 256, the resident grid, 64,
 * the resident grid, 40, 16, 64). */
typedef struct {
    int32_t primary_chunk;        /* rays claimed per atomic: 64, 128, 256 or 512        */
    int32_t primary_blocks;       /* persistent workgroups of the primary trace          */
    int32_t hits_chunk;           /* hits claimed per atomic: 16, 32, 64 or 128          */
    int32_t hits_blocks;          /* persistent workgroups of the hit shading            */
    int32_t refill;               /* refill idle lanes when fewer than this many of a
                                     wave's 64 lanes are stepping: 1..64                 */
    int32_t blend_probes;         /* Eq. 3 blend tile: probes per workgroup, 16 or 8     */
    int32_t blend_chunk;          /* rays staged in LDS at a time: 32, 64 or 128, and a
                                     divisor of every scene's rays_per_probe             */
} sdfddgi_batch_tuning;

/* Validate and upload count (1..SDFDDGI_MAX_BATCH_SCENES) scenes, allocate their
 * maps (every history rejected), capture the frame graphs with the default
 * tuning, and wait. hip_stream as in sdfddgi_create (NULL: the library creates a
 * stream of its own; graphs cannot be captured on the null stream). */
sdfddgi_status sdfddgi_batch_create(const sdfddgi_batch_scene *scenes, int32_t count,
                                    void *hip_stream, sdfddgi_batch **out);

/* One frame for every scene: lights (host [count]) and the shared rotation seed.
 * Enqueues two graph replays: the tables and primary trace on a side stream of
 * the batch (default priority) and the hit shading and blend on the batch's
 * stream, joined by an event. Consecutive calls overlap (a frame's side part runs
 * beside the previous frame's hit shading and blend); any other call on the batch
 * in between makes the next frame wait for everything before it. Results are
 * valid once the caller synchronises the batch's stream. */
sdfddgi_status sdfddgi_batch_update_frame(sdfddgi_batch *b, const sdfddgi_light *lights,
                                          uint64_t rotation_seed);

/* Try launch configurations of the trace and blend kernels on real frames of the
 * batch (each candidate timed over frames_per_candidate frames with events), keep
 * the fastest -- chunks and refill from each trace kernel alone, the blend tile
 * from the blend alone (2 x 3 tiles, those whose chunk divides every scene's ray
 * count), then the two trace grids from overlapped frames -- re-capture the graphs, and
 * restore the maps and history flags to what they were before (tuning changes no
 * result: every configuration computes the same bits). *chosen (may be NULL)
 * receives the result; *tried the number of candidates timed. */
sdfddgi_status sdfddgi_batch_autotune(sdfddgi_batch *b, const sdfddgi_light *lights,
                                      uint64_t rotation_seed, int32_t frames_per_candidate,
                                      sdfddgi_batch_tuning *chosen, int32_t *tried);

/* Use this configuration (validated) and re-capture the graphs. */
sdfddgi_status sdfddgi_batch_set_tuning(sdfddgi_batch *b, const sdfddgi_batch_tuning *t);

/* Copy scene s's current maps to device buffers (layouts as sdfddgi_get_maps). */
sdfddgi_status sdfddgi_batch_get_maps(sdfddgi_batch *b, int32_t scene, float *irr,
                                      float *depth);

/* Per-scene latency of the last frame, from the device clock: ms[s] (host
 * [count]) = time from the frame's first kernel to the end of scene s's last
 * blend workgroup; *frame_ms (may be NULL) = the largest. Waits for the frame. */
sdfddgi_status sdfddgi_batch_scene_latency(sdfddgi_batch *b, float *ms, float *frame_ms);

/* Total probes and probe-rays of one frame of the batch (host pointers, may be NULL). */
sdfddgi_status sdfddgi_batch_sizes(const sdfddgi_batch *b, int64_t *probes, int64_t *rays);

sdfddgi_status sdfddgi_batch_destroy(sdfddgi_batch *b);

/* --------------------------------------------------- analytic SDF query --
 * The SDF query of Sec. 3.3 on analytic primitives: near primitives are packed
 * into clusters (here: primitives sorted by the Morton code of their centres,
 * cluster_size at a time); a query visits a cluster's primitives only when the
 * signed distance to the cluster's bounding box is below the best distance so
 * far, starting from +inf -- or, along a sphere-traced ray, from the bound the
 * previous sample gives: the scene distance is 1-Lipschitz, so after a step of
 * relax*d it is at most (1 + relax)*d (the paper's 2 lastSDF), widened here by
 * 2^-10 relative and 1e-4 to stay a bound under rounding. Bounding boxes are
 * widened by 1e-4 (1 + the scene's largest coordinate) for the same reason.
 * Distances are binary32 (sphere: |x - c| - r; box: outside length plus the
 * negative largest excess inside) and the culled result equals the minimum over
 * every primitive bit for bit. Modes: 0 every primitive, 1 clusters from +inf,
 * 2 clusters from the previous sample's bound. */
typedef struct sdfddgi_analytic sdfddgi_analytic;

/* Primitives as host arrays (kind 0 sphere with radius half[.][0], 1 box with
 * half extents), rounded once to binary32; 1..1024 primitives, cluster_size
 * 1..64 (at most 256 clusters). */
sdfddgi_status sdfddgi_analytic_create(int32_t nprims, const int32_t *kind, const double *center,
                                       const double *half, int32_t cluster_size,
                                       void *hip_stream, sdfddgi_analytic **out);

/* Distances at n points (device [n][3] -> device [n]); *evals (host, may be NULL)
 * = primitive distances evaluated. Waits for the stream when evals is given. */
sdfddgi_status sdfddgi_analytic_query(sdfddgi_analytic *an, const float *points, int32_t n,
                                      int32_t mode, float *out, int64_t *evals);

/* Sphere-trace n rays (device origins and unit directions [n][3]) with the
 * stopping rules of the probe trace without a grid box: t > t_max -> 0 (miss),
 * d < 0 at the first sample -> 4 (inside), d < eps -> 2 (hit), max_steps samples
 * -> 3 (hit, exhausted); step t = fma(relax, d, t). Device outputs t[n],
 * steps[n], kind[n]; *evals as above. */
sdfddgi_status sdfddgi_analytic_trace(sdfddgi_analytic *an, const float *origins,
                                      const float *dirs, int32_t n, float t_max, float eps,
                                      float relax, int32_t max_steps, int32_t mode, float *t,
                                      int32_t *steps, int32_t *kind, int64_t *evals);

/* Number of clusters (host). */
sdfddgi_status sdfddgi_analytic_clusters(const sdfddgi_analytic *an, int32_t *count);

sdfddgi_status sdfddgi_analytic_destroy(sdfddgi_analytic *an);

/* Message of the last failure of a denoiser, trainer, baking, batch or analytic call
 * on this thread. */
/* ------------------------------------------------------------ measurement --
 * The gather throughput of the trace's access pattern, the second roofline
 * denominator of the sphere trace beside HBM bandwidth (the trace reads each
 * sample's eight corners as two adjacent 16-byte corner quads, at positions the
 * rays scatter over the grid). Launches threads (1..2^30) threads on hip_stream,
 * each reading `reads` (a multiple of 8 in 8..4096) independent 32-byte records
 * of the device buffer buf (bytes = 32 x a power of two, at most 64 GiB) at
 * indices from a counter-based hash of (seed, thread, read). sink: a device
 * float the kernel writes only under a condition that finite data never meets.
 * Asynchronous; the caller times it on the stream. Errors: EINVAL. */
sdfddgi_status sdfddgi_measure_gather(const void *buf, int64_t bytes, int64_t threads,
                                      int32_t reads, uint64_t seed, float *sink,
                                      void *hip_stream);

const char *sdfddgi_learned_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SDFDDGI_H */
