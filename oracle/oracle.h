/*
 * Reference checker for the SDFDDGI per-frame probe update (Hu et al.,
 * "Signed Distance Fields Dynamic Diffuse Global Illumination", Sec. 3.3).
 *
 * TEST INFRASTRUCTURE ONLY. This is a plain, slow, serial-per-ray CPU
 * implementation used by the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg to check the GPU library. The library never links, loads or
 * calls it, and it shares no code with the library.
 *
 * Precision policy. The geometry of a ray (which cascade level each sample
 * falls in, when a sphere-traced ray stops and why, how many steps it took,
 * the hit point and normal, whether a shadow ray is traced and whether it is
 * blocked) has two evaluations:
 *   - ORC_GEOMETRY_64, the reference: the trace written plainly in IEEE
 *     binary64 from its definition (sample x = o + t w, grid coordinate
 *     (x - origin) / spacing, trilinear interpolation, t += relax d). Each ray
 *     also reports its decision margin: the smallest distance, over every
 *     decision it took, between the decision value and its threshold.
 *   - ORC_GEOMETRY_32, the decision copy: IEEE binary32 following one fixed
 *     operation sequence, the precision and order in which the GPU kernels
 *     take their decisions. fmaf() marks every fused multiply-add of that
 *     sequence; everything else is a single correctly rounded binary32
 *     operation (compile with -ffp-contract=off). Its ray geometry can be
 *     given to the binary64 frame update for chosen rays, so that a ray whose
 *     binary64 decision sits within rounding of a threshold (or whose trace
 *     is ill-conditioned) can be compared with binary32 arithmetic that took
 *     the other branch.
 * Everything continuous downstream of the geometry (albedo, direct light,
 * the multi-bounce lookup, ray radiance, the Eq. 3 irradiance estimate,
 * depth moments and the temporal blend) is computed in binary64.
 *
 * Array layouts (all row-major, x fastest):
 *   SDF level       float [n2][n1][n0], vertex (i,j,k) at origin + spacing*(i,j,k)
 *   albedo level    float [n2][n1][n0][3]
 *   irradiance tile [res+2 rows (v)][res+2 cols (u)][3], interior at 1..res
 *   depth tile      [res+2][res+2][2]  (E[t], E[t^2])
 *   atlas           tiles of all probes, probe p = x + nx*(y + ny*z)
 */
#ifndef SDFDDGI_ORACLE_H
#define SDFDDGI_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_LEVELS 4

/* Ray outcome codes (low byte of a record's first word; level in bits 8..15). */
enum {
    ORC_MISS_TMAX = 0,      /* travelled past t_max                       */
    ORC_MISS_EXIT = 1,      /* left the outermost grid level              */
    ORC_HIT = 2,            /* distance fell below the hit epsilon        */
    ORC_HIT_EXHAUSTED = 3,  /* ran out of steps: hit at the last sample   */
    ORC_INSIDE = 4          /* primary ray started inside geometry        */
};

typedef struct {
    int32_t n[3];
    double origin[3];
    double spacing;
    const float *sdf;
    const float *albedo;  /* NULL: the constant albedo of the setup */
} orc_level;

/* Analytic scene (Sec. 3.1: the scene as a union of primitives; Sec. 3.3 queries
 * their distance): kind 0 sphere (radius half[.][0]), 1 axis-aligned box (half
 * extents). Distances in binary32 from the binary32 centre and half extents. */
typedef struct {
    int32_t count;
    const int32_t *kind;          /* [count] */
    const float *center;          /* [count][3] */
    const float *half;            /* [count][3] */
    const double *albedo;         /* [count][3] */
} orc_analytic_scene;

typedef struct {
    int32_t num_levels;           /* level 0 finest; levels are nested */
    orc_level level[ORC_MAX_LEVELS];
    int32_t probe_n[3];
    double probe_origin[3];
    double probe_spacing[3];
    int32_t rays;
    int32_t max_steps;
    int32_t irr_res;
    int32_t depth_res;
    float hit_eps;
    float t_max;
    float hysteresis;
    float bounce_gain;
    float depth_sharpness;
    float shadow_bias;
    float relax;
    float sky[3];
    float albedo[3];
    const float *probe_pos;       /* [P][3] relocated positions, or NULL: the grid */
    /* Non-NULL: the geometry comes from these primitives instead of the grid
     * levels (num_levels is ignored). The trace's sample distance is the
     * minimum over the primitives; there is no grid box, so a ray only misses
     * past t_max. At a hit the normal is the normalised gradient of the nearest
     * primitive (lowest index on a tie) and the albedo is that primitive's.
     * Only ORC_GEOMETRY_32 is provided for this mode. */
    const orc_analytic_scene *analytic;
} orc_setup;

typedef struct {
    float dir_to_light[3];
    float radiance[3];
    uint64_t rotation_seed;
    int32_t reset_history;  /* 1: no temporal blending this frame (M = U) */
} orc_frame;

/* ---- per-frame constants ---------------------------------------------- */
uint64_t orc_splitmix64(uint64_t *state);
void orc_frame_rotation(uint64_t seed, double q[9]);
void orc_ray_directions(uint64_t seed, int32_t rays, double *dirs /* [rays][3] */);
void orc_probe_position(const orc_setup *s, int32_t probe, double pos[3]);

/* Alg. 1 (UpdateProbePos) for probe p: from its grid position x, while the SDF
 * at x is below threshold1 (at most `iterations` times) step along the
 * normalised SDF gradient by threshold1 - SDF(x) (a Newton step on the distance
 * field), keeping each coordinate within max_offset * spacing of the grid
 * position; outside every level x is left as it is. All in binary32:
 *   x_c = min(max(fma(threshold1 - d, n_c, x_c), g_c - o_c), g_c + o_c)
 * with n the normal rule of the hit points (fallback +y when the gradient
 * vanishes) and o_c = (float)(max_offset * spacing_c). *reject = 1 when
 * |x - last|^2 = fma(dz, dz, fma(dy, dy, dx*dx)) > threshold2^2 (binary32). */
void orc_relocate_probe(const orc_setup *s, int32_t p, const float last[3], float threshold1,
                        float threshold2, int32_t iterations, float max_offset, float out[3],
                        int32_t *reject);

/* ---- octahedral parameterisation --------------------------------------- */
void orc_oct_encode(const double n[3], double uv[2]);
void orc_oct_decode(const double uv[2], double n[3]);
void orc_texel_direction(int32_t res, int32_t i, int32_t j, double n[3]);
void orc_border_source(int32_t res, int32_t a, int32_t b, int32_t *i, int32_t *j);

/* ---- binary32 geometry -------------------------------------------------- */
float orc_sdf32(const orc_setup *s, int32_t level, const float x[3]);
int32_t orc_level32(const orc_setup *s, const float x[3]);
/* record: [kind|level<<8, steps, visibility(1 lit, 0 blocked, -1 not traced),
 *          shadow steps, bits(t), bits(nx), bits(ny), bits(nz)] */
void orc_trace_ray32(const orc_setup *s, const float origin[3], const float dir[3],
                     const float dir_to_light[3], int32_t record[8]);

/* ---- binary64 geometry -------------------------------------------------- */
enum { ORC_GEOMETRY_32 = 0, ORC_GEOMETRY_64 = 1 };
/* record64: [kind, level (0 unless a hit), steps, visibility, shadow steps,
 *            t (t_max on a miss, 0 inside), nx, ny, nz,
 *            margin: smallest |decision value - threshold| over the ray's
 *                    decisions (scene units),
 *            tie ratio: smallest margin / error bound of a binary32
 *                    evaluation of that decision (below 1: a near-tie),
 *            bound on a binary32 evaluation's |t| error (hits; 0 otherwise),
 *            bound on its normal error (L-inf)]
 * The last four are -1 for rays whose geometry was given. */
#define ORC_RAY64_FIELDS 13
double orc_sdf64(const orc_setup *s, int32_t level, const double x[3]);
int32_t orc_level64(const orc_setup *s, const double x[3], double *margin);
void orc_trace_ray64(const orc_setup *s, const double origin[3], const double dir[3],
                     const double dir_to_light[3], double record[ORC_RAY64_FIELDS]);

/* ---- binary64 radiometry and blending ---------------------------------- */
void orc_interp_irradiance(const orc_setup *s, const double *irr_atlas, const double x[3],
                           const double n[3], double out[3]);
int32_t orc_blend_probe(const orc_setup *s, uint64_t rotation_seed, int32_t reset_history,
                        const double *payload /* [rays][4] */,
                        const double *prev_irr_tile, const double *prev_depth_tile,
                        double *irr_tile, double *depth_tile);
int32_t orc_update_probes(const orc_setup *s, const orc_frame *f,
                          const double *prev_irr, const double *prev_depth,
                          const int32_t *probes, int32_t count,
                          double *irr_tiles, double *depth_tiles,
                          double *payload /* [count][rays][4] or NULL */,
                          int32_t *records /* [count][rays][8] or NULL */,
                          int32_t threads);
/* The frame update with a choice of geometry. ORC_GEOMETRY_32 is
 * orc_update_probes. ORC_GEOMETRY_64 traces from the binary64 probe position
 * along the binary64 ray directions and light; given ([count][rays] or NULL)
 * marks rays whose geometry (outcome, level, steps, hit point and distance,
 * normal, shadow result) is taken from the binary32 sequence instead, with
 * everything downstream (shading, Eq. 3, blend) still in binary64; rays64
 * ([count][rays][ORC_RAY64_FIELDS] or NULL) receives the records; records is
 * ignored. */
int32_t orc_update_probes_ex(const orc_setup *s, const orc_frame *f, const double *prev_irr,
                             const double *prev_depth, const int32_t *probes, int32_t count,
                             double *irr_tiles, double *depth_tiles, double *payload,
                             int32_t *records, int32_t geometry, const uint8_t *given,
                             double *rays64, int32_t threads);

#ifdef __cplusplus
}
#endif
#endif
