/*
 * Reference checker for the SDFDDGI per-frame probe update.
 * TEST INFRASTRUCTURE ONLY: see oracle.h for the precision policy and layouts.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
 * this file; it shares no code with the GPU library.
 *
 * What it computes, step by step (paper Sec. 3.3, Probe update):
 *   1. per frame, one random rotation of a spherical-Fibonacci direction set
 *      (the paper's random low-discrepancy ray directions);
 *   2. per probe and ray, a sphere trace through the baked distance grid
 *      (the paper's sphere tracing of probe rays);
 *   3. at a hit, the radiance leaving the hit point: albedo/pi times the sum
 *      of the direct sun term, seen through an SDF shadow ray, and the previous
 *      frame's probe irradiance scaled by the multi-bounce coefficient (the
 *      paper's hit shading and its reuse of last frame's probes for
 *      multi-bounce);
 *   4. per texel direction D of the octahedral map, Eq. 3's irradiance
 *      E(D) = integral of max(0, cos(D, D')) L(D') dD' estimated from the ray
 *      samples, plus the depth moments of the ray distances;
 *   5. the temporal mix of new and old values (the paper's temporal mixing),
 *      skipped when the probe's history is rejected (Alg. 1's
 *      markRejectHistory);
 *   6. the octahedral tile's one-texel border.
 */
#define _GNU_SOURCE
#include "oracle.h"
#include "cluster.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

static const double kPi = 3.14159265358979323846;

/* ======================================================================== */
/* Per-frame constants                                                       */
/* ======================================================================== */

/* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): a Weyl sequence with increment 0x9E3779B97F4A7C15
 * followed by a 64-bit finaliser. */
uint64_t orc_splitmix64(uint64_t *state)
{
    *state += 0x9E3779B97F4A7C15ull;
    uint64_t z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double unit_double(uint64_t *state)
{
    return (double)(orc_splitmix64(state) >> 11) * 0x1.0p-53;
}

/* One uniformly random rotation per frame (Shoemake, "Uniform random
 * rotations", Graphics Gems III, 1992): three uniforms u1,u2,u3 give the unit
 * quaternion (x,y,z,w) = (sqrt(1-u1) sin 2pi u2, sqrt(1-u1) cos 2pi u2,
 * sqrt(u1) sin 2pi u3, sqrt(u1) cos 2pi u3), turned into a row-major matrix. */
void orc_frame_rotation(uint64_t seed, double q[9])
{
    uint64_t st = seed;
    double u1 = unit_double(&st);
    double u2 = unit_double(&st);
    double u3 = unit_double(&st);
    double two_pi = 2.0 * kPi;
    double r1 = sqrt(1.0 - u1);
    double r2 = sqrt(u1);
    double t1 = two_pi * u2;
    double t2 = two_pi * u3;
    double x = r1 * sin(t1), y = r1 * cos(t1);
    double z = r2 * sin(t2), w = r2 * cos(t2);
    q[0] = 1.0 - 2.0 * (y * y + z * z);
    q[1] = 2.0 * (x * y - z * w);
    q[2] = 2.0 * (x * z + y * w);
    q[3] = 2.0 * (x * y + z * w);
    q[4] = 1.0 - 2.0 * (x * x + z * z);
    q[5] = 2.0 * (y * z - x * w);
    q[6] = 2.0 * (x * z - y * w);
    q[7] = 2.0 * (y * z + x * w);
    q[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Ray i of R: the spherical-Fibonacci point z = 1 - (2i+1)/R,
 * phi = 2 pi frac(i * gamma) with gamma = (sqrt 5 - 1)/2, rotated by the
 * frame's rotation (Sec. 3.3: random low-discrepancy directions). */
void orc_ray_directions(uint64_t seed, int32_t rays, double *dirs)
{
    double q[9];
    orc_frame_rotation(seed, q);
    double gamma = (sqrt(5.0) - 1.0) * 0.5;
    double two_pi = 2.0 * kPi;
    for (int32_t i = 0; i < rays; ++i) {
        double z = 1.0 - (2.0 * (double)i + 1.0) / (double)rays;
        double r = sqrt(1.0 - z * z);
        double g = (double)i * gamma;
        double phi = two_pi * (g - floor(g));
        double s0 = r * cos(phi), s1 = r * sin(phi), s2 = z;
        for (int a = 0; a < 3; ++a)
            dirs[3 * i + a] = q[3 * a + 0] * s0 + q[3 * a + 1] * s1 + q[3 * a + 2] * s2;
    }
}

/* Probe p = x + nx*(y + ny*z) sits on the uniform grid (Sec. 3.2). */
void orc_probe_position(const orc_setup *s, int32_t p, double pos[3])
{
    if (s->probe_pos) {
        for (int c = 0; c < 3; ++c) pos[c] = (double)s->probe_pos[3 * p + c];
        return;
    }
    int32_t idx[3];
    idx[0] = p % s->probe_n[0];
    idx[1] = (p / s->probe_n[0]) % s->probe_n[1];
    idx[2] = p / (s->probe_n[0] * s->probe_n[1]);
    for (int c = 0; c < 3; ++c)
        pos[c] = s->probe_origin[c] + s->probe_spacing[c] * (double)idx[c];
}

/* ======================================================================== */
/* Octahedral parameterisation (Sec. 3.3 stores each probe's directions in   */
/* an octahedral map, after Cigolle et al. 2014).                            */
/* ======================================================================== */

static double sgn(double v) { return v >= 0.0 ? 1.0 : -1.0; }

void orc_oct_encode(const double n[3], double uv[2])
{
    double l1 = fabs(n[0]) + fabs(n[1]) + fabs(n[2]);
    double u = n[0] / l1, v = n[1] / l1;
    if (n[2] < 0.0) {
        double fu = (1.0 - fabs(v)) * sgn(u);
        double fv = (1.0 - fabs(u)) * sgn(v);
        u = fu;
        v = fv;
    }
    uv[0] = u;
    uv[1] = v;
}

void orc_oct_decode(const double uv[2], double n[3])
{
    double x = uv[0], y = uv[1];
    double z = 1.0 - fabs(x) - fabs(y);
    if (z < 0.0) {
        double fx = (1.0 - fabs(y)) * sgn(x);
        double fy = (1.0 - fabs(x)) * sgn(y);
        x = fx;
        y = fy;
    }
    double len = sqrt(x * x + y * y + z * z);
    n[0] = x / len;
    n[1] = y / len;
    n[2] = z / len;
}

/* Interior texel (i = column along u, j = row along v) has its centre at
 * ((i + 1/2)/res * 2 - 1, (j + 1/2)/res * 2 - 1). */
void orc_texel_direction(int32_t res, int32_t i, int32_t j, double n[3])
{
    double uv[2];
    uv[0] = ((double)i + 0.5) / (double)res * 2.0 - 1.0;
    uv[1] = ((double)j + 0.5) / (double)res * 2.0 - 1.0;
    orc_oct_decode(uv, n);
}

/* Padded texel (a = column, b = row, both 0..res+1) -> interior source
 * (i, j). Crossing an edge of the octahedral square lands on the same edge
 * reflected about its midpoint; the four corners all meet at the -z pole and
 * take the diagonally opposite interior corner. */
void orc_border_source(int32_t res, int32_t a, int32_t b, int32_t *i, int32_t *j)
{
    int32_t n = res;
    int left = a == 0, right = a == n + 1, top = b == 0, bottom = b == n + 1;
    if ((left || right) && (top || bottom)) {
        *i = left ? n - 1 : 0;
        *j = top ? n - 1 : 0;
    } else if (top || bottom) {
        *i = n - a;
        *j = top ? 0 : n - 1;
    } else if (left || right) {
        *i = left ? 0 : n - 1;
        *j = n - b;
    } else {
        *i = a - 1;
        *j = b - 1;
    }
}

/* ======================================================================== */
/* Geometry in binary32: the integer decisions of the trace.                 */
/* ======================================================================== */

typedef struct {
    float org[3];
    float inv;   /* (float)(1 / spacing) */
    float half;  /* (float)(spacing / 2): central-difference offset */
} lvl32;

static void level_constants(const orc_level *L, lvl32 *g)
{
    for (int c = 0; c < 3; ++c) g->org[c] = (float)L->origin[c];
    g->inv = (float)(1.0 / L->spacing);
    g->half = (float)(0.5 * L->spacing);
}

/* Trilinear interpolation at grid coordinate u of a vertex-centred grid; the
 * cell is clamped to the grid and the fraction to [0,1]. */
static float trilinear32(const float *grid, const int32_t n[3], const float u[3])
{
    int32_t i[3];
    float f[3];
    for (int c = 0; c < 3; ++c) {
        float fl = floorf(u[c]);
        fl = fminf(fmaxf(fl, 0.0f), (float)(n[c] - 2));
        i[c] = (int32_t)fl;
        f[c] = fminf(fmaxf(u[c] - fl, 0.0f), 1.0f);
    }
    size_t sx = 1, sy = (size_t)n[0], sz = (size_t)n[0] * (size_t)n[1];
    const float *g = grid + (size_t)i[2] * sz + (size_t)i[1] * sy + (size_t)i[0];
    float v000 = g[0], v100 = g[sx], v010 = g[sy], v110 = g[sy + sx];
    float v001 = g[sz], v101 = g[sz + sx], v011 = g[sz + sy], v111 = g[sz + sy + sx];
    float c00 = fmaf(f[0], v100 - v000, v000);
    float c10 = fmaf(f[0], v110 - v010, v010);
    float c01 = fmaf(f[0], v101 - v001, v001);
    float c11 = fmaf(f[0], v111 - v011, v011);
    float c0 = fmaf(f[1], c10 - c00, c00);
    float c1 = fmaf(f[1], c11 - c01, c01);
    return fmaf(f[2], c1 - c0, c0);
}

static void grid_coord32(const lvl32 *g, const float x[3], float u[3])
{
    for (int c = 0; c < 3; ++c) u[c] = (x[c] - g->org[c]) * g->inv;
}

float orc_sdf32(const orc_setup *s, int32_t level, const float x[3])
{
    lvl32 g;
    level_constants(&s->level[level], &g);
    float u[3];
    grid_coord32(&g, x, u);
    return trilinear32(s->level[level].sdf, s->level[level].n, u);
}

/* The finest level whose box, shrunk by one voxel, holds x; the coarsest level
 * counts with its full box. -1 when x is outside the coarsest box. */
int32_t orc_level32(const orc_setup *s, const float x[3])
{
    for (int32_t L = 0; L < s->num_levels; ++L) {
        lvl32 g;
        level_constants(&s->level[L], &g);
        int inner = L < s->num_levels - 1;
        int ok = 1;
        for (int c = 0; c < 3; ++c) {
            float u = (x[c] - g.org[c]) * g.inv;
            float lo = inner ? 1.0f : 0.0f;
            float hi = (float)(s->level[L].n[c] - (inner ? 2 : 1));
            if (!(u >= lo && u <= hi)) ok = 0;
        }
        if (ok) return L;
    }
    return -1;
}

typedef struct {
    int32_t kind, steps, level;
    float t;
    float x[3];
} trace32_result;

/* Sphere tracing (Hart 1996, as used in Sec. 3.3): step along the ray by the
 * distance bound until it falls under the hit epsilon, the ray passes t_max or
 * leaves the grid, or the step budget runs out (then: a hit at the last
 * sample). A primary ray whose first sample is inside geometry reports
 * "inside". */
static trace32_result trace32(const orc_setup *s, const float o[3], const float w[3],
                              int primary)
{
    trace32_result r = {ORC_HIT_EXHAUSTED, s->max_steps, -1, 0.0f, {0.0f, 0.0f, 0.0f}};
    float t = 0.0f;
    for (int32_t k = 0; k < s->max_steps; ++k) {
        if (t > s->t_max) {
            r.kind = ORC_MISS_TMAX;
            r.steps = k;
            return r;
        }
        float x[3];
        for (int c = 0; c < 3; ++c) x[c] = fmaf(t, w[c], o[c]);
        int32_t L = orc_level32(s, x);
        if (L < 0) {
            r.kind = ORC_MISS_EXIT;
            r.steps = k;
            return r;
        }
        float d = orc_sdf32(s, L, x);
        r.t = t;
        r.level = L;
        memcpy(r.x, x, sizeof x);
        if (primary && k == 0 && d < 0.0f) {
            r.kind = ORC_INSIDE;
            r.steps = 1;
            return r;
        }
        if (d < s->hit_eps) {
            r.kind = ORC_HIT;
            r.steps = k + 1;
            return r;
        }
        t = fmaf(s->relax, d, t);
    }
    return r; /* exhausted: hit at the last sample */
}

/* Surface normal from central differences of the grid the hit was found on,
 * offset half a voxel; a vanishing gradient falls back to facing the ray. */
static void normal32(const orc_setup *s, int32_t level, const float x[3], const float w[3],
                     float n[3])
{
    lvl32 g;
    level_constants(&s->level[level], &g);
    float grad[3];
    for (int c = 0; c < 3; ++c) {
        float xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
        xp[c] = x[c] + g.half;
        xm[c] = x[c] - g.half;
        float up[3], um[3];
        grid_coord32(&g, xp, up);
        grid_coord32(&g, xm, um);
        grad[c] = trilinear32(s->level[level].sdf, s->level[level].n, up) -
                  trilinear32(s->level[level].sdf, s->level[level].n, um);
    }
    float len2 = fmaf(grad[2], grad[2], fmaf(grad[1], grad[1], grad[0] * grad[0]));
    if (!(len2 >= 1e-24f)) {
        for (int c = 0; c < 3; ++c) n[c] = -w[c];
        return;
    }
    float inv = 1.0f / sqrtf(len2);
    for (int c = 0; c < 3; ++c) n[c] = grad[c] * inv;
}

/* Alg. 1: move a probe that is too close to (or inside) geometry out along the
 * distance field's gradient; reject its history if it moved too far. */
void orc_relocate_probe(const orc_setup *s, int32_t p, const float last[3], float threshold1,
                        float threshold2, int32_t iterations, float max_offset, float out[3],
                        int32_t *reject)
{
    int32_t idx[3];
    idx[0] = p % s->probe_n[0];
    idx[1] = (p / s->probe_n[0]) % s->probe_n[1];
    idx[2] = p / (s->probe_n[0] * s->probe_n[1]);
    float g[3], o[3], x[3];
    for (int c = 0; c < 3; ++c) {
        g[c] = (float)(s->probe_origin[c] + s->probe_spacing[c] * (double)idx[c]);
        o[c] = (float)((double)max_offset * s->probe_spacing[c]);
        x[c] = g[c];
    }
    const float down[3] = {0.0f, -1.0f, 0.0f};   /* normal fallback -down = +y */
    for (int32_t it = 0; it < iterations; ++it) {
        int32_t L = orc_level32(s, x);
        if (L < 0) break;
        float d = orc_sdf32(s, L, x);
        if (!(d < threshold1)) break;
        float n[3];
        normal32(s, L, x, down, n);
        float step = threshold1 - d;
        for (int c = 0; c < 3; ++c) {
            float v = fmaf(step, n[c], x[c]);
            float lo = g[c] - o[c], hi = g[c] + o[c];
            x[c] = v < lo ? lo : (v > hi ? hi : v);
        }
    }
    float dx = x[0] - last[0], dy = x[1] - last[1], dz = x[2] - last[2];
    float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    *reject = d2 > threshold2 * threshold2 ? 1 : 0;
    for (int c = 0; c < 3; ++c) out[c] = x[c];
}

typedef struct {
    trace32_result prim;
    int32_t nearest;        /* analytic scenes: the nearest primitive at the hit */
    float n[3];
    int32_t visibility;     /* 1 lit, 0 blocked, -1 not traced */
    int32_t shadow_steps;
} ray32;

static int is_hit(int32_t kind) { return kind == ORC_HIT || kind == ORC_HIT_EXHAUSTED; }

/* ---- analytic scenes ----------------------------------------------------- */

/* The scene distance at x: the smallest primitive distance; *nearest receives
 * the primitive that gives it (the lowest index on a tie). */
static float analytic_distance32(const orc_analytic_scene *a, const float x[3],
                                 int32_t *nearest)
{
    float best = INFINITY;
    int32_t arg = -1;
    for (int32_t m = 0; m < a->count; ++m) {
        float d = orc_prim_distance32(a->kind[m], a->center + 3 * m, a->half + 3 * m, x);
        if (d < best) {
            best = d;
            arg = m;
        }
    }
    *nearest = arg;
    return best;
}

/* The same sphere trace as trace32 on the primitives' distance; no grid box, so
 * a ray misses only past t_max. */
static trace32_result trace_analytic32(const orc_setup *s, const float o[3], const float w[3],
                                       int primary, int32_t *nearest)
{
    trace32_result r = {ORC_HIT_EXHAUSTED, s->max_steps, 0, 0.0f, {0.0f, 0.0f, 0.0f}};
    float tt = 0.0f;
    *nearest = -1;
    for (int32_t k = 0; k < s->max_steps; ++k) {
        if (tt > s->t_max) {
            r.kind = ORC_MISS_TMAX;
            r.steps = k;
            return r;
        }
        float x[3];
        for (int c = 0; c < 3; ++c) x[c] = fmaf(tt, w[c], o[c]);
        float dist = analytic_distance32(s->analytic, x, nearest);
        r.t = tt;
        memcpy(r.x, x, sizeof x);
        if (primary && k == 0 && dist < 0.0f) {
            r.kind = ORC_INSIDE;
            r.steps = 1;
            return r;
        }
        if (dist < s->hit_eps) {
            r.kind = ORC_HIT;
            r.steps = k + 1;
            return r;
        }
        tt = fmaf(s->relax, dist, tt);
    }
    return r;
}

/* Normal at x from the gradient of primitive m's distance: a sphere's radial
 * direction x - c; outside a box the offset from its nearest point, inside it the
 * signed axis of the face nearest to x (the largest q, lowest axis on a tie);
 * normalised as the grid normal, -w when the gradient vanishes. */
static void normal_analytic32(const orc_analytic_scene *a, int32_t m, const float x[3],
                              const float w[3], float n[3])
{
    const float *c = a->center + 3 * m, *h = a->half + 3 * m;
    float d[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    float g[3] = {0.0f, 0.0f, 0.0f};
    if (a->kind[m] == 0) {
        for (int k = 0; k < 3; ++k) g[k] = d[k];
    } else {
        float q[3];
        for (int k = 0; k < 3; ++k) q[k] = fabsf(d[k]) - h[k];
        float qm = fmaxf(q[0], fmaxf(q[1], q[2]));
        if (qm > 0.0f) {
            for (int k = 0; k < 3; ++k) {
                float o = fmaxf(q[k], 0.0f);
                g[k] = d[k] >= 0.0f ? o : -o;
            }
        } else {
            int ax = q[0] >= q[1] ? (q[0] >= q[2] ? 0 : 2) : (q[1] >= q[2] ? 1 : 2);
            g[ax] = d[ax] >= 0.0f ? 1.0f : -1.0f;
        }
    }
    float len2 = fmaf(g[2], g[2], fmaf(g[1], g[1], g[0] * g[0]));
    if (!(len2 >= 1e-24f)) {
        for (int k = 0; k < 3; ++k) n[k] = -w[k];
        return;
    }
    float inv = 1.0f / sqrtf(len2);
    for (int k = 0; k < 3; ++k) n[k] = g[k] * inv;
}

/* Primary trace, hit normal and the SDF shadow ray toward the light. The
 * shadow ray starts at x + bias*n, is traced only where n.l > 0, and counts as
 * blocked on a hit or on running out of steps. */
static ray32 ray_geometry32(const orc_setup *s, const float o[3], const float w[3],
                            const float l[3])
{
    ray32 g;
    memset(&g, 0, sizeof g);
    g.nearest = -1;
    if (s->analytic)
        g.prim = trace_analytic32(s, o, w, 1, &g.nearest);
    else
        g.prim = trace32(s, o, w, 1);
    g.visibility = -1;
    if (!is_hit(g.prim.kind)) return g;
    if (s->analytic)
        normal_analytic32(s->analytic, g.nearest, g.prim.x, w, g.n);
    else
        normal32(s, g.prim.level, g.prim.x, w, g.n);
    float ndl = fmaf(g.n[2], l[2], fmaf(g.n[1], l[1], g.n[0] * l[0]));
    if (ndl > 0.0f) {
        float xs[3];
        for (int c = 0; c < 3; ++c) xs[c] = fmaf(g.n[c], s->shadow_bias, g.prim.x[c]);
        if (s->analytic) {
            int32_t unused;
            trace32_result sa = trace_analytic32(s, xs, l, 0, &unused);
            g.visibility = is_hit(sa.kind) ? 0 : 1;
            g.shadow_steps = sa.steps;
            return g;
        }
        trace32_result sh = trace32(s, xs, l, 0);
        g.visibility = is_hit(sh.kind) ? 0 : 1;
        g.shadow_steps = sh.steps;
    }
    return g;
}

static int32_t bits_of(float v)
{
    int32_t b;
    memcpy(&b, &v, sizeof b);
    return b;
}

static void fill_record(const orc_setup *s, const ray32 *g, int32_t rec[8])
{
    float t = g->prim.t;
    if (g->prim.kind == ORC_MISS_TMAX || g->prim.kind == ORC_MISS_EXIT) t = s->t_max;
    if (g->prim.kind == ORC_INSIDE) t = 0.0f;
    int32_t lev = is_hit(g->prim.kind) ? g->prim.level : 0;
    rec[0] = g->prim.kind | (lev << 8);
    rec[1] = g->prim.steps;
    rec[2] = g->visibility;
    rec[3] = g->shadow_steps;
    rec[4] = bits_of(t);
    rec[5] = bits_of(g->n[0]);
    rec[6] = bits_of(g->n[1]);
    rec[7] = bits_of(g->n[2]);
}

static void light_direction(const float in[3], double l64[3], float l32[3])
{
    double d0 = in[0], d1 = in[1], d2 = in[2];
    double len = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    l64[0] = d0 / len;
    l64[1] = d1 / len;
    l64[2] = d2 / len;
    for (int c = 0; c < 3; ++c) l32[c] = (float)l64[c];
}

void orc_trace_ray32(const orc_setup *s, const float origin[3], const float dir[3],
                     const float dir_to_light[3], int32_t record[8])
{
    double l64[3];
    float l32[3];
    light_direction(dir_to_light, l64, l32);
    ray32 g = ray_geometry32(s, origin, dir, l32);
    fill_record(s, &g, record);
}

/* ======================================================================== */
/* Radiometry in binary64                                                    */
/* ======================================================================== */

static double trilinear64(const float *grid, int32_t comps, int32_t comp, const int32_t n[3],
                          const double u[3])
{
    int32_t i[3];
    double f[3];
    for (int c = 0; c < 3; ++c) {
        double fl = floor(u[c]);
        if (fl < 0.0) fl = 0.0;
        if (fl > (double)(n[c] - 2)) fl = (double)(n[c] - 2);
        i[c] = (int32_t)fl;
        double fr = u[c] - fl;
        f[c] = fr < 0.0 ? 0.0 : (fr > 1.0 ? 1.0 : fr);
    }
    double acc = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                size_t v = ((size_t)(i[2] + dz) * n[1] + (size_t)(i[1] + dy)) * n[0] +
                           (size_t)(i[0] + dx);
                double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *
                           (dz ? f[2] : 1.0 - f[2]);
                acc += w * (double)grid[v * comps + comp];
            }
    return acc;
}

/* ======================================================================== */
/* Geometry in binary64: the trace written plainly from its definition.      */
/* ======================================================================== */

/* Whether x lies in level L's box (shrunk by one voxel unless L is the
 * coarsest level), and how far x is from changing that answer: the smallest
 * slack to a face when inside, the largest excess over a face (the L-inf
 * distance to the box) when outside. */
static int in_level_box64(const orc_setup *s, int32_t L, const double x[3], double *margin)
{
    const orc_level *lv = &s->level[L];
    double shrink = L < s->num_levels - 1 ? 1.0 : 0.0;
    double slack = INFINITY, excess = 0.0;
    int inside = 1;
    for (int c = 0; c < 3; ++c) {
        double lo = lv->origin[c] + lv->spacing * shrink;
        double hi = lv->origin[c] + lv->spacing * ((double)(lv->n[c] - 1) - shrink);
        double a = x[c] - lo, b = hi - x[c];
        if (a < 0.0 || b < 0.0) {
            inside = 0;
            double e = a < 0.0 ? -a : -b;
            if (e > excess) excess = e;
        } else {
            double m = a < b ? a : b;
            if (m < slack) slack = m;
        }
    }
    *margin = inside ? slack : excess;
    return inside;
}

/* The finest level holding x (-1 outside the coarsest box); *margin is the
 * smallest margin of the box tests that chose it. */
static int32_t level64(const orc_setup *s, const double x[3], double *margin)
{
    double m = INFINITY;
    for (int32_t L = 0; L < s->num_levels; ++L) {
        double mL;
        int in = in_level_box64(s, L, x, &mL);
        if (mL < m) m = mL;
        if (in) {
            *margin = m;
            return L;
        }
    }
    *margin = m;
    return -1;
}

/* Trilinear distance of level L at x; grid coordinate (x - origin) / spacing. */
static double sdf64(const orc_setup *s, int32_t L, const double x[3])
{
    const orc_level *lv = &s->level[L];
    double u[3];
    for (int c = 0; c < 3; ++c) u[c] = (x[c] - lv->origin[c]) / lv->spacing;
    return trilinear64(lv->sdf, 1, 0, lv->n, u);
}

/* ---- forward error bounds of the binary32 evaluation -------------------- */
/*
 * To tell a legitimate disagreement from a wrong one, each binary64 ray also
 * carries a first-order bound on how far a binary32 evaluation of the same
 * trace (unit roundoff u = 2^-24; one rounding per operation, the sequence of
 * the decision copy) can drift from it, as long as both take the same
 * decisions. With e_k = t~_k - t_k and g_k the gradient of the interpolated
 * distance at sample k (scene units):
 *   sample point  x~_k - x_k = e_k w + p_k,
 *                 |p_k| <= o_err + t_k w_err + u (|x_k| + 3 |x_k - origin_L|)
 *                 (rounded direction and origin, the fma, and the grid
 *                 coordinate's subtraction, product and rounded 1/spacing)
 *   distance      |d~_k - d_k| <= |g_k.w| |e_k| + |g_k|_1 |p_k| + 8 u (|d_k| + 2 spacing_L)
 *                 (the position error, and the seven lerps' roundings of corner
 *                 values no larger than |d_k| + 2 spacing)
 *   step          |e_k+1| <= |1 + relax g_k.w| |e_k| + relax (|g_k|_1 |p_k| + 8 u (...))
 *                            + u t_k+1
 * (all norms L-inf unless marked). Every decision then has an error bound:
 * |e_k| for t > t_max, |e_k| + |p_k| for the level boxes, the distance bound
 * for the inside and hit tests. The ratio margin / bound, minimised over the
 * ray's decisions, is its tie ratio: below 1 the binary32 evaluation may take
 * the other branch. The hit normal's bound follows from the same position
 * error at its six samples. First-order: the gradient is taken at the
 * binary64 point, so users of the bounds allow a small factor.
 */
static const double kU32 = 0x1.0p-24;

static double max_abs3(const double v[3])
{
    double m = fabs(v[0]);
    if (fabs(v[1]) > m) m = fabs(v[1]);
    if (fabs(v[2]) > m) m = fabs(v[2]);
    return m;
}

/* Gradient (scene units) of level L's trilinear interpolant at x, as the
 * derivative of the same cell's polynomial (zero along an axis whose
 * fraction is clamped). */
static void sdf64_gradient(const orc_setup *s, int32_t L, const double x[3], double g[3])
{
    const orc_level *lv = &s->level[L];
    int32_t i[3];
    double f[3];
    int clamped[3];
    for (int c = 0; c < 3; ++c) {
        double u = (x[c] - lv->origin[c]) / lv->spacing;
        double fl = floor(u);
        if (fl < 0.0) fl = 0.0;
        if (fl > (double)(lv->n[c] - 2)) fl = (double)(lv->n[c] - 2);
        i[c] = (int32_t)fl;
        double fr = u - fl;
        clamped[c] = fr < 0.0 || fr > 1.0;
        f[c] = fr < 0.0 ? 0.0 : (fr > 1.0 ? 1.0 : fr);
    }
    double v[2][2][2];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                v[dz][dy][dx] = (double)lv->sdf[((size_t)(i[2] + dz) * lv->n[1] +
                                                 (size_t)(i[1] + dy)) * lv->n[0] +
                                                (size_t)(i[0] + dx)];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double wa_y = a ? f[1] : 1.0 - f[1], wb_z = b ? f[2] : 1.0 - f[2];
            double wa_x = a ? f[0] : 1.0 - f[0], wb_y = b ? f[1] : 1.0 - f[1];
            gx += wa_y * wb_z * (v[b][a][1] - v[b][a][0]);
            gy += wa_x * wb_z * (v[b][1][a] - v[b][0][a]);
            gz += wa_x * wb_y * (v[1][b][a] - v[0][b][a]);
        }
    g[0] = clamped[0] ? 0.0 : gx / lv->spacing;
    g[1] = clamped[1] ? 0.0 : gy / lv->spacing;
    g[2] = clamped[2] ? 0.0 : gz / lv->spacing;
}

/* Bound on the non-t part p of a binary32 sample point's error at x. */
static double point_error(const orc_setup *s, int32_t L, const double x[3], double t,
                          double o_err, double w_err)
{
    double rel[3];
    for (int c = 0; c < 3; ++c) rel[c] = x[c] - s->level[L].origin[c];
    return o_err + t * w_err + kU32 * (max_abs3(x) + 3.0 * max_abs3(rel));
}

static double sum_abs3(const double v[3]) { return fabs(v[0]) + fabs(v[1]) + fabs(v[2]); }

typedef struct {
    int32_t kind, steps, level;
    double t, x[3];
    double margin;     /* smallest |decision value - threshold|, scene units */
    double tie;        /* smallest margin / binary32 error bound of that decision */
    double t_err;      /* bound on |t32 - t| at the last sample */
    double x_err;      /* bound on the last sample point's error (L-inf) */
} trace64_result;

static void min_into(double *m, double v)
{
    if (v < *m) *m = v;
}

static void decision(trace64_result *r, double margin, double err)
{
    min_into(&r->margin, margin);
    min_into(&r->tie, err > 0.0 ? margin / err : INFINITY);
}

/* Sphere tracing in binary64 with the same stopping rules as the binary32
 * sequence (t past t_max, outside the coarsest box, inside at the first
 * sample of a probe ray, distance below the hit epsilon, step budget spent).
 * o_err, w_err: bounds on the binary32 origin's and direction's rounding. */
static trace64_result trace64(const orc_setup *s, const double o[3], const double w[3],
                              int primary, double o_err, double w_err)
{
    trace64_result r = {ORC_HIT_EXHAUSTED, s->max_steps, -1, 0.0, {0.0, 0.0, 0.0},
                        INFINITY, INFINITY, 0.0, 0.0};
    const double t_max = (double)s->t_max, eps = (double)s->hit_eps, relax = (double)s->relax;
    double t = 0.0, e = 0.0;
    for (int32_t k = 0; k < s->max_steps; ++k) {
        decision(&r, fabs(t - t_max), e + kU32 * t);
        if (t > t_max) {
            r.kind = ORC_MISS_TMAX;
            r.steps = k;
            return r;
        }
        double x[3], mL;
        for (int c = 0; c < 3; ++c) x[c] = o[c] + t * w[c];
        int32_t L = level64(s, x, &mL);
        int32_t Lb = L >= 0 ? L : s->num_levels - 1;
        double pk = point_error(s, Lb, x, t, o_err, w_err);
        decision(&r, mL, e * max_abs3(w) + pk);
        if (L < 0) {
            r.kind = ORC_MISS_EXIT;
            r.steps = k;
            return r;
        }
        double d = sdf64(s, L, x), g[3];
        sdf64_gradient(s, L, x, g);
        double gw = g[0] * w[0] + g[1] * w[1] + g[2] * w[2];
        double tri = 8.0 * kU32 * (fabs(d) + 2.0 * s->level[L].spacing);
        double derr = fabs(gw) * e + sum_abs3(g) * pk + tri;
        r.t = t;
        r.level = L;
        memcpy(r.x, x, sizeof x);
        r.t_err = e;
        r.x_err = e * max_abs3(w) + pk;
        if (primary && k == 0) {
            decision(&r, fabs(d), derr);
            if (d < 0.0) {
                r.kind = ORC_INSIDE;
                r.steps = 1;
                return r;
            }
        }
        decision(&r, fabs(d - eps), derr);
        if (d < eps) {
            r.kind = ORC_HIT;
            r.steps = k + 1;
            return r;
        }
        t += relax * d;
        e = fabs(1.0 + relax * gw) * e + relax * (sum_abs3(g) * pk + tri) + kU32 * t;
    }
    return r;
}

/* Normalised central differences at +-spacing/2 on level L; -w when the
 * difference vector vanishes (returns 1 then). */
static int normal64(const orc_setup *s, int32_t L, const double x[3], const double w[3],
                    double n[3])
{
    double h = 0.5 * s->level[L].spacing, g[3];
    for (int c = 0; c < 3; ++c) {
        double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
        xp[c] += h;
        xm[c] -= h;
        g[c] = sdf64(s, L, xp) - sdf64(s, L, xm);
    }
    double len2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    if (!(len2 >= 1e-24)) {
        for (int c = 0; c < 3; ++c) n[c] = -w[c];
        return 1;
    }
    double len = sqrt(len2);
    for (int c = 0; c < 3; ++c) n[c] = g[c] / len;
    return 0;
}

/* Distance (scene units) from x to the nearest cell face of level L. */
static double face_distance(const orc_setup *s, int32_t L, const double x[3])
{
    const orc_level *lv = &s->level[L];
    double m = INFINITY;
    for (int c = 0; c < 3; ++c) {
        double u = (x[c] - lv->origin[c]) / lv->spacing;
        double fr = u - floor(u);
        double d = (fr < 0.5 ? fr : 1.0 - fr) * lv->spacing;
        if (d < m) m = d;
    }
    return m;
}

/* Bound on a binary32 evaluation's normal error when the hit point is off by
 * at most x_err (L-inf). The six samples x +- h e_c share the hit point's
 * error, so a difference G_c = S(x + h e_c) - S(x - h e_c) moves by the
 * difference of the two gradients times x_err (the sum of their magnitudes
 * where a sample lies within x_err of a cell face, across which the gradient
 * jumps), plus each sample's own rounding (offset, grid coordinate, lerps)
 * and the subtraction's; normalising at most doubles the relative error of
 * the vector. */
static double normal64_error(const orc_setup *s, int32_t L, const double x[3], double x_err)
{
    double h = 0.5 * s->level[L].spacing, G[3], dG = 0.0;
    for (int c = 0; c < 3; ++c) {
        double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
        xp[c] += h;
        xm[c] -= h;
        double gp[3], gm[3], gd[3];
        sdf64_gradient(s, L, xp, gp);
        sdf64_gradient(s, L, xm, gm);
        for (int k = 0; k < 3; ++k) gd[k] = gp[k] - gm[k];
        int near_face = face_distance(s, L, xp) <= x_err || face_distance(s, L, xm) <= x_err;
        double shift = (near_face ? sum_abs3(gp) + sum_abs3(gm) : sum_abs3(gd)) * x_err;
        double own = sum_abs3(gp) * (kU32 * h + point_error(s, L, xp, 0.0, 0.0, 0.0)) +
                     sum_abs3(gm) * (kU32 * h + point_error(s, L, xm, 0.0, 0.0, 0.0));
        double vp = sdf64(s, L, xp), vm = sdf64(s, L, xm);
        G[c] = vp - vm;
        double tri = 8.0 * kU32 * (fabs(vp) + fabs(vm) + 4.0 * s->level[L].spacing);
        double e = shift + own + tri + kU32 * fabs(G[c]);
        if (e > dG) dG = e;
    }
    double len = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
    if (!(len > 0.0)) return INFINITY;
    return 2.0 * sqrt(3.0) * dG / len + 4.0 * kU32;
}

typedef struct {
    trace64_result prim;
    double n[3];
    int32_t visibility;     /* 1 lit, 0 blocked, -1 not traced */
    int32_t shadow_steps;
    double margin, tie;     /* smallest over the primary and shadow decisions */
    double n_err;           /* bound on the binary32 normal's error (L-inf) */
} ray64;

/* Primary trace, hit normal and shadow ray in binary64. The decision whether
 * to trace the shadow ray adds |n.l| to the margins; the shadow ray starts
 * from a point whose binary32 error includes the hit point's and the bias
 * times the normal's. */
static ray64 ray_geometry64(const orc_setup *s, const double o[3], const double w[3],
                            const double l[3])
{
    ray64 g;
    memset(&g, 0, sizeof g);
    g.prim = trace64(s, o, w, 1, kU32 * max_abs3(o), kU32);
    g.margin = g.prim.margin;
    g.tie = g.prim.tie;
    g.visibility = -1;
    if (!is_hit(g.prim.kind)) return g;
    normal64(s, g.prim.level, g.prim.x, w, g.n);
    g.n_err = normal64_error(s, g.prim.level, g.prim.x, g.prim.x_err);
    double ndl = g.n[0] * l[0] + g.n[1] * l[1] + g.n[2] * l[2];
    min_into(&g.margin, fabs(ndl));
    min_into(&g.tie, fabs(ndl) / (3.0 * g.n_err + 4.0 * kU32));
    if (ndl > 0.0) {
        double xs[3], bias = (double)s->shadow_bias;
        for (int c = 0; c < 3; ++c) xs[c] = g.prim.x[c] + bias * g.n[c];
        double xs_err = g.prim.x_err + bias * g.n_err + kU32 * max_abs3(xs);
        trace64_result sh = trace64(s, xs, l, 0, xs_err, kU32);
        min_into(&g.margin, sh.margin);
        min_into(&g.tie, sh.tie);
        g.visibility = is_hit(sh.kind) ? 0 : 1;
        g.shadow_steps = sh.steps;
    }
    return g;
}

/* A ray whose geometry is given by the binary32 sequence (`d32`: outcome,
 * level, steps, hit point and distance, normal, shadow result). */
static ray64 ray_geometry64_given(const ray32 *d32)
{
    ray64 g;
    memset(&g, 0, sizeof g);
    g.prim.kind = d32->prim.kind;
    g.prim.steps = d32->prim.steps;
    g.prim.level = d32->prim.level;
    g.prim.t = (double)d32->prim.t;
    for (int c = 0; c < 3; ++c) g.prim.x[c] = (double)d32->prim.x[c];
    g.margin = g.tie = -1.0;
    g.visibility = d32->visibility;
    g.shadow_steps = d32->shadow_steps;
    for (int c = 0; c < 3; ++c) g.n[c] = (double)d32->n[c];
    return g;
}

/* Per-ray binary64 record (ORC_RAY64_FIELDS doubles): kind, level (0 unless a
 * hit), steps, visibility, shadow steps, t (t_max for a miss, 0 inside),
 * normal, margin, tie ratio, bound on the binary32 t error, bound on the
 * binary32 normal error (the last four -1 for given geometry). */
static void fill_record64(const orc_setup *s, const ray64 *g, double rec[ORC_RAY64_FIELDS])
{
    double t = g->prim.t;
    if (g->prim.kind == ORC_MISS_TMAX || g->prim.kind == ORC_MISS_EXIT) t = (double)s->t_max;
    if (g->prim.kind == ORC_INSIDE) t = 0.0;
    int given = g->margin < 0.0;
    rec[0] = (double)g->prim.kind;
    rec[1] = is_hit(g->prim.kind) ? (double)g->prim.level : 0.0;
    rec[2] = (double)g->prim.steps;
    rec[3] = (double)g->visibility;
    rec[4] = (double)g->shadow_steps;
    rec[5] = t;
    for (int c = 0; c < 3; ++c) rec[6 + c] = g->n[c];
    rec[9] = g->margin;
    rec[10] = g->tie;
    rec[11] = given ? -1.0 : (is_hit(g->prim.kind) ? g->prim.t_err : 0.0);
    rec[12] = given ? -1.0 : g->n_err;
}

void orc_trace_ray64(const orc_setup *s, const double origin[3], const double dir[3],
                     const double dir_to_light[3], double record[ORC_RAY64_FIELDS])
{
    double len = sqrt(dir_to_light[0] * dir_to_light[0] + dir_to_light[1] * dir_to_light[1] +
                      dir_to_light[2] * dir_to_light[2]);
    double l[3] = {dir_to_light[0] / len, dir_to_light[1] / len, dir_to_light[2] / len};
    ray64 g = ray_geometry64(s, origin, dir, l);
    fill_record64(s, &g, record);
}

double orc_sdf64(const orc_setup *s, int32_t level, const double x[3])
{
    return sdf64(s, level, x);
}

int32_t orc_level64(const orc_setup *s, const double x[3], double *margin)
{
    double m;
    int32_t L = level64(s, x, &m);
    if (margin) *margin = m;
    return L;
}

/* Irradiance at x for direction n from a probe atlas: trilinear over the 8
 * probes of the cell around x, each read bilinearly from its padded
 * octahedral tile (the probe interpolation of Sec. 3.4, without visibility). */
void orc_interp_irradiance(const orc_setup *s, const double *atlas, const double x[3],
                           const double n[3], double out[3])
{
    int32_t base[3];
    double f[3];
    for (int c = 0; c < 3; ++c) {
        double g = (x[c] - s->probe_origin[c]) / s->probe_spacing[c];
        double b = floor(g);
        if (b < 0.0) b = 0.0;
        if (b > (double)(s->probe_n[c] - 2)) b = (double)(s->probe_n[c] - 2);
        base[c] = (int32_t)b;
        double fr = g - b;
        f[c] = fr < 0.0 ? 0.0 : (fr > 1.0 ? 1.0 : fr);
    }
    int32_t res = s->irr_res, side = res + 2;
    double uv[2];
    orc_oct_encode(n, uv);
    int32_t a0[2];
    double fa[2];
    for (int k = 0; k < 2; ++k) {
        double sc = ((double)res * (uv[k] + 1.0) + 1.0) * 0.5; /* padded texel units */
        double fl = floor(sc);
        if (fl < 0.0) fl = 0.0;
        if (fl > (double)res) fl = (double)res;
        a0[k] = (int32_t)fl;
        double fr = sc - fl;
        fa[k] = fr < 0.0 ? 0.0 : (fr > 1.0 ? 1.0 : fr);
    }
    out[0] = out[1] = out[2] = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double wp = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *
                            (dz ? f[2] : 1.0 - f[2]);
                int32_t p = (base[0] + dx) +
                            s->probe_n[0] * ((base[1] + dy) + s->probe_n[1] * (base[2] + dz));
                const double *tile = atlas + (size_t)p * side * side * 3;
                for (int dv = 0; dv < 2; ++dv)
                    for (int du = 0; du < 2; ++du) {
                        double wt = (du ? fa[0] : 1.0 - fa[0]) * (dv ? fa[1] : 1.0 - fa[1]);
                        const double *texel = tile + ((size_t)(a0[1] + dv) * side +
                                                      (size_t)(a0[0] + du)) * 3;
                        for (int c = 0; c < 3; ++c) out[c] += wp * wt * texel[c];
                    }
            }
}

/* What the shading of a ray needs from its geometry. */
typedef struct {
    int32_t kind, level, visibility;
    double t, x[3], n[3];
    const double *albedo;   /* analytic scenes: the nearest primitive's albedo */
} ray_hit;

static ray_hit hit_of32(const orc_setup *s, const ray32 *g)
{
    ray_hit h = {g->prim.kind, g->prim.level, g->visibility, (double)g->prim.t,
                 {(double)g->prim.x[0], (double)g->prim.x[1], (double)g->prim.x[2]},
                 {(double)g->n[0], (double)g->n[1], (double)g->n[2]}, NULL};
    if (s->analytic && g->nearest >= 0) h.albedo = s->analytic->albedo + 3 * g->nearest;
    return h;
}

static ray_hit hit_of64(const ray64 *g)
{
    ray_hit h = {g->prim.kind, g->prim.level, g->visibility, g->prim.t,
                 {g->prim.x[0], g->prim.x[1], g->prim.x[2]}, {g->n[0], g->n[1], g->n[2]}, NULL};
    return h;
}

/* Radiance carried back along one probe ray, and its distance (payload). */
static void shade_ray(const orc_setup *s, const orc_frame *f, const double l64[3],
                      const double *prev_irr, const ray_hit *g, double out[4])
{
    int32_t kind = g->kind;
    if (kind == ORC_MISS_TMAX || kind == ORC_MISS_EXIT) {
        for (int c = 0; c < 3; ++c) out[c] = (double)s->sky[c];
        out[3] = (double)s->t_max;
        return;
    }
    if (kind == ORC_INSIDE) {
        out[0] = out[1] = out[2] = out[3] = 0.0;
        return;
    }
    const double *x = g->x, *n = g->n;
    const orc_level *L = &s->level[g->level];
    double albedo[3];
    if (g->albedo) {
        for (int c = 0; c < 3; ++c) albedo[c] = g->albedo[c];
    } else if (L->albedo) {
        double u[3];
        for (int c = 0; c < 3; ++c) u[c] = (x[c] - L->origin[c]) / L->spacing;
        for (int c = 0; c < 3; ++c) albedo[c] = trilinear64(L->albedo, 3, c, L->n, u);
    } else {
        for (int c = 0; c < 3; ++c) albedo[c] = (double)s->albedo[c];
    }
    double ndl = n[0] * l64[0] + n[1] * l64[1] + n[2] * l64[2];
    double lit = (g->visibility == 1 && ndl > 0.0) ? ndl : 0.0;
    double indirect[3] = {0.0, 0.0, 0.0};
    if (s->bounce_gain != 0.0f && prev_irr) orc_interp_irradiance(s, prev_irr, x, n, indirect);
    for (int c = 0; c < 3; ++c) {
        double direct = (double)f->radiance[c] * lit;
        out[c] = albedo[c] / kPi * (direct + (double)s->bounce_gain * indirect[c]);
    }
    out[3] = g->t;
}

/* Eq. 3 estimated from the probe's ray samples as a ratio of weighted sums,
 * E(D) = pi * sum_i w_i L_i / sum_i w_i with w_i = max(0, D . omega_i), which
 * returns pi*L exactly when every sample sees the same radiance L. Depth
 * moments use w_i^s. The new value is mixed with the old one by the
 * hysteresis unless the history is rejected; a texel whose weights all vanish
 * keeps its old value. The border is then filled from the interior. */
static void blend_tile(const orc_setup *s, const double *dirs, int32_t reset,
                       const double *payload, const double *prev_irr, const double *prev_depth,
                       double *irr, double *depth)
{
    double h = reset ? 0.0 : (double)s->hysteresis;
    double sharp = (double)s->depth_sharpness;
    for (int pass = 0; pass < 2; ++pass) {
        int32_t res = pass == 0 ? s->irr_res : s->depth_res;
        int32_t comps = pass == 0 ? 3 : 2;
        int32_t side = res + 2;
        const double *old = pass == 0 ? prev_irr : prev_depth;
        double *out = pass == 0 ? irr : depth;
        for (int32_t j = 0; j < res; ++j)
            for (int32_t i = 0; i < res; ++i) {
                double dn[3];
                orc_texel_direction(res, i, j, dn);
                double sw = 0.0, acc[3] = {0.0, 0.0, 0.0};
                for (int32_t r = 0; r < s->rays; ++r) {
                    const double *w3 = dirs + 3 * r;
                    double c = dn[0] * w3[0] + dn[1] * w3[1] + dn[2] * w3[2];
                    double w = c > 0.0 ? c : 0.0;
                    const double *pl = payload + 4 * (size_t)r;
                    if (pass == 0) {
                        sw += w;
                        for (int k = 0; k < 3; ++k) acc[k] += w * pl[k];
                    } else {
                        double wd = pow(w, sharp);
                        sw += wd;
                        acc[0] += wd * pl[3];
                        acc[1] += wd * pl[3] * pl[3];
                    }
                }
                size_t at = ((size_t)(j + 1) * side + (size_t)(i + 1)) * comps;
                for (int k = 0; k < comps; ++k) {
                    double prev = old ? old[at + k] : 0.0;
                    double v;
                    if (sw > 0.0) {
                        double u = (pass == 0 ? kPi : 1.0) * acc[k] / sw;
                        v = h * prev + (1.0 - h) * u;
                    } else {
                        v = prev;
                    }
                    out[at + k] = v;
                }
            }
        for (int32_t b = 0; b < side; ++b)
            for (int32_t a = 0; a < side; ++a) {
                if (a >= 1 && a <= res && b >= 1 && b <= res) continue;
                int32_t si, sj;
                orc_border_source(res, a, b, &si, &sj);
                size_t dst = ((size_t)b * side + a) * comps;
                size_t src = ((size_t)(sj + 1) * side + (size_t)(si + 1)) * comps;
                for (int k = 0; k < comps; ++k) out[dst + k] = out[src + k];
            }
    }
}

int32_t orc_blend_probe(const orc_setup *s, uint64_t rotation_seed, int32_t reset_history,
                        const double *payload, const double *prev_irr_tile,
                        const double *prev_depth_tile, double *irr_tile, double *depth_tile)
{
    if (s->rays <= 0) return -1;
    double *dirs = (double *)malloc(sizeof(double) * 3 * (size_t)s->rays);
    if (!dirs) return -1;
    orc_ray_directions(rotation_seed, s->rays, dirs);
    blend_tile(s, dirs, reset_history, payload, prev_irr_tile, prev_depth_tile, irr_tile,
               depth_tile);
    free(dirs);
    return 0;
}

/* ======================================================================== */
/* Whole-frame update of a list of probes (Jacobi: every probe reads only    */
/* the previous frame's atlas).                                              */
/* ======================================================================== */

typedef struct {
    const orc_setup *s;
    const orc_frame *f;
    const double *prev_irr, *prev_depth;
    const int32_t *probes;
    int32_t count, stride, first;
    double *irr_tiles, *depth_tiles, *payload;
    int32_t *records;
    int32_t geometry;
    const uint8_t *given;
    double *rays64;
    const double *dirs64;
    const float *dirs32;
    double l64[3];
    float l32[3];
} frame_job;

static void *frame_worker(void *arg)
{
    const frame_job *J = (const frame_job *)arg;
    const orc_setup *s = J->s;
    int32_t R = s->rays;
    size_t irr_tile = (size_t)(s->irr_res + 2) * (s->irr_res + 2) * 3;
    size_t dep_tile = (size_t)(s->depth_res + 2) * (s->depth_res + 2) * 2;
    double *pl = (double *)malloc(sizeof(double) * 4 * (size_t)R);
    if (!pl) return (void *)1;
    for (int32_t q = J->first; q < J->count; q += J->stride) {
        int32_t p = J->probes[q];
        double pos[3];
        orc_probe_position(s, p, pos);
        float o[3] = {(float)pos[0], (float)pos[1], (float)pos[2]};
        for (int32_t r = 0; r < R; ++r) {
            size_t ray = (size_t)q * R + r;
            ray_hit h;
            if (J->geometry == ORC_GEOMETRY_64) {
                ray64 g64;
                if (J->given && J->given[ray]) {
                    ray32 g = ray_geometry32(s, o, J->dirs32 + 3 * r, J->l32);
                    g64 = ray_geometry64_given(&g);
                } else {
                    g64 = ray_geometry64(s, pos, J->dirs64 + 3 * r, J->l64);
                }
                h = hit_of64(&g64);
                if (J->rays64) fill_record64(s, &g64, J->rays64 + ray * ORC_RAY64_FIELDS);
            } else {
                ray32 g = ray_geometry32(s, o, J->dirs32 + 3 * r, J->l32);
                h = hit_of32(s, &g);
                if (J->records) fill_record(s, &g, J->records + ray * 8);
            }
            shade_ray(s, J->f, J->l64, J->prev_irr, &h, pl + 4 * r);
        }
        if (J->payload) memcpy(J->payload + (size_t)q * R * 4, pl, sizeof(double) * 4 * R);
        blend_tile(s, J->dirs64, J->f->reset_history, pl,
                   J->prev_irr ? J->prev_irr + (size_t)p * irr_tile : NULL,
                   J->prev_depth ? J->prev_depth + (size_t)p * dep_tile : NULL,
                   J->irr_tiles + (size_t)q * irr_tile, J->depth_tiles + (size_t)q * dep_tile);
    }
    free(pl);
    return NULL;
}

int32_t orc_update_probes_ex(const orc_setup *s, const orc_frame *f, const double *prev_irr,
                             const double *prev_depth, const int32_t *probes, int32_t count,
                             double *irr_tiles, double *depth_tiles, double *payload,
                             int32_t *records, int32_t geometry, const uint8_t *given,
                             double *rays64, int32_t threads)
{
    if (s->rays <= 0 || s->max_steps < 1 || count < 0) return -1;
    if (geometry != ORC_GEOMETRY_32 && geometry != ORC_GEOMETRY_64) return -1;
    if (s->analytic && geometry != ORC_GEOMETRY_32) return -1;
    int32_t P = s->probe_n[0] * s->probe_n[1] * s->probe_n[2];
    for (int32_t q = 0; q < count; ++q)
        if (probes[q] < 0 || probes[q] >= P) return -1;
    double *d64 = (double *)malloc(sizeof(double) * 3 * (size_t)s->rays);
    float *d32 = (float *)malloc(sizeof(float) * 3 * (size_t)s->rays);
    if (!d64 || !d32) { free(d64); free(d32); return -1; }
    orc_ray_directions(f->rotation_seed, s->rays, d64);
    for (int32_t k = 0; k < 3 * s->rays; ++k) d32[k] = (float)d64[k];
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    frame_job jobs[256];
    pthread_t th[256];
    int32_t rc = 0;
    for (int32_t t = 0; t < threads; ++t) {
        frame_job *J = &jobs[t];
        J->s = s; J->f = f; J->prev_irr = prev_irr; J->prev_depth = prev_depth;
        J->probes = probes; J->count = count; J->stride = threads; J->first = t;
        J->irr_tiles = irr_tiles; J->depth_tiles = depth_tiles; J->payload = payload;
        J->records = geometry == ORC_GEOMETRY_32 ? records : NULL;
        J->geometry = geometry;
        J->given = geometry == ORC_GEOMETRY_64 ? given : NULL;
        J->rays64 = geometry == ORC_GEOMETRY_64 ? rays64 : NULL;
        J->dirs64 = d64; J->dirs32 = d32;
        light_direction(f->dir_to_light, J->l64, J->l32);
    }
    for (int32_t t = 1; t < threads; ++t) pthread_create(&th[t], NULL, frame_worker, &jobs[t]);
    if (frame_worker(&jobs[0])) rc = -1;
    for (int32_t t = 1; t < threads; ++t) {
        void *ret = NULL;
        pthread_join(th[t], &ret);
        if (ret) rc = -1;
    }
    free(d64);
    free(d32);
    return rc;
}

int32_t orc_update_probes(const orc_setup *s, const orc_frame *f, const double *prev_irr,
                          const double *prev_depth, const int32_t *probes, int32_t count,
                          double *irr_tiles, double *depth_tiles, double *payload,
                          int32_t *records, int32_t threads)
{
    return orc_update_probes_ex(s, f, prev_irr, prev_depth, probes, count, irr_tiles,
                                depth_tiles, payload, records, ORC_GEOMETRY_32, NULL, NULL,
                                threads);
}
