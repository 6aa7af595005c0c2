/*
 * Reference checker for the analytic-primitive SDF query (see cluster.h).
 *
 * TEST INFRASTRUCTURE ONLY: plain CPU code for the test-suite; shares no code with
 * the GPU library.
 */
#include "cluster.h"

#include <math.h>

float orc_prim_distance32(int32_t kind, const float c[3], const float h[3], const float x[3])
{
    float dx = x[0] - c[0], dy = x[1] - c[1], dz = x[2] - c[2];
    if (kind == 0) return sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))) - h[0];
    float qx = fabsf(dx) - h[0], qy = fabsf(dy) - h[1], qz = fabsf(dz) - h[2];
    float ox = fmaxf(qx, 0.0f), oy = fmaxf(qy, 0.0f), oz = fmaxf(qz, 0.0f);
    float outside = sqrtf(fmaf(oz, oz, fmaf(oy, oy, ox * ox)));
    float inside = fminf(fmaxf(qx, fmaxf(qy, qz)), 0.0f);
    return outside + inside;
}

float orc_brute_sdf32(const orc_prims32 *p, const float x[3], int64_t *evals)
{
    float best = INFINITY;
    for (int32_t m = 0; m < p->count; ++m) {
        float d = orc_prim_distance32(p->kind[m], p->center + 3 * m, p->half + 3 * m, x);
        if (d < best) best = d;
    }
    if (evals) *evals += p->count;
    return best;
}

void orc_analytic_trace32(const orc_prims32 *p, const float o[3], const float w[3],
                          float t_max, float eps, float relax, int32_t max_steps, float *t,
                          int32_t *steps, int32_t *kind)
{
    float tt = 0.0f;
    for (int32_t k = 0;; ) {
        if (tt > t_max) { *kind = 0; *steps = k; *t = tt; return; }
        float x[3] = {fmaf(tt, w[0], o[0]), fmaf(tt, w[1], o[1]), fmaf(tt, w[2], o[2])};
        float d = orc_brute_sdf32(p, x, 0);
        if (k == 0 && d < 0.0f) { *kind = 4; *steps = 1; *t = tt; return; }
        if (d < eps) { *kind = 2; *steps = k + 1; *t = tt; return; }
        tt = fmaf(relax, d, tt);
        ++k;
        if (k == max_steps) { *kind = 3; *steps = k; *t = tt; return; }
    }
}
