/*
 * Reference checker for the analytic-primitive SDF query of Sec. 3.3 (the
 * cluster culling with the 2 lastSDF bound) and for sphere tracing with it.
 *
 * TEST INFRASTRUCTURE ONLY: plain CPU code for the test-suite; the library never
 * links or calls it. Distances are binary32 in one fixed operation sequence
 * (fmaf marks every fused multiply-add), the precision the kernel works in, so
 * results compare bit for bit.
 *
 * Primitive distances (binary32):
 *   sphere  d = sqrt(fma(dz,dz, fma(dy,dy, dx*dx))) - r,   d* = x* - c*
 *   box     q* = |x* - c*| - h*;  d = sqrt(fma(oz,oz, fma(oy,oy, ox*ox)))
 *           + min(max(qx, qy, qz), 0),   o* = max(q*, 0)
 * The scene distance is the minimum over all primitives (exact: no rounding).
 */
#ifndef SDFDDGI_ORACLE_CLUSTER_H
#define SDFDDGI_ORACLE_CLUSTER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t count;
    const int32_t *kind;      /* 0 sphere (radius half[0]), 1 axis-aligned box */
    const float *center;      /* [count][3] */
    const float *half;        /* [count][3] */
} orc_prims32;

float orc_prim_distance32(int32_t kind, const float c[3], const float h[3], const float x[3]);

/* Minimum over every primitive (+inf for none); *evals (may be NULL) += count. */
float orc_brute_sdf32(const orc_prims32 *p, const float x[3], int64_t *evals);

/* Sphere trace with the brute-force distance, the same stopping rules as the grid
 * trace without a grid box: t > t_max -> 0 (miss), d < 0 at the first sample -> 4
 * (inside), d < eps -> 2 (hit), max_steps samples -> 3 (hit, exhausted); the
 * step is t = fma(relax, d, t), the sample fma(t, w, o). */
void orc_analytic_trace32(const orc_prims32 *p, const float o[3], const float w[3],
                          float t_max, float eps, float relax, int32_t max_steps, float *t,
                          int32_t *steps, int32_t *kind);

#ifdef __cplusplus
}
#endif
#endif
