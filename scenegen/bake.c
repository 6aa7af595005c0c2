/*
 * Baker for the synthetic test scenes: evaluates the exact signed distance of a
 * union of spheres and axis-aligned boxes at the vertices of a vertex-centred
 * grid, and records the albedo of the nearest primitive at each vertex.
 *
 * This is input preparation only (the probe update consumes a baked grid); it
 * holds none of the probe-update arithmetic and is shared, as data, by both the
 * reference checker and the GPU library.
 *
 * Grid convention: vertex (i, j, k) sits at origin + spacing * (i, j, k); the
 * arrays are laid out [k][j][i] (x fastest); albedo is [k][j][i][3].
 * Distances are evaluated in binary64 and rounded once to binary32.
 * Ties in the nearest-primitive choice go to the lower primitive index.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

enum { PRIM_SPHERE = 0, PRIM_BOX = 1 };

typedef struct {
    int32_t nprims;
    const int32_t *kind;   /* [nprims] */
    const double *center;  /* [nprims][3] */
    const double *half;    /* [nprims][3]; sphere radius in half[0] */
    const double *albedo;  /* [nprims][3] */
    int32_t n[3];
    double origin[3];
    double spacing;
    float *sdf;            /* [n2][n1][n0] */
    float *alb;            /* [n2][n1][n0][3] or NULL */
    float empty_value;     /* distance stored when there are no primitives */
    int32_t k0, k1;        /* z-slice range for one worker */
} bake_job;

static double prim_distance(int32_t kind, const double *c, const double *h,
                            double px, double py, double pz)
{
    double dx = px - c[0], dy = py - c[1], dz = pz - c[2];
    if (kind == PRIM_SPHERE)
        return sqrt(dx * dx + dy * dy + dz * dz) - h[0];
    /* box: distance outside plus (negative) distance inside */
    double qx = fabs(dx) - h[0], qy = fabs(dy) - h[1], qz = fabs(dz) - h[2];
    double ox = qx > 0 ? qx : 0, oy = qy > 0 ? qy : 0, oz = qz > 0 ? qz : 0;
    double outside = sqrt(ox * ox + oy * oy + oz * oz);
    double m = qx > qy ? qx : qy;
    m = m > qz ? m : qz;
    double inside = m < 0 ? m : 0;
    return outside + inside;
}

static void *bake_slices(void *arg)
{
    const bake_job *b = (const bake_job *)arg;
    for (int32_t k = b->k0; k < b->k1; ++k)
        for (int32_t j = 0; j < b->n[1]; ++j)
            for (int32_t i = 0; i < b->n[0]; ++i) {
                double px = b->origin[0] + b->spacing * i;
                double py = b->origin[1] + b->spacing * j;
                double pz = b->origin[2] + b->spacing * k;
                double best = INFINITY;
                int32_t arg_best = -1;
                for (int32_t m = 0; m < b->nprims; ++m) {
                    double d = prim_distance(b->kind[m], b->center + 3 * m,
                                             b->half + 3 * m, px, py, pz);
                    if (d < best) { best = d; arg_best = m; }
                }
                size_t v = ((size_t)k * b->n[1] + j) * b->n[0] + i;
                b->sdf[v] = arg_best < 0 ? b->empty_value : (float)best;
                if (b->alb) {
                    for (int c = 0; c < 3; ++c)
                        b->alb[3 * v + c] = arg_best < 0 ? 0.0f
                                                         : (float)b->albedo[3 * arg_best + c];
                }
            }
    return NULL;
}

/* Bake one grid level. Returns 0 on success, -1 on bad arguments. */
int bake_level(int32_t nprims, const int32_t *kind, const double *center,
               const double *half, const double *albedo, const int32_t n[3],
               const double origin[3], double spacing, float empty_value,
               float *sdf, float *alb, int32_t nthreads)
{
    if (n[0] < 2 || n[1] < 2 || n[2] < 2 || !(spacing > 0) || !sdf) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    if (nthreads > n[2]) nthreads = n[2];
    bake_job jobs[64];
    pthread_t th[64];
    for (int t = 0; t < nthreads; ++t) {
        bake_job *b = &jobs[t];
        b->nprims = nprims; b->kind = kind; b->center = center; b->half = half;
        b->albedo = albedo;
        for (int c = 0; c < 3; ++c) { b->n[c] = n[c]; b->origin[c] = origin[c]; }
        b->spacing = spacing; b->sdf = sdf; b->alb = alb; b->empty_value = empty_value;
        b->k0 = (int32_t)((int64_t)n[2] * t / nthreads);
        b->k1 = (int32_t)((int64_t)n[2] * (t + 1) / nthreads);
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, bake_slices, &jobs[t]);
    bake_slices(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    return 0;
}
