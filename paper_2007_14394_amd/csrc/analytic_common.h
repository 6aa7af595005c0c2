// Device code of the analytic-primitive SDF query of Sec. 3.3, shared by the
// standalone query and trace kernels (cluster.hip) and by the probe update's trace
// kernels when a context traces the primitives instead of a grid (kernels.hip).
// Primitives are packed into clusters; a cluster's primitives are visited only
// when the signed distance to its bounding box is below the best distance so far,
// and along a sphere-traced ray the best distance starts from the bound the
// previous sample gives (the paper's 2 lastSDF) instead of infinity. Distances are
// binary32 in one fixed sequence; the culled minimum equals the minimum over every
// primitive bit for bit (a minimum is exact, and every culling test compares a
// lower bound of a cluster's distances, widened beyond rounding, against an upper
// bound of the scene's).
#pragma once

#include "internal.h"

namespace sdfddgi {

__device__ __forceinline__ float prim_distance32(int kind, const float *c, const float *h,
                                                 float x0, float x1, float x2) {
    const float dx = x0 - c[0], dy = x1 - c[1], dz = x2 - c[2];
    if (kind == 0) return sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))) - h[0];
    const float qx = fabsf(dx) - h[0], qy = fabsf(dy) - h[1], qz = fabsf(dz) - h[2];
    const float ox = fmaxf(qx, 0.0f), oy = fmaxf(qy, 0.0f), oz = fmaxf(qz, 0.0f);
    const float outside = sqrtf(fmaf(oz, oz, fmaf(oy, oy, ox * ox)));
    const float inside = fminf(fmaxf(qx, fmaxf(qy, qz)), 0.0f);
    return outside + inside;
}

// Signed distance to an axis-aligned box given by its corners.
__device__ __forceinline__ float box_distance32(const float *lo, const float *hi, float x0,
                                                float x1, float x2) {
    const float qx = fmaxf(lo[0] - x0, x0 - hi[0]);
    const float qy = fmaxf(lo[1] - x1, x1 - hi[1]);
    const float qz = fmaxf(lo[2] - x2, x2 - hi[2]);
    const float ox = fmaxf(qx, 0.0f), oy = fmaxf(qy, 0.0f), oz = fmaxf(qz, 0.0f);
    return sqrtf(fmaf(oz, oz, fmaf(oy, oy, ox * ox))) + fminf(fmaxf(qx, fmaxf(qy, qz)), 0.0f);
}

struct ClusterLds {
    int kind[kMaxAnalyticPrims];
    int orig[kMaxAnalyticPrims];    // the primitive's index in the caller's order
    float cen[kMaxAnalyticPrims][3], hal[kMaxAnalyticPrims][3];
    float lo[kMaxClusters][3], hi[kMaxClusters][3];
    int first[kMaxClusters + 1];
};

__device__ __forceinline__ void load_clusters(const AnalyticArgs &a, ClusterLds &s) {
    for (int e = threadIdx.x; e < a.nprims; e += blockDim.x) {
        s.kind[e] = a.kind[e];
        s.orig[e] = a.orig ? a.orig[e] : e;
        for (int c = 0; c < 3; ++c) {
            s.cen[e][c] = a.center[3 * e + c];
            s.hal[e][c] = a.half[3 * e + c];
        }
    }
    for (int e = threadIdx.x; e < a.nclusters; e += blockDim.x)
        for (int c = 0; c < 3; ++c) {
            s.lo[e][c] = a.lo[3 * e + c];
            s.hi[e][c] = a.hi[3 * e + c];
        }
    for (int e = threadIdx.x; e <= a.nclusters; e += blockDim.x) s.first[e] = a.first[e];
    __syncthreads();
}

// The scene distance at x: mode 0 every primitive; otherwise the cluster walk from
// the bound d_init (+inf, or the previous sample's bound along a ray).
__device__ __forceinline__ float scene_distance(const AnalyticArgs &a, const ClusterLds &s,
                                                int mode, float x0, float x1, float x2,
                                                float d_init, uint32_t &evals) {
    if (mode == 0) {
        float best = INFINITY;
        for (int m = 0; m < a.nprims; ++m)
            best = fminf(best, prim_distance32(s.kind[m], s.cen[m], s.hal[m], x0, x1, x2));
        evals += (uint32_t)a.nprims;
        return best;
    }
    float D = d_init;
    for (int c = 0; c < a.nclusters; ++c) {
        if (!(box_distance32(s.lo[c], s.hi[c], x0, x1, x2) < D)) continue;
        for (int m = s.first[c]; m < s.first[c + 1]; ++m)
            D = fminf(D, prim_distance32(s.kind[m], s.cen[m], s.hal[m], x0, x1, x2));
        evals += (uint32_t)(s.first[c + 1] - s.first[c]);
    }
    return D;
}

// The cluster walk from the bound d_init that also names the nearest primitive: its
// cluster-order slot in *slot, the one of lowest caller index among those at the
// minimum. Every primitive at the minimum is visited: its cluster's box distance is
// strictly below its own (the boxes are widened), hence below the minimum.
__device__ __forceinline__ float nearest_distance(const AnalyticArgs &a, const ClusterLds &s,
                                                  float x0, float x1, float x2, float d_init,
                                                  int &slot) {
    float D = d_init;
    int best_orig = 0x7fffffff;
    slot = -1;
    for (int c = 0; c < a.nclusters; ++c) {
        if (!(box_distance32(s.lo[c], s.hi[c], x0, x1, x2) < D)) continue;
        for (int m = s.first[c]; m < s.first[c + 1]; ++m) {
            const float d = prim_distance32(s.kind[m], s.cen[m], s.hal[m], x0, x1, x2);
            if (d < D || (d == D && s.orig[m] < best_orig)) {
                D = d;
                best_orig = s.orig[m];
                slot = m;
            }
        }
    }
    return D;
}

// The bound on the next sample's distance from the previous one d: the scene
// distance is 1-Lipschitz and the ray moved relax * d, so it is at most
// (1 + relax) d (the paper's 2 lastSDF for relax = 1); widened by 2^-10
// relative and 1e-4 m so that it stays a bound under binary32 rounding.
__device__ __forceinline__ float next_bound(float relax, float d) {
    return fmaf((1.0f + relax) * d, 1.0009765625f, 1.0e-4f);
}

// Normal at x from the gradient of the distance of primitive slot m: a sphere's
// radial direction x - c; outside a box the offset from its nearest point, inside
// it the signed axis of the face nearest to x (the largest q, lowest axis on a
// tie); normalised like the grid normal, -w where the gradient vanishes.
__device__ __forceinline__ void analytic_normal(const ClusterLds &s, int m, float x0, float x1,
                                                float x2, float w0, float w1, float w2,
                                                float &n0, float &n1, float &n2) {
    const float d[3] = {x0 - s.cen[m][0], x1 - s.cen[m][1], x2 - s.cen[m][2]};
    float g[3] = {0.0f, 0.0f, 0.0f};
    if (s.kind[m] == 0) {
        g[0] = d[0]; g[1] = d[1]; g[2] = d[2];
    } else {
        float q[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) q[k] = fabsf(d[k]) - s.hal[m][k];
        const float qm = fmaxf(q[0], fmaxf(q[1], q[2]));
        if (qm > 0.0f) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float o = fmaxf(q[k], 0.0f);
                g[k] = d[k] >= 0.0f ? o : -o;
            }
        } else {
            const int ax = q[0] >= q[1] ? (q[0] >= q[2] ? 0 : 2) : (q[1] >= q[2] ? 1 : 2);
            g[ax] = d[ax] >= 0.0f ? 1.0f : -1.0f;
        }
    }
    const float len2 = fmaf(g[2], g[2], fmaf(g[1], g[1], g[0] * g[0]));
    if (!(len2 >= 1e-24f)) { n0 = -w0; n1 = -w1; n2 = -w2; return; }
    const float inv = 1.0f / sqrtf(len2);
    n0 = g[0] * inv; n1 = g[1] * inv; n2 = g[2] * inv;
}

}  // namespace sdfddgi
