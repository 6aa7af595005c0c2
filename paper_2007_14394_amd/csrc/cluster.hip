// gfx950 kernels of the analytic-primitive SDF query of Sec. 3.3: primitives packed
// into clusters, a cluster's primitives visited only when the signed distance to
// its bounding box is below the best distance so far, and along a sphere-traced
// ray the best distance starting from the bound the previous sample gives (the
// paper's 2 lastSDF), instead of infinity.
//
//   cluster_query_kernel  one distance per point
//   cluster_trace_kernel  one sphere-traced ray per thread
//
// Distances are binary32 in the fixed sequence of the reference checker; the
// culled minimum equals the minimum over every primitive bit for bit (minimum is
// exact, and every culling test compares a lower bound of a cluster's distances,
// widened beyond rounding, against an upper bound of the scene's).
#include "internal.h"

#pragma clang fp contract(off)

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
    float cen[kMaxAnalyticPrims][3], hal[kMaxAnalyticPrims][3];
    float lo[kMaxClusters][3], hi[kMaxClusters][3];
    int first[kMaxClusters + 1];
};

__device__ __forceinline__ void load_clusters(const AnalyticArgs &a, ClusterLds &s) {
    for (int e = threadIdx.x; e < a.nprims; e += blockDim.x) {
        s.kind[e] = a.kind[e];
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

__global__ __launch_bounds__(256) void cluster_query_kernel(AnalyticArgs a, const float *pts,
                                                            int n, int mode, float *out,
                                                            unsigned long long *evals) {
    __shared__ ClusterLds s;
    load_clusters(a, s);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t ev = 0;
    if (q < n)
        out[q] = scene_distance(a, s, mode, pts[3 * q], pts[3 * q + 1], pts[3 * q + 2], INFINITY,
                                ev);
    if (evals && ev) atomicAdd(evals, (unsigned long long)ev);
}

// The bound on the next sample's distance from the previous one d: the scene
// distance is 1-Lipschitz and the ray moved relax * d, so it is at most
// (1 + relax) d (the paper's 2 lastSDF for relax = 1); widened by 2^-10
// relative and 1e-4 m so that it stays a bound under binary32 rounding.
__device__ __forceinline__ float next_bound(float relax, float d) {
    return fmaf((1.0f + relax) * d, 1.0009765625f, 1.0e-4f);
}

__global__ __launch_bounds__(256) void cluster_trace_kernel(AnalyticArgs a, AnalyticTrace r) {
    __shared__ ClusterLds s;
    load_clusters(a, s);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t ev = 0;
    if (q < r.n) {
        const float o0 = r.o[3 * q], o1 = r.o[3 * q + 1], o2 = r.o[3 * q + 2];
        const float w0 = r.w[3 * q], w1 = r.w[3 * q + 1], w2 = r.w[3 * q + 2];
        float t = 0.0f, bound = INFINITY;
        int k = 0, kind = -1, steps = 0;
        while (kind < 0) {
            if (t > r.t_max) { kind = 0; steps = k; break; }
            const float x0 = fmaf(t, w0, o0), x1 = fmaf(t, w1, o1), x2 = fmaf(t, w2, o2);
            const float d = scene_distance(a, s, r.mode, x0, x1, x2, r.mode == 2 ? bound : INFINITY,
                                           ev);
            if (k == 0 && d < 0.0f) { kind = 4; steps = 1; break; }
            if (d < r.eps) { kind = 2; steps = k + 1; break; }
            t = fmaf(r.relax, d, t);
            bound = next_bound(r.relax, d);
            ++k;
            if (k == r.max_steps) { kind = 3; steps = k; break; }
        }
        r.t_out[q] = t;
        r.steps_out[q] = steps;
        r.kind_out[q] = kind;
    }
    if (r.evals && ev) atomicAdd(r.evals, (unsigned long long)ev);
}

hipError_t launch_cluster_query(const AnalyticArgs &a, const float *pts, int n, int mode,
                                float *out, unsigned long long *evals, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(cluster_query_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a,
                       pts, n, mode, out, evals);
    return hipGetLastError();
}

hipError_t launch_cluster_trace(const AnalyticArgs &a, const AnalyticTrace &r, hipStream_t s) {
    if (r.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(cluster_trace_kernel, dim3((unsigned)((r.n + 255) / 256)), dim3(256), 0, s,
                       a, r);
    return hipGetLastError();
}

}  // namespace sdfddgi
