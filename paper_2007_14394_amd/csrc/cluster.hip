// gfx950 kernels of the analytic-primitive SDF query of Sec. 3.3 on their own
// (the cluster walk itself is in analytic_common.h):
//
//   cluster_query_kernel  one distance per point
//   cluster_trace_kernel  one sphere-traced ray per thread
#include "internal.h"
#include "analytic_common.h"

#pragma clang fp contract(off)

namespace sdfddgi {

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
