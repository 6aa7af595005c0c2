// Device baker of scene distance grids: the exact signed distance of a union of
// spheres and axis-aligned boxes at the vertices of a vertex-centred grid, with the
// albedo of the nearest primitive. Input preparation (the probe update consumes
// a baked grid); it lets the learned form's training generate thousands of scenes
// on the GPU. Distances are evaluated in binary64 and rounded once to binary32,
// ties in the nearest primitive go to the lower index.
#include "internal.h"

#pragma clang fp contract(off)

namespace sdfddgi {

constexpr int kPrimChunk = 256;   // primitives staged in LDS at a time

__device__ __forceinline__ double prim_distance(int kind, const double *c, const double *h,
                                                double px, double py, double pz) {
    const double dx = px - c[0], dy = py - c[1], dz = pz - c[2];
    if (kind == 0) return sqrt(dx * dx + dy * dy + dz * dz) - h[0];
    // box: Euclidean distance outside plus the (negative) largest axis excess inside
    const double qx = fabs(dx) - h[0], qy = fabs(dy) - h[1], qz = fabs(dz) - h[2];
    const double ox = qx > 0 ? qx : 0, oy = qy > 0 ? qy : 0, oz = qz > 0 ? qz : 0;
    const double outside = sqrt(ox * ox + oy * oy + oz * oz);
    double m = qx > qy ? qx : qy;
    m = m > qz ? m : qz;
    const double inside = m < 0 ? m : 0;
    return outside + inside;
}

// One thread per vertex; every workgroup walks the primitives chunk by chunk.
__global__ __launch_bounds__(256) void bake_kernel(BakeArgs a) {
    __shared__ double s_c[kPrimChunk][3], s_h[kPrimChunk][3];
    __shared__ int s_k[kPrimChunk];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nv = (int64_t)a.n0 * a.n1 * a.n2;
    const int i = (int)(v % a.n0), j = (int)((v / a.n0) % a.n1), k = (int)(v / ((int64_t)a.n0 * a.n1));
    const double px = a.org0 + a.spacing * i;
    const double py = a.org1 + a.spacing * j;
    const double pz = a.org2 + a.spacing * k;
    double best = INFINITY;
    int arg = -1;
    for (int m0 = 0; m0 < a.nprims; m0 += kPrimChunk) {
        const int cnt = min(kPrimChunk, a.nprims - m0);
        __syncthreads();
        for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
            s_k[e] = a.kind[m0 + e];
            for (int c = 0; c < 3; ++c) {
                s_c[e][c] = a.center[3 * (m0 + e) + c];
                s_h[e][c] = a.half[3 * (m0 + e) + c];
            }
        }
        __syncthreads();
        for (int m = 0; m < cnt; ++m) {
            const double d = prim_distance(s_k[m], s_c[m], s_h[m], px, py, pz);
            if (d < best) { best = d; arg = m0 + m; }
        }
    }
    if (v >= nv) return;
    a.sdf[v] = arg < 0 ? a.empty_value : (float)best;
    if (a.alb)
        for (int c = 0; c < 3; ++c)
            a.alb[3 * v + c] = arg < 0 ? 0.0f : (float)a.albedo[3 * arg + c];
}

hipError_t launch_bake(const BakeArgs &a, hipStream_t s) {
    const int64_t nv = (int64_t)a.n0 * a.n1 * a.n2;
    hipLaunchKernelGGL(bake_kernel, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sdfddgi
