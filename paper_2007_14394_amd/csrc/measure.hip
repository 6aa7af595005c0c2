// Measurement kernel: the gather throughput the trace's sampler pattern can reach,
// the second roofline denominator of the trace (beside HBM bandwidth). Each
// thread reads `reads` records of 32 bytes (two adjacent 16-byte loads: the
// layout of one trilinear sample's two corner quads) at indices from a
// counter-based hash, independent of one another so that many are in flight, and
// folds them into a value that is stored only under a condition the data never
// meets (so no load is dead code).
#include "internal.h"

namespace sdfddgi {

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    // the 32-bit finaliser of MurmurHash3 (Appleby)
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

constexpr int kGatherUnroll = 8;

__global__ __launch_bounds__(256) void gather_kernel(const float4 *__restrict__ buf,
                                                     uint32_t mask, int reads, uint32_t seed,
                                                     float *sink) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    float acc = 0.0f;
    for (int r0 = 0; r0 < reads; r0 += kGatherUnroll) {
        float4 a[kGatherUnroll], b[kGatherUnroll];
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) {
            const uint32_t rec = hash32(seed ^ (tid * (uint32_t)reads + (uint32_t)(r0 + u))) & mask;
            a[u] = buf[2 * (size_t)rec];
            b[u] = buf[2 * (size_t)rec + 1];
        }
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) acc += a[u].x + b[u].w;
    }
    if (acc == -1.0f) sink[0] = acc;   // the buffers hold no such values
}

hipError_t launch_gather(const void *buf, int64_t records, int64_t threads, int reads,
                         uint32_t seed, float *sink, hipStream_t s) {
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                       static_cast<const float4 *>(buf), (uint32_t)(records - 1), reads, seed,
                       sink);
    return hipGetLastError();
}

}  // namespace sdfddgi
