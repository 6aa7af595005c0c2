// gfx950 kernels of the batched form: many scenes of uneven size updated by one
// set of launches per frame (captured once in a graph and replayed).
//
//   batch_begin_kernel    zero the counters, stamp the frame start on the device clock
//   batch_primary_kernel  primary sphere trace of every scene's rays, one persistent
//                         wave-compacted grid over the concatenated ray space
//   batch_hits_kernel     hit shading of every scene's queued hits
//   batch_blend_kernel    the precision-form blend of every scene's probes, one
//                         workgroup per 16 probes of a scene; stamps each scene's end
//
// Each ray runs the same binary32 sequence as the single-scene kernels with the
// scene's binary16 grid (one level: the grid box is the whole domain), so a scene's
// rays, payload and maps are bit-identical to a single-scene context in the
// precision form. A lane's scene comes from the ray's slot (binary search over the
// scenes' first slots) or from the hit-queue entry; the fields the sample loop needs
// are copied to registers when the lane takes the ray. The chunk sizes, refill
// threshold and grid sizes are chosen by the runtime's autotuner.
#include "internal.h"
#include "octahedral.h"
#include "trace_common.h"
#include "blend_common.h"

#pragma clang fp contract(off)

namespace sdfddgi {

// The fields of a lane's scene that every sample reads.
struct LaneScene {
    LevelLds lv;
    float xlo0, xlo1, xlo2, xhi0, xhi1, xhi2;
    float eps, t_max, relax;
    int max_steps;
};

__device__ __forceinline__ LaneScene lane_scene(const BatchScene &s) {
    LaneScene d;
    d.lv = s.lv;
    d.xlo0 = s.xlo0; d.xlo1 = s.xlo1; d.xlo2 = s.xlo2;
    d.xhi0 = s.xhi0; d.xhi1 = s.xhi1; d.xhi2 = s.xhi2;
    d.eps = s.eps; d.t_max = s.t_max; d.relax = s.relax; d.max_steps = s.max_steps;
    return d;
}

// One sample of the fixed sphere-trace sequence (as trace_step of the single-scene
// kernels with one level: a point inside the grid box is level 0, else the ray
// escapes).
template <bool kPrimary>
__device__ __forceinline__ int batch_step(const LaneScene &d, float o0, float o1, float o2,
                                          float w0, float w1, float w2, float &t, int &k,
                                          float &x0, float &x1, float &x2, int &steps) {
    if (t > d.t_max) { steps = k; return kMissTmax; }
    x0 = fmaf(t, w0, o0); x1 = fmaf(t, w1, o1); x2 = fmaf(t, w2, o2);
    const bool in = (x0 >= d.xlo0) & (x0 <= d.xhi0) & (x1 >= d.xlo1) & (x1 <= d.xhi1) &
                    (x2 >= d.xlo2) & (x2 <= d.xhi2);
    if (!in) { steps = k; return kMissExit; }
    const float dist = trilinear<true>(d.lv, (x0 - d.lv.org0) * d.lv.inv,
                                       (x1 - d.lv.org1) * d.lv.inv, (x2 - d.lv.org2) * d.lv.inv);
    if (kPrimary && k == 0 && dist < 0.0f) { steps = 1; return kInside; }
    if (dist < d.eps) { steps = k + 1; return kHit; }
    t = fmaf(d.relax, dist, t);
    ++k;
    if (k == d.max_steps) { steps = k; return kHitExhausted; }
    return -1;
}

__device__ __forceinline__ void load_scenes(const BatchArgs &a, BatchScene *s_sc, int *s_base) {
    for (int e = threadIdx.x; e < a.nscenes; e += blockDim.x) {
        s_sc[e] = a.scenes[e];
        s_base[e] = a.scenes[e].ray_base;
    }
    __syncthreads();
}

// Scene of a ray slot: the last scene whose first slot is <= slot.
__device__ __forceinline__ int scene_of(const int *s_base, int n, int slot) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_base[mid] <= slot) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(64) void batch_begin_kernel(int *counter,
                                                         unsigned long long *stamps, int n) {
    // stamps[0]: frame start; stamps[1 + s]: end of scene s's blend
    for (int e = threadIdx.x; e <= n; e += blockDim.x) stamps[e] = 0ull;
    for (int e = threadIdx.x; e < kBatchCounters; e += blockDim.x) counter[e] = 0;
    __syncthreads();
    if (threadIdx.x == 0) stamps[0] = wall_clock64();
}

__device__ __forceinline__ void batch_flush(const BatchArgs &a, int4 *buf, int count) {
    if (count == 0) return;
    int base = 0;
    if (__lane_id() == 0) base = atomicAdd(a.counter + 2, count);
    base = __builtin_amdgcn_readfirstlane(base);
    const int lane = (int)__lane_id();
    if (lane < count) a.hitq[base + lane] = buf[lane];
    __builtin_amdgcn_wave_barrier();
}

// Primary trace over the concatenated rays of all scenes (see primary_kernel).
template <int kChunkSize>
__global__ __launch_bounds__(256) void batch_primary_kernel(BatchArgs a) {
    __shared__ BatchScene s_sc[kMaxBatchScenes];
    __shared__ int s_base[kMaxBatchScenes];
    __shared__ int4 s_hits[4][64];
    load_scenes(a, s_sc, s_base);
    const int lane = (int)__lane_id();
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    int staged = 0;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // blocks of the concatenated rays dealt to the XCDs in turn (see BlockFeeder)
    BlockFeeder<kChunkSize, kBatchBlockRays / kChunkSize> feed;
    feed.start();
    bool active = false;
    int ray = 0, k = 0, sc = 0;
    float o0 = 0, o1 = 0, o2 = 0, w0 = 0, w1 = 0, w2 = 0, t = 0;
    LaneScene d{};
    while (true) {
        uint64_t stepping = __ballot(active);
        if (__popcll(stepping) < a.refill) {
            uint64_t idle = ~stepping;
            while (idle != 0 && !feed.exhausted) {
                int first = 0;
                const int n = feed.claim(a.counter + kPartStride, a.total_rays, __popcll(idle), first);
                const int rank = __popcll(idle & below);
                if (!active && rank < n) {
                    const int slot = first + rank;
                    sc = scene_of(s_base, a.nscenes, slot);
                    const BatchScene &s = s_sc[sc];
                    const int local = slot - s.ray_base;
                    const int q = local / s.R, i = local - q * s.R;
                    const int p = a.probe_order[s.probe_base + q];
                    ray = s.ray_base + p * s.R + i;
                    const int gp = s.probe_base + p;
                    o0 = a.probe_pos[3 * gp]; o1 = a.probe_pos[3 * gp + 1]; o2 = a.probe_pos[3 * gp + 2];
                    const int di = s.dir_base + i;
                    w0 = a.dirs[3 * di]; w1 = a.dirs[3 * di + 1]; w2 = a.dirs[3 * di + 2];
                    d = lane_scene(s);
                    t = 0.0f;
                    k = 0;
                    active = true;
                }
                idle = __ballot(!active);
            }
            stepping = __ballot(active);
            if (stepping == 0) {
                batch_flush(a, s_hits[wave], staged);
                break;
            }
        }
        bool hit_now = false;
        int4 entry = make_int4(0, 0, 0, 0);
        if (active) {
            const float tt = t;
            float x0, x1, x2;
            int steps = 0;
            const int kind = batch_step<true>(d, o0, o1, o2, w0, w1, w2, t, k, x0, x1, x2, steps);
            if (kind >= 0) {
                if (kind == kHit || kind == kHitExhausted) {
                    hit_now = true;
                    entry = make_int4(ray, __float_as_int(tt), pack_hit(kind, 0, steps), sc);
                } else {
                    const BatchScene &s = s_sc[sc];
                    a.payload[ray] = kind == kInside ? make_float4(0.0f, 0.0f, 0.0f, 0.0f)
                                                     : make_float4(s.sky0, s.sky1, s.sky2, s.t_max);
                }
                active = false;
            }
        }
        const uint64_t hm = __ballot(hit_now);
        if (hm) {
            const int n = __popcll(hm);
            if (staged + n > 64) {
                batch_flush(a, s_hits[wave], staged);
                staged = 0;
            }
            if (hit_now) s_hits[wave][staged + __popcll(hm & below)] = entry;
            __builtin_amdgcn_wave_barrier();
            staged += n;
            if (staged == 64) {
                batch_flush(a, s_hits[wave], staged);
                staged = 0;
            }
        }
    }
}

enum : int { kBIdle = 0, kBShadow = 1, kBNew = 2, kBPendShade = 3 };
constexpr int kBShadeBatch = 16;

__device__ __forceinline__ float3 batch_albedo(const BatchScene &s, float x0, float x1, float x2) {
    const LevelLds &d = s.lv;
    if (!d.alb) return make_float3(s.alb0, s.alb1, s.alb2);
    int i0, i1, i2;
    float f0, f1, f2;
    cell_of((x0 - d.org0) * d.inv, d.cmax0, i0, f0);
    cell_of((x1 - d.org1) * d.inv, d.cmax1, i1, f1);
    cell_of((x2 - d.org2) * d.inv, d.cmax2, i2, f2);
    const uint32_t sy = d.arow, sz = d.aslice;
    const float *p = d.alb + 3u * ((uint32_t)i2 * sz + (uint32_t)i1 * sy + (uint32_t)i0);
    float out[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float v000 = p[c], v100 = p[3 + c], v010 = p[3 * sy + c], v110 = p[3 * (sy + 1) + c];
        const float v001 = p[3 * sz + c], v101 = p[3 * (sz + 1) + c];
        const float v011 = p[3 * (sz + sy) + c], v111 = p[3 * (sz + sy + 1) + c];
        const float c00 = fmaf(f0, v100 - v000, v000), c10 = fmaf(f0, v110 - v010, v010);
        const float c01 = fmaf(f0, v101 - v001, v001), c11 = fmaf(f0, v111 - v011, v011);
        const float c0 = fmaf(f1, c10 - c00, c00), c1 = fmaf(f1, c11 - c01, c01);
        out[c] = fmaf(f2, c1 - c0, c0);
    }
    return make_float3(out[0], out[1], out[2]);
}

// Hit shading of every scene's queued hits (see hits_kernel).
template <int kChunkSize>
__global__ __launch_bounds__(256) void batch_hits_kernel(BatchArgs a) {
    __shared__ BatchScene s_sc[kMaxBatchScenes];
    __shared__ int s_base[kMaxBatchScenes];
    load_scenes(a, s_sc, s_base);
    const int lane = (int)__lane_id();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int total = a.counter[2];
    Feeder<kChunkSize> feed;
    const int tile = 10 * 10 * 3;   // 8x8 irradiance tile with its border

    int mode = kBIdle, ray = 0, info = 0, k = 0, vis = -1, sc = 0;
    float ht = 0, hx0 = 0, hx1 = 0, hx2 = 0, n0 = 0, n1 = 0, n2 = 0;
    float o0 = 0, o1 = 0, o2 = 0, t = 0, l0 = 0, l1 = 0, l2 = 0;
    LaneScene d{};
    while (true) {
        uint64_t stepping = __ballot(mode == kBShadow);
        const int waiting = __popcll(__ballot(mode == kBPendShade));
        if (__popcll(stepping) < a.refill || waiting >= kBShadeBatch) {
            for (int round = 0; round < 2; ++round) {
                if (__ballot(mode == kBPendShade)) {
                    if (mode == kBPendShade) {
                        const BatchScene &s = s_sc[sc];
                        const float *lt = a.lights + 6 * sc;
                        const float ndl = fmaf(n2, l2, fmaf(n1, l1, n0 * l0));
                        const float lit = vis == 1 ? ndl : 0.0f;
                        const float3 alb = batch_albedo(s, hx0, hx1, hx2);
                        float3 ind = make_float3(0.0f, 0.0f, 0.0f);
                        if (s.gain != 0.0f)
                            ind = interp_irradiance(a.prev_irr + (size_t)s.probe_base * tile, 8,
                                                    s.pg, hx0, hx1, hx2, n0, n1, n2);
                        const float inv_pi = 0.318309886183790671538f;
                        float4 out;
                        out.x = alb.x * inv_pi * (lt[3] * lit + s.gain * ind.x);
                        out.y = alb.y * inv_pi * (lt[4] * lit + s.gain * ind.y);
                        out.z = alb.z * inv_pi * (lt[5] * lit + s.gain * ind.z);
                        out.w = ht;
                        a.payload[ray] = out;
                        mode = kBIdle;
                    }
                }
                if (round == 1) break;
                uint64_t idle = __ballot(mode == kBIdle);
                while (idle != 0 && !feed.exhausted) {
                    int first = 0;
                    const int n = feed.claim(a.counter + 1, total, __popcll(idle), first);
                    const int rank = __popcll(idle & below);
                    if (mode == kBIdle && rank < n) {
                        const int4 e = a.hitq[first + rank];
                        ray = e.x;
                        ht = __int_as_float(e.y);
                        info = e.z;
                        sc = e.w;
                        mode = kBNew;
                    }
                    idle = __ballot(mode == kBIdle);
                }
                if (__ballot(mode == kBNew)) {
                    if (mode == kBNew) {
                        const BatchScene &s = s_sc[sc];
                        const int local = ray - s.ray_base;
                        const int p = local / s.R, i = local - (local / s.R) * s.R;
                        const int gp = s.probe_base + p;
                        const float po0 = a.probe_pos[3 * gp], po1 = a.probe_pos[3 * gp + 1],
                                    po2 = a.probe_pos[3 * gp + 2];
                        const int di = s.dir_base + i;
                        const float w0 = a.dirs[3 * di], w1 = a.dirs[3 * di + 1],
                                    w2 = a.dirs[3 * di + 2];
                        const float *lt = a.lights + 6 * sc;
                        l0 = lt[0]; l1 = lt[1]; l2 = lt[2];
                        hx0 = fmaf(ht, w0, po0); hx1 = fmaf(ht, w1, po1); hx2 = fmaf(ht, w2, po2);
                        hit_normal<true>(s.lv, hx0, hx1, hx2, w0, w1, w2, n0, n1, n2);
                        const float ndl = fmaf(n2, l2, fmaf(n1, l1, n0 * l0));
                        if (ndl > 0.0f) {
                            o0 = fmaf(n0, s.bias, hx0);
                            o1 = fmaf(n1, s.bias, hx1);
                            o2 = fmaf(n2, s.bias, hx2);
                            d = lane_scene(s);
                            t = 0.0f;
                            k = 0;
                            mode = kBShadow;
                        } else {
                            vis = -1;
                            k = 0;
                            mode = kBPendShade;
                        }
                    }
                }
            }
            stepping = __ballot(mode == kBShadow);
            if (stepping == 0 && feed.exhausted) break;
        }
        if (mode == kBShadow) {
            float x0, x1, x2;
            int steps = 0;
            const int kind = batch_step<false>(d, o0, o1, o2, l0, l1, l2, t, k, x0, x1, x2, steps);
            if (kind >= 0) {
                vis = (kind == kHit || kind == kHitExhausted) ? 0 : 1;
                k = steps;
                mode = kBPendShade;
            }
        }
    }
    (void)info;
}

// One workgroup per kP probes of one scene (16 / kP workgroups per entry of the
// 16-probe block table): that scene's blend arguments, the shared precision-form
// blend body with the tile (kP, kChunk), then the scene's end stamp.
template <int kP, int kChunk>
__global__ __launch_bounds__(256) void batch_blend_kernel(BatchBlendArgs b) {
    constexpr int kSub = kBlendProbes / kP;
    const int2 blk = b.blocks[blockIdx.x / kSub];
    const int pb = blk.y + (int)(blockIdx.x % kSub) * kP;
    const BatchScene &s = b.scenes[blk.x];
    const size_t ti = (size_t)s.probe_base * 10 * 10 * 3, td = (size_t)s.probe_base * 18 * 18 * 2;
    BlendArgs a{};
    a.P = s.P;
    a.R = s.R;
    a.irr_res = 8;
    a.depth_res = 16;
    a.hysteresis = s.hysteresis;
    a.payload = b.payload + s.ray_base;
    a.Rpad = s.R;
    a.w16_i = s.w16_i;
    a.w16_d = s.w16_d;
    a.norm_i = s.norm_i;
    a.norm_d = s.norm_d;
    a.prev_irr = b.prev_irr + ti;
    a.prev_depth = b.prev_depth + td;
    a.new_irr = b.new_irr + ti;
    a.new_depth = b.new_depth + td;
    a.reject = b.reject + s.probe_base;
    blend16_block<true, kP, kChunk>(a, pb);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicMax(b.done + blk.x, (unsigned long long)wall_clock64());
    }
}

// ---------------------------------------------------------------- launchers --

template <int kChunk>
static hipError_t launch_primary_chunk(const BatchArgs &a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(batch_primary_kernel<kChunk>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int kChunk>
static hipError_t launch_hits_chunk(const BatchArgs &a, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(batch_hits_kernel<kChunk>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

bool batch_chunk_supported(int chunk, bool hits) {
    if (hits) return chunk == 16 || chunk == 32 || chunk == 64 || chunk == 128;
    return chunk == 64 || chunk == 128 || chunk == 256 || chunk == 512;
}

int batch_max_blocks(int device, bool hits) {
    int per_cu = 0, cus = 0;
    const void *k = hits ? (const void *)batch_hits_kernel<64> : (const void *)batch_primary_kernel<256>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus < 1)
        cus = 256;
    return per_cu * cus;
}

hipError_t launch_batch_begin(int *counter, unsigned long long *stamps, int n, hipStream_t s) {
    hipLaunchKernelGGL(batch_begin_kernel, dim3(1), dim3(64), 0, s, counter, stamps, n);
    return hipGetLastError();
}

hipError_t launch_batch_primary(const BatchArgs &a, const BatchTuning &t, hipStream_t s) {
    switch (t.primary_chunk) {
        case 64: return launch_primary_chunk<64>(a, t.primary_blocks, s);
        case 128: return launch_primary_chunk<128>(a, t.primary_blocks, s);
        case 256: return launch_primary_chunk<256>(a, t.primary_blocks, s);
        case 512: return launch_primary_chunk<512>(a, t.primary_blocks, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_hits(const BatchArgs &a, const BatchTuning &t, hipStream_t s) {
    switch (t.hits_chunk) {
        case 16: return launch_hits_chunk<16>(a, t.hits_blocks, s);
        case 32: return launch_hits_chunk<32>(a, t.hits_blocks, s);
        case 64: return launch_hits_chunk<64>(a, t.hits_blocks, s);
        case 128: return launch_hits_chunk<128>(a, t.hits_blocks, s);
        default: return hipErrorInvalidValue;
    }
}

template <int kP, int kChunk>
static hipError_t launch_blend_tile(const BatchBlendArgs &a, int nblocks16, hipStream_t s) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(batch_blend_kernel<kP, kChunk>),
                       dim3(nblocks16 * (kBlendProbes / kP)), dim3(256), 0, s, a);
    return hipGetLastError();
}

bool batch_blend_tile_supported(int probes, int chunk) {
    return (probes == 16 || probes == 8) && (chunk == 32 || chunk == 64 || chunk == 128);
}

hipError_t launch_batch_blend(const BatchBlendArgs &a, int nblocks16, const BatchTuning &t,
                              hipStream_t s) {
    if (nblocks16 <= 0) return hipSuccess;
    const int key = t.blend_probes * 1000 + t.blend_chunk;
    switch (key) {
        case 16032: return launch_blend_tile<16, 32>(a, nblocks16, s);
        case 16064: return launch_blend_tile<16, 64>(a, nblocks16, s);
        case 16128: return launch_blend_tile<16, 128>(a, nblocks16, s);
        case 8032: return launch_blend_tile<8, 32>(a, nblocks16, s);
        case 8064: return launch_blend_tile<8, 64>(a, nblocks16, s);
        case 8128: return launch_blend_tile<8, 128>(a, nblocks16, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sdfddgi
