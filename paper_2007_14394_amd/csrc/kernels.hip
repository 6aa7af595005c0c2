// gfx950 kernels of the SDFDDGI per-frame probe update (paper Sec. 3.3).
//
//   tables_kernel   frame ray directions (binary64 rotation of the fixed
//                   spherical-Fibonacci set, rounded once) and the Eq. 3 texel-by-
//                   ray weight matrices w_ti = max(0, n_t . w_i) and w_ti^s with
//                   their reciprocal row sums
//   primary_kernel  per ray: primary sphere trace; payload of misses, hit records
//   hits_kernel     per hit: normal, SDF shadow ray, albedo, multi-bounce lookup into
//                   the previous atlas, payload (R,G,B,t)
//   blend_kernel    per probe: Eq. 3 ratio estimate for every texel, depth
//                   moments, temporal mix, octahedral border
//   sample_kernel   probe interpolation at arbitrary points and normals
//
// The geometric part of the trace (everything that decides an integer) follows
// one fixed binary32 operation sequence, spelled out with fmaf; contraction of
// any other multiply-add is disabled for this file.
#include <algorithm>

#include "internal.h"
#include "octahedral.h"
#include "trace_common.h"
#include "blend_common.h"
#include "analytic_common.h"

#pragma clang fp contract(off)

namespace sdfddgi {

// ------------------------------------------------------------- geometry -----

__device__ __forceinline__ void load_levels(const TraceArgs &a, LevelLds *s_lv) {
    if (threadIdx.x < kMaxLevels && (int)threadIdx.x < a.nl) {
        const DevLevel &d = a.lv[threadIdx.x];
        LevelLds v;
        v.quad = d.quad; v.alb = d.alb;
        v.org0 = d.org0; v.org1 = d.org1; v.org2 = d.org2; v.inv = d.inv;
        v.cmax0 = (float)(d.n0 - 2); v.cmax1 = (float)(d.n1 - 2); v.cmax2 = (float)(d.n2 - 2);
        v.half = d.half;
        v.row = (uint32_t)d.n0; v.slice = (uint32_t)d.n0 * (uint32_t)(d.n1 - 1);
        v.arow = (uint32_t)d.n0; v.aslice = (uint32_t)d.n0 * (uint32_t)d.n1;
        s_lv[threadIdx.x] = v;
    }
    __syncthreads();
}

// Finest level whose box, shrunk by one voxel (the coarsest level: its full box),
// holds x; -1 outside the coarsest box. The test "grid coordinate within [lo, hi]"
// is made on x itself against per-level bounds: u = (x - org) * inv is monotone in x,
// so the host finds the exact binary32 thresholds once and the result is the same.
__device__ __forceinline__ int select_level(const TraceArgs &a, float x0, float x1, float x2) {
    int L = -1;
#pragma unroll
    for (int l = kMaxLevels - 1; l >= 0; --l) {
        if (l < a.nl) {
            const DevLevel &d = a.lv[l];
            const bool in = (x0 >= d.xlo0) & (x0 <= d.xhi0) & (x1 >= d.xlo1) & (x1 <= d.xhi1) &
                            (x2 >= d.xlo2) & (x2 <= d.xhi2);
            L = in ? l : L;
        }
    }
    return L;
}

// Distance backends of the trace kernels: the cascade of grids with binary32 or
// binary16 values, or the scene's analytic primitives (Sec. 3.1) through the
// cluster-culled query of Sec. 3.3. The per-workgroup LDS state of each:
enum : int { kSdfGrid32 = 0, kSdfGrid16 = 1, kSdfAnalytic = 2 };
template <int kSdf> struct SdfLds { LevelLds lv[kMaxLevels]; };
template <> struct SdfLds<kSdfAnalytic> { ClusterLds cl; };

template <int kSdf>
__device__ __forceinline__ void load_sdf(const TraceArgs &a, SdfLds<kSdf> &s) {
    if constexpr (kSdf == kSdfAnalytic) load_clusters(a.an, s.cl);
    else load_levels(a, s.lv);
}

// One sample of the fixed sphere-trace sequence for a ray o + t w at sample k.
// Returns the outcome code when the ray stops here (steps in *steps), -1 otherwise
// (t and k are then advanced). x and the level of the sample are returned too.
// Analytic backend: no grid box, so a ray misses only past t_max; the distance is
// the culled minimum over the primitives, starting from `bound` (the previous
// sample's bound, +inf at a ray's first sample), and a primary ray's sample names
// its nearest primitive in `slot` (level is 0).
template <bool kPrimary, int kSdf>
__device__ __forceinline__ int trace_step(const TraceArgs &a, const SdfLds<kSdf> &s, float o0,
                                          float o1, float o2, float w0, float w1, float w2,
                                          float &t, int &k, float &x0, float &x1, float &x2,
                                          int &level, int &steps, float &bound, int &slot) {
    if (t > a.t_max) { steps = k; return kMissTmax; }
    x0 = fmaf(t, w0, o0); x1 = fmaf(t, w1, o1); x2 = fmaf(t, w2, o2);
    float dist;
    if constexpr (kSdf == kSdfAnalytic) {
        level = 0;
        if (kPrimary) {
            dist = nearest_distance(a.an, s.cl, x0, x1, x2, bound, slot);
        } else {
            uint32_t evals = 0;
            dist = scene_distance(a.an, s.cl, 2, x0, x1, x2, bound, evals);
        }
    } else {
        level = select_level(a, x0, x1, x2);
        if (level < 0) { steps = k; return kMissExit; }
        const LevelLds &d = s.lv[level];
        dist = trilinear<kSdf == kSdfGrid16>(d, (x0 - d.org0) * d.inv, (x1 - d.org1) * d.inv,
                                             (x2 - d.org2) * d.inv);
    }
    if (kPrimary && k == 0 && dist < 0.0f) { steps = 1; return kInside; }
    if (dist < a.eps) { steps = k + 1; return kHit; }
    t = fmaf(a.relax, dist, t);
    if constexpr (kSdf == kSdfAnalytic) bound = next_bound(a.relax, dist);
    ++k;
    if (k == a.max_steps) { steps = k; return kHitExhausted; }
    return -1;
}

// ----------------------------------------------------------- radiometry -----

__device__ __forceinline__ float3 albedo_at(const TraceArgs &a, const LevelLds &d, float x0,
                                            float x1, float x2) {
    if (!d.alb) return make_float3(a.alb0, a.alb1, a.alb2);
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

// ------------------------------------------------------------- kernels ------

__device__ __forceinline__ void write_record(const TraceArgs &a, int ray, float t, int kind,
                                             int level, int steps, int vis, int shadow_steps,
                                             float n0, float n1, float n2) {
    if (a.records) {
        int4 *rec = reinterpret_cast<int4 *>(a.records) + 2 * (int64_t)ray;
        rec[0] = make_int4(kind | (level << 8), steps, vis, shadow_steps);
        rec[1] = make_int4(__float_as_int(t), __float_as_int(n0), __float_as_int(n1),
                           __float_as_int(n2));
    }
}

__device__ __forceinline__ void write_ray(const TraceArgs &a, int ray, float4 out, int kind,
                                          int level, int steps, int vis, int shadow_steps,
                                          float n0, float n1, float n2) {
    a.payload[ray] = out;
    write_record(a, ray, out.w, kind, level, steps, vis, shadow_steps, n0, n1, n2);
}

// Payload of a hit: (albedo / pi) (sun radiance x n.l-or-0 + gain x multi-bounce), t.
__device__ __forceinline__ float4 shade_hit(const TraceArgs &a, float3 alb, float lit, float3 ind,
                                            float t) {
    const float inv_pi = 0.318309886183790671538f;
    float4 out;
    out.x = alb.x * inv_pi * (a.rad0 * lit + a.gain * ind.x);
    out.y = alb.y * inv_pi * (a.rad1 * lit + a.gain * ind.y);
    out.z = alb.z * inv_pi * (a.rad2 * lit + a.gain * ind.z);
    out.w = t;
    return out;
}

// Per-wave staging of hit-queue entries (ray, bits of t, packed info, 0) in LDS;
// flushed to the global queue 64 at a time with one atomic.
__device__ __forceinline__ void flush_hits(const TraceArgs &a, int4 *buf, int count) {
    if (count == 0) return;
    int base = 0;
    if (__lane_id() == 0) base = atomicAdd(a.counter + 2, count);
    base = __builtin_amdgcn_readfirstlane(base);
    const int lane = (int)__lane_id();
    if (lane < count) a.hitq[base + lane] = buf[lane];
    __builtin_amdgcn_wave_barrier();
}

constexpr int kChunk = 256;       // primary rays claimed from the global counter at a time
constexpr int kHitChunk = 64;     // queued hits claimed at a time (spreads them over all waves)
// Chunks per block of the XCD interleave (BlockFeeder): blocks of 256 probes keep
// the 8 XCDs on neighbouring blocks of the Morton order (one compact window for the
// shared Infinity Cache and HBM) with a compact region per L2. Measured at 16384 x 256
// (frame time, FP32 / FP16): one shared counter 0.862 / 0.758 ms; blocks of 1, 16,
// 64, 256, 512 chunks 0.844, 0.833, 0.823, 0.799, 0.802 / -, -, 0.669, 0.652, 0.666;
// one contiguous part per XCD (blocks of 2048) was 1.6x slower than one counter.
constexpr int kXcdBlock = 256;
constexpr int kRefillBelow = 32;  // refill / run batched work when fewer lanes are stepping
constexpr int kAnalyticBin = 64;  // probes whose rays of one direction the analytic trace groups

// Primary sphere trace, persistent and wave-compacted: each lane owns one ray and
// takes one sample per iteration; when fewer than kRefillBelow lanes are stepping,
// idle lanes take the next rays (kChunk per atomic: the rays of one probe, probes
// visited in Morton order of their grid cell, blocks of that order dealt to the XCDs
// in turn -- see BlockFeeder). Misses and probes inside geometry write their payload here; hits are
// appended to a compact queue (ray, t, outcome, level, steps) for hits_kernel, staged
// per wave in LDS. Each ray's arithmetic is the fixed sequence of trace_step,
// whatever lane or wave runs it. Every wave exits once the counter has passed the
// last ray and its lanes are idle, after flushing its staged hits.
template <int kSdf>
__global__ __launch_bounds__(256) void primary_kernel(TraceArgs a) {
    __shared__ SdfLds<kSdf> s_sdf;
    __shared__ int4 s_hits[4][64];
    load_sdf<kSdf>(a, s_sdf);
    const int lane = (int)__lane_id();
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    int staged = 0;  // wave-uniform count of entries in s_hits[wave]
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int total = (a.probe_count ? *a.probe_count : a.P) * a.R;
    BlockFeeder<kChunk, kXcdBlock> feed;
    feed.start();
    bool active = false;
    int ray = 0, k = 0, slot = -1;
    float o0 = 0, o1 = 0, o2 = 0, w0 = 0, w1 = 0, w2 = 0, t = 0, bound = INFINITY;
    while (true) {
        uint64_t stepping = __ballot(active);
        if (__popcll(stepping) < kRefillBelow) {
            uint64_t idle = ~stepping;
            while (idle != 0 && !feed.exhausted) {
                int first = 0;
                const int n = feed.claim(a.parts, total, __popcll(idle), first);
                const int rank = __popcll(idle & below);
                if (!active && rank < n) {
                    // slot -> (probe in Morton order, ray): neighbouring slots trace
                    // neighbouring probes, so the rays in flight share cache lines
                    const int sid = first + rank;
                    int q, i;
                    if constexpr (kSdf == kSdfAnalytic) {
                        // groups of kAnalyticBin probes of the Morton order, consecutive
                        // slots taking one direction across the group's probes: a wave's
                        // lanes march side by side from neighbouring probes, so the
                        // clusters that any lane's bound admits stay few
                        const int nq = total / a.R, gsz = kAnalyticBin * a.R;
                        const int g = sid / gsz, within = sid - g * gsz;
                        const int gq = min(kAnalyticBin, nq - g * kAnalyticBin);
                        i = within / gq;
                        q = g * kAnalyticBin + (within - i * gq);
                    } else {
                        q = sid / a.R;
                        i = sid - q * a.R;
                    }
                    const int p = a.probe_order[q];
                    ray = p * a.R + i;
                    o0 = a.probe_pos[3 * p]; o1 = a.probe_pos[3 * p + 1]; o2 = a.probe_pos[3 * p + 2];
                    w0 = a.dirs[3 * i]; w1 = a.dirs[3 * i + 1]; w2 = a.dirs[3 * i + 2];
                    t = 0.0f;
                    k = 0;
                    bound = INFINITY;
                    if (a.probe_first && a.max_steps > 1) {
                        // the first sample sits at the probe (fma(0, w, o) = o) for every
                        // ray of it: where that sample only steps on (a level holds the
                        // probe, or the primitives are traced; distance >= eps), take
                        // the step from the probe's precomputed sample; otherwise the
                        // first trace_step samples
                        const int2 f = a.probe_first[p];
                        const float d0 = __int_as_float(f.x);
                        if ((kSdf == kSdfAnalytic || f.y >= 0) && !(d0 < a.eps)) {
                            t = fmaf(a.relax, d0, 0.0f);
                            k = 1;
                            if constexpr (kSdf == kSdfAnalytic) {
                                bound = next_bound(a.relax, d0);
                                slot = f.y;
                            }
                        }
                    }
                    active = true;
                }
                idle = __ballot(!active);
            }
            stepping = __ballot(active);
            if (stepping == 0) {  // counter exhausted and every lane idle
                flush_hits(a, s_hits[wave], staged);
                break;
            }
        }
        bool hit_now = false;
        int4 entry = make_int4(0, 0, 0, 0);
        if (active) {
            const float tt = t;
            float x0, x1, x2;
            int level = 0, steps = 0;
            const int kind = trace_step<true, kSdf>(a, s_sdf, o0, o1, o2, w0, w1, w2, t, k, x0,
                                                    x1, x2, level, steps, bound, slot);
            if (kind >= 0) {
                if (kind == kHit || kind == kHitExhausted) {
                    hit_now = true;
                    entry = make_int4(ray, __float_as_int(tt), pack_hit(kind, level, steps),
                                      kSdf == kSdfAnalytic ? slot : 0);
                } else {
                    const float4 out = kind == kInside ? make_float4(0.0f, 0.0f, 0.0f, 0.0f)
                                                       : make_float4(a.sky0, a.sky1, a.sky2, a.t_max);
                    write_ray(a, ray, out, kind, 0, steps, -1, 0, 0.0f, 0.0f, 0.0f);
                }
                active = false;
            }
        }
        const uint64_t hm = __ballot(hit_now);
        if (hm) {
            const int n = __popcll(hm);
            if (staged + n > 64) {
                flush_hits(a, s_hits[wave], staged);
                staged = 0;
            }
            if (hit_now) s_hits[wave][staged + __popcll(hm & below)] = entry;
            __builtin_amdgcn_wave_barrier();
            staged += n;
            if (staged == 64) {
                flush_hits(a, s_hits[wave], staged);
                staged = 0;
            }
        }
    }
}

enum : int { kIdle = 0, kShadow = 1, kNew = 2, kPendShade = 3 };
constexpr int kShadeBatch = 16;   // shade when this many lanes wait (or stepping runs low)

// Hit rays from the queue the primary trace built: idle lanes take the next entries
// (kHitChunk per global atomic), then per lane: hit point and normal (batched for all
// newly assigned lanes), the SDF shadow ray toward the light (wave-compacted like the
// primary trace), and shading -- albedo, sun, multi-bounce lookup -- batched when
// kShadeBatch lanes wait or stepping runs low.
template <int kSdf>
__global__ __launch_bounds__(256) void hits_kernel(TraceArgs a) {
    __shared__ SdfLds<kSdf> s_sdf;
    load_sdf<kSdf>(a, s_sdf);
    const int lane = (int)__lane_id();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int total = a.counter[2];  // queue length, final once primary_kernel has finished
    Feeder<kHitChunk> feed;

    int mode = kIdle, ray = 0, info = 0, k = 0, vis = -1, slot = 0, qi = 0;
    float ht = 0, hx0 = 0, hx1 = 0, hx2 = 0, n0 = 0, n1 = 0, n2 = 0;
    float o0 = 0, o1 = 0, o2 = 0, t = 0, bound = INFINITY;
    while (true) {
        uint64_t stepping = __ballot(mode == kShadow);
        const int waiting = __popcll(__ballot(mode == kPendShade));
        if (__popcll(stepping) < kRefillBelow || waiting >= kShadeBatch) {
            for (int round = 0; round < 2; ++round) {
                if (__ballot(mode == kPendShade)) {
                    if (mode == kPendShade) {
                        // k holds the shadow ray's step count here
                        const float ndl = fmaf(n2, a.l2, fmaf(n1, a.l1, n0 * a.l0));
                        const float lit = vis == 1 ? ndl : 0.0f;
                        float3 alb;
                        if constexpr (kSdf == kSdfAnalytic)
                            alb = make_float3(a.prim_alb[3 * slot], a.prim_alb[3 * slot + 1],
                                              a.prim_alb[3 * slot + 2]);
                        else
                            alb = albedo_at(a, s_sdf.lv[(info >> 4) & 15], hx0, hx1, hx2);
                        if (a.geo) {
                            // 64-bit: 2 qi passes INT_MAX from 2^30 queued hits
                            a.geo[2 * (int64_t)qi] = make_float4(n0, n1, n2, lit);
                            a.geo[2 * (int64_t)qi + 1] = make_float4(alb.x, alb.y, alb.z, 0.0f);
                            write_record(a, ray, ht, info & 15, (info >> 4) & 15, info >> 8, vis,
                                         k, n0, n1, n2);
                        } else {
                            float3 ind = make_float3(0.0f, 0.0f, 0.0f);
                            if (a.gain != 0.0f)
                                ind = interp_irradiance(a.prev_irr, a.irr_res, a.pg, hx0, hx1,
                                                        hx2, n0, n1, n2);
                            write_ray(a, ray, shade_hit(a, alb, lit, ind, ht), info & 15,
                                      (info >> 4) & 15, info >> 8, vis, k, n0, n1, n2);
                        }
                        mode = kIdle;
                    }
                }
                if (round == 1) break;
                // refill idle lanes with entries of the hit queue
                uint64_t idle = __ballot(mode == kIdle);
                while (idle != 0 && !feed.exhausted) {
                    int first = 0;
                    const int n = feed.claim(a.counter + 1, total, __popcll(idle), first);
                    const int rank = __popcll(idle & below);
                    if (mode == kIdle && rank < n) {
                        qi = first + rank;
                        const int4 e = a.hitq[qi];
                        ray = e.x;
                        ht = __int_as_float(e.y);
                        info = e.z;
                        slot = e.w;
                        mode = kNew;
                    }
                    idle = __ballot(mode == kIdle);
                }
                // newly assigned hits: hit point, normal, shadow ray set-up
                if (__ballot(mode == kNew)) {
                    if (mode == kNew) {
                        const int p = ray / a.R, i = ray - (ray / a.R) * a.R;
                        const float po0 = a.probe_pos[3 * p], po1 = a.probe_pos[3 * p + 1],
                                    po2 = a.probe_pos[3 * p + 2];
                        const float w0 = a.dirs[3 * i], w1 = a.dirs[3 * i + 1], w2 = a.dirs[3 * i + 2];
                        hx0 = fmaf(ht, w0, po0); hx1 = fmaf(ht, w1, po1); hx2 = fmaf(ht, w2, po2);
                        if constexpr (kSdf == kSdfAnalytic)
                            analytic_normal(s_sdf.cl, slot, hx0, hx1, hx2, w0, w1, w2, n0, n1, n2);
                        else
                            hit_normal<kSdf == kSdfGrid16>(s_sdf.lv[(info >> 4) & 15], hx0, hx1,
                                                           hx2, w0, w1, w2, n0, n1, n2);
                        const float ndl = fmaf(n2, a.l2, fmaf(n1, a.l1, n0 * a.l0));
                        if (ndl > 0.0f) {
                            o0 = fmaf(n0, a.bias, hx0);
                            o1 = fmaf(n1, a.bias, hx1);
                            o2 = fmaf(n2, a.bias, hx2);
                            t = 0.0f;
                            k = 0;
                            bound = INFINITY;
                            mode = kShadow;
                        } else {
                            vis = -1;
                            k = 0;
                            mode = kPendShade;
                        }
                    }
                }
            }
            stepping = __ballot(mode == kShadow);
            if (stepping == 0 && feed.exhausted) break;
        }
        if (mode == kShadow) {
            float x0, x1, x2;
            int level = 0, steps = 0;
            int unused = 0;
            const int kind = trace_step<false, kSdf>(a, s_sdf, o0, o1, o2, a.l0, a.l1, a.l2, t,
                                                     k, x0, x1, x2, level, steps, bound, unused);
            if (kind >= 0) {
                vis = (kind == kHit || kind == kHitExhausted) ? 0 : 1;
                k = steps;
                mode = kPendShade;
            }
        }
    }
}

// Second half of split hit shading: per hit-queue entry, the hit point again (the
// same operations as hits_kernel), the multi-bounce lookup into the previous atlas
// and the payload. Grid-stride over the queue, whose length the primary trace left
// in counter[2].
__global__ __launch_bounds__(256) void shade_kernel(TraceArgs a) {
    const int total = a.counter[2];
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
        const int4 e = a.hitq[q];
        const float4 g0 = a.geo[2 * (int64_t)q], g1 = a.geo[2 * (int64_t)q + 1];
        const int ray = e.x;
        const float ht = __int_as_float(e.y);
        float3 ind = make_float3(0.0f, 0.0f, 0.0f);
        if (a.gain != 0.0f) {
            const int p = ray / a.R, i = ray - (ray / a.R) * a.R;
            const float hx0 = fmaf(ht, a.dirs[3 * i], a.probe_pos[3 * p]);
            const float hx1 = fmaf(ht, a.dirs[3 * i + 1], a.probe_pos[3 * p + 1]);
            const float hx2 = fmaf(ht, a.dirs[3 * i + 2], a.probe_pos[3 * p + 2]);
            ind = interp_irradiance(a.prev_irr, a.irr_res, a.pg, hx0, hx1, hx2, g0.x, g0.y, g0.z);
        }
        a.payload[ray] = shade_hit(a, make_float3(g1.x, g1.y, g1.z), g0.w, ind, ht);
    }
}

// One block per texel row of the weight matrices (irradiance rows, then depth
// rows), plus one block that writes the binary32 directions.
__global__ __launch_bounds__(256) void tables_kernel(TableArgs a) {
    __shared__ double red[256];
    const int row = blockIdx.x + a.row0;
    const int tid = threadIdx.x;
    const bool is_dirs = row == a.Ti + a.Td;
    const bool is_depth = row >= a.Ti && !is_dirs;
    const int t = is_depth ? row - a.Ti : row;
    double q[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) q[k] = a.q_dev ? a.q_dev[k] : a.q[k];
    double nt0 = 0, nt1 = 0, nt2 = 0;
    if (!is_dirs) {
        const double *nt = is_depth ? a.texel_d + 3 * t : a.texel_i + 3 * t;
        nt0 = nt[0]; nt1 = nt[1]; nt2 = nt[2];
    }
    double part = 0.0;
    for (int i = tid; i < a.R; i += 256) {
        const double s0 = a.base[3 * i], s1 = a.base[3 * i + 1], s2 = a.base[3 * i + 2];
        const double w0 = q[0] * s0 + q[1] * s1 + q[2] * s2;
        const double w1 = q[3] * s0 + q[4] * s1 + q[5] * s2;
        const double w2 = q[6] * s0 + q[7] * s1 + q[8] * s2;
        if (is_dirs) {
            a.dirs[3 * i] = (float)w0;
            a.dirs[3 * i + 1] = (float)w1;
            a.dirs[3 * i + 2] = (float)w2;
            continue;
        }
        double c = nt0 * w0 + nt1 * w1 + nt2 * w2;
        double w = c > 0.0 ? c : 0.0;
        if (is_depth) {
            w = pow(w, a.sharp);
            if (a.w16_d) {  // precision form: BF16 depth weights, sums of the rounded values
                const __bf16 b = (__bf16)(float)w;
                a.w16_d[(size_t)t * a.Rpad + i] = b;
                w = (double)(float)b;
            } else {
                a.wt_d[(size_t)i * a.Tpd + t] = (float)w;
            }
        } else {
            if (a.w16_i) {  // precision form: FP16 irradiance weights
                const _Float16 h = (_Float16)w;
                a.w16_i[(size_t)t * a.Rpad + i] = h;
                w = (double)(float)h;
            } else {
                a.wt_i[(size_t)i * a.Tpi + t] = (float)w;
            }
        }
        part += w;
    }
    if (is_dirs) {
        if (a.counter)  // trace (and fallback) counters
            for (int e = tid; e < a.ncounter; e += blockDim.x) a.counter[e] = 0;
        return;
    }
    red[tid] = part;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) {
        const double sum = red[0];
        const double pi = 3.14159265358979323846;
        if (is_depth) a.norm_d[t] = sum > 0.0 ? (float)(1.0 / sum) : -1.0f;
        else a.norm_i[t] = sum > 0.0 ? (float)(pi / sum) : -1.0f;
    }
}

template <bool kStd>
__global__ __launch_bounds__(256) void blend16_kernel(BlendArgs a) {
    blend16_block<kStd>(a, blockIdx.x * kBlendProbes);
}

// kStd: the 8x8 irradiance + 16x16 depth layout (4 + 16 M-tiles, one pass), where
// slot 0 of every wave is an irradiance tile and slots 1..4 are depth tiles, known at
// compile time; other resolutions take the general instantiation.
template <bool kStd>
__global__ __launch_bounds__(256) void blend_kernel(BlendArgs a) {
    // payload of 16 probes x 4 channels x 64 rays, plus one zero row for absent
    // probes; the standard layout's epilogue reuses the buffer
    constexpr int kStage = (kBlendProbes * 4 + 1) * kBlendPitch;
    __shared__ float sbuf[kStage > kEpilogueFloats ? kStage : kEpilogueFloats];
    float *sx = sbuf;
    __shared__ float s_h[kBlendProbes];
    __shared__ int s_pid[kBlendProbes];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row = lane & 15, krow = lane >> 4;
    const int pb = blockIdx.x * kBlendProbes;
    const int count = a.probe_list ? min(*a.probe_count, a.P) : a.P;
    if (pb >= count) return;
    const int np = min(kBlendProbes, count - pb);
    const int ri = a.irr_res, rd = a.depth_res;
    const int Ti = ri * ri, Td = rd * rd;
    const int mti = (Ti + 15) >> 4, mtd = (Td + 15) >> 4;
    const int Tpi = mti * 16, Tpd = mtd * 16;   // padded rows of the weight tables
    const int mtiles = mti + mtd;
    const int si = ri + 2, sd = rd + 2;
    constexpr int kZeroRow = kBlendProbes * 4 * kBlendPitch;
    load_blend_probes(a, pb, np, s_pid, s_h);
    for (int e = tid; e < kBlendPitch; e += 256) sx[kZeroRow + e] = 0.0f;

    // B-operand columns of this lane: irradiance (q, c) for 3 N-tiles, depth (q, m) for 2
    int bi_off[3], bd_off[2];
    bool bd_sq[2];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        const int col = n * 16 + row, q = col / 3, c = col - 3 * (col / 3);
        bi_off[n] = q < np ? (q * 4 + c) * kBlendPitch : kZeroRow;
    }
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const int col = n * 16 + row, q = col >> 1;
        bd_off[n] = q < np ? (q * 4 + 3) * kBlendPitch : kZeroRow;
        bd_sq[n] = (col & 1) != 0;
    }

    const int passes = kStd ? 1 : (mtiles + 4 * kMSlots - 1) / (4 * kMSlots);
    for (int pass = 0; pass < passes; ++pass) {
        floatx4 acc[kMSlots][3];
        int mt[kMSlots];          // wave-uniform M-tile of each slot
        const float *wcol[kMSlots];
        int wstride[kMSlots];
#pragma unroll
        for (int s = 0; s < kMSlots; ++s) {
            mt[s] = pass * 4 * kMSlots + s * 4 + wave;
            const bool irr = kStd ? s == 0 : mt[s] < mti;
            wcol[s] = irr ? a.wt_i + mt[s] * 16 + row : a.wt_d + (mt[s] - mti) * 16 + row;
            wstride[s] = irr ? Tpi : Tpd;
#pragma unroll
            for (int n = 0; n < 3; ++n) acc[s][n] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        }
        for (int k0 = 0; k0 < a.R; k0 += kBlendChunk) {
            __syncthreads();
            const int kc = min(kBlendChunk, a.R - k0);
            // every read of the chunk issued at once (absent probes and rays read a
            // present one and are zeroed)
            constexpr int kLoads = kBlendProbes * kBlendChunk / 256;
            float4 pv[kLoads];
#pragma unroll
            for (int b = 0; b < kLoads; ++b) {
                const int e = tid + 256 * b, q = e / kBlendChunk, kk = e - q * kBlendChunk;
                pv[b] = a.payload[(size_t)s_pid[min(q, np - 1)] * a.R + k0 + min(kk, kc - 1)];
            }
#pragma unroll
            for (int b = 0; b < kLoads; ++b) {
                const int e = tid + 256 * b, q = e / kBlendChunk, kk = e - q * kBlendChunk;
                const float4 v = (q < np && kk < kc) ? pv[b] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                float *d = sx + q * 4 * kBlendPitch + kk;
                d[0] = v.x; d[kBlendPitch] = v.y; d[2 * kBlendPitch] = v.z; d[3 * kBlendPitch] = v.w;
            }
            __syncthreads();
            float a_cur[kMSlots], a_nxt[kMSlots];
#pragma unroll
            for (int s = 0; s < kMSlots; ++s)
                a_cur[s] = (kStd || mt[s] < mtiles) ? wcol[s][(size_t)(k0 + krow) * wstride[s]] : 0.0f;
            for (int kk = 0; kk < kc; kk += 4) {
                const int kl = kk + krow;
                if (kk + 4 < kc) {
#pragma unroll
                    for (int s = 0; s < kMSlots; ++s)
                        a_nxt[s] = (kStd || mt[s] < mtiles) ? wcol[s][(size_t)(k0 + kl + 4) * wstride[s]]
                                                            : 0.0f;
                }
                float bi[3], bd[2];
#pragma unroll
                for (int n = 0; n < 3; ++n) bi[n] = sx[bi_off[n] + kl];
#pragma unroll
                for (int n = 0; n < 2; ++n) {
                    const float tv = sx[bd_off[n] + kl];
                    bd[n] = bd_sq[n] ? tv * tv : tv;
                }
#pragma unroll
                for (int s = 0; s < kMSlots; ++s) {
                    if (kStd ? s == 0 : mt[s] < mti) {
#pragma unroll
                        for (int n = 0; n < 3; ++n)
                            acc[s][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_cur[s], bi[n], acc[s][n], 0, 0, 0);
                    } else if (kStd || mt[s] < mtiles) {
#pragma unroll
                        for (int n = 0; n < 2; ++n)
                            acc[s][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_cur[s], bd[n], acc[s][n], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int s = 0; s < kMSlots; ++s) a_cur[s] = a_nxt[s];
            }
        }
        // epilogue: lane holds D[4*krow + r][row] of each tile
        if (kStd) {
            blend_epilogue_std<false, 3, 2, true>(a, s_h, s_pid, np, wave, row, krow, acc, sbuf);
            continue;
        }
#pragma unroll
        for (int s = 0; s < kMSlots; ++s) {
            if (!kStd && mt[s] >= mtiles) continue;
            const bool irr = kStd ? s == 0 : mt[s] < mti;
            const int res = irr ? ri : rd, T = irr ? Ti : Td, comps = irr ? 3 : 2;
            const int side = irr ? si : sd;
            const int m0 = (irr ? mt[s] : mt[s] - mti) * 16 + 4 * krow;
            const float *norm = irr ? a.norm_i : a.norm_d;
#pragma unroll
            for (int n = 0; n < 3; ++n) {
                if (!irr && n == 2) break;
                const int col = n * 16 + row;
                const int q = irr ? col / 3 : col >> 1;
                const int c = irr ? col - 3 * q : col & 1;
                if (q >= np) continue;
                const size_t tile_floats = (size_t)side * side * comps;
                const float *old_tile = (irr ? a.prev_irr : a.prev_depth) + (size_t)s_pid[q] * tile_floats;
                float *new_tile = (irr ? a.new_irr : a.new_depth) + (size_t)s_pid[q] * tile_floats;
                const float h = s_h[q];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int t = m0 + r;
                    if (t >= T) continue;
                    const int i = t % res, j = t / res;
                    const float nrm = norm[t];
                    const float old = old_tile[((j + 1) * side + (i + 1)) * comps + c];
                    const float u = acc[s][n][r] * nrm;
                    const float v = nrm < 0.0f ? old : fmaf(h, old - u, u);
                    store_with_border(new_tile, res, comps, i, j, c, v);
                }
            }
        }
    }
    __syncthreads();
    if (tid < np && a.reject) a.reject[s_pid[tid]] = 0;
}

// Alg. 1 per probe: from the grid position, while the distance is below t1 (at most
// `iterations` times) take a Newton step t1 - d along the normalised distance
// gradient (the hit-normal rule; +y where it vanishes), each coordinate kept within
// the offset of the grid position; stop outside every level. Then compare with the
// last position and reject the history of a probe that moved more than t2.
template <bool kHalf>
__global__ __launch_bounds__(256) void relocate_kernel(TraceArgs a, RelocateArgs r) {
    __shared__ LevelLds s_lv[kMaxLevels];
    load_levels(a, s_lv);
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    const float g0 = r.grid_pos[3 * p], g1 = r.grid_pos[3 * p + 1], g2 = r.grid_pos[3 * p + 2];
    const float lo0 = g0 - r.off0, lo1 = g1 - r.off1, lo2 = g2 - r.off2;
    const float hi0 = g0 + r.off0, hi1 = g1 + r.off1, hi2 = g2 + r.off2;
    float x0 = g0, x1 = g1, x2 = g2;
    for (int it = 0; it < r.iterations; ++it) {
        const int L = select_level(a, x0, x1, x2);
        if (L < 0) break;
        const float d = sample_at<kHalf>(s_lv[L], x0, x1, x2);
        if (!(d < r.t1)) break;
        float n0, n1, n2;
        hit_normal<kHalf>(s_lv[L], x0, x1, x2, 0.0f, -1.0f, 0.0f, n0, n1, n2);
        const float step = r.t1 - d;
        x0 = fminf(fmaxf(fmaf(step, n0, x0), lo0), hi0);
        x1 = fminf(fmaxf(fmaf(step, n1, x1), lo1), hi1);
        x2 = fminf(fmaxf(fmaf(step, n2, x2), lo2), hi2);
    }
    const float dx = x0 - r.pos[3 * p], dy = x1 - r.pos[3 * p + 1], dz = x2 - r.pos[3 * p + 2];
    const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    if (d2 > r.t2 * r.t2) r.reject[p] = 1;
    r.pos[3 * p] = x0;
    r.pos[3 * p + 1] = x1;
    r.pos[3 * p + 2] = x2;
}

// Signed distance at each probe position: the trace's own level choice and sampler.
template <bool kHalf>
__global__ __launch_bounds__(256) void probe_sdf_kernel(TraceArgs a, float *out) {
    __shared__ LevelLds s_lv[kMaxLevels];
    load_levels(a, s_lv);
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    const float x0 = a.probe_pos[3 * p], x1 = a.probe_pos[3 * p + 1], x2 = a.probe_pos[3 * p + 2];
    const int L = select_level(a, x0, x1, x2);
    out[p] = L < 0 ? 1e30f : sample_at<kHalf>(s_lv[L], x0, x1, x2);
}

// Each probe's first sample: the level its position selects and the distance there,
// by the same sequence as a ray's sample at t = 0.
template <bool kHalf>
__global__ __launch_bounds__(256) void probe_first_kernel(TraceArgs a, int2 *out) {
    __shared__ LevelLds s_lv[kMaxLevels];
    load_levels(a, s_lv);
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    const float x0 = a.probe_pos[3 * p], x1 = a.probe_pos[3 * p + 1], x2 = a.probe_pos[3 * p + 2];
    const int L = select_level(a, x0, x1, x2);
    const float d = L < 0 ? 0.0f : sample_at<kHalf>(s_lv[L], x0, x1, x2);
    out[p] = make_int2(__float_as_int(d), L);
}

// The same for the analytic backend: the culled query's distance at the probe from an
// unbounded start, and the nearest primitive's slot.
__global__ __launch_bounds__(256) void probe_first_analytic_kernel(TraceArgs a, int2 *out) {
    __shared__ ClusterLds s_cl;
    load_clusters(a.an, s_cl);
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    int slot = -1;
    const float d = nearest_distance(a.an, s_cl, a.probe_pos[3 * p], a.probe_pos[3 * p + 1],
                                     a.probe_pos[3 * p + 2], INFINITY, slot);
    out[p] = make_int2(__float_as_int(d), slot);
}

__global__ __launch_bounds__(256) void sample_kernel(SampleArgs a) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.n) return;
    float3 e = interp_irradiance(a.atlas, a.irr_res, a.pg, a.points[3 * q], a.points[3 * q + 1],
                                 a.points[3 * q + 2], a.normals[3 * q], a.normals[3 * q + 1],
                                 a.normals[3 * q + 2]);
    a.out[3 * q] = e.x;
    a.out[3 * q + 1] = e.y;
    a.out[3 * q + 2] = e.z;
}

// Corner-quad repacking of one grid level (see trilinear). The binary16 form clamps
// each value to +-65504 and rounds it to nearest even.
__device__ __forceinline__ _Float16 to_half(float v) {
    return (_Float16)fminf(fmaxf(v, -65504.0f), 65504.0f);
}

__global__ __launch_bounds__(256) void pack_quads_half_kernel(const float *__restrict__ g, int n0,
                                                              int n1, int n2,
                                                              half4_t *__restrict__ quad) {
    const int64_t total = (int64_t)n0 * (n1 - 1) * (n2 - 1);
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int i = (int)(q % n0);
    const int j = (int)((q / n0) % (n1 - 1));
    const int k = (int)(q / ((int64_t)n0 * (n1 - 1)));
    const int64_t sy = n0, sz = (int64_t)n0 * n1;
    const int64_t v = k * sz + j * sy + i;
    half4_t h;
    h.x = to_half(g[v]); h.y = to_half(g[v + sy]); h.z = to_half(g[v + sz]); h.w = to_half(g[v + sz + sy]);
    quad[q] = h;
}

__global__ __launch_bounds__(256) void pack_quads_kernel(const float *__restrict__ g, int n0, int n1,
                                                         int n2, float4 *__restrict__ quad) {
    const int64_t total = (int64_t)n0 * (n1 - 1) * (n2 - 1);
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int i = (int)(q % n0);
    const int j = (int)((q / n0) % (n1 - 1));
    const int k = (int)(q / ((int64_t)n0 * (n1 - 1)));
    const int64_t sy = n0, sz = (int64_t)n0 * n1;
    const int64_t v = k * sz + j * sy + i;
    quad[q] = make_float4(g[v], g[v + sy], g[v + sz], g[v + sz + sy]);
}

__global__ __launch_bounds__(256) void fill_u8_kernel(uint8_t *dst, uint8_t value, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = value;
}

// ------------------------------------------------------------ launchers -----

static unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_tables(const TableArgs &a, hipStream_t s) {
    TableArgs t = a;
    t.row0 = 0;
    hipLaunchKernelGGL(tables_kernel, dim3(t.Ti + t.Td + 1), dim3(256), 0, s, t);
    return hipGetLastError();
}

hipError_t launch_tables_dirs(TableArgs a, hipStream_t s) {
    a.row0 = a.Ti + a.Td;
    hipLaunchKernelGGL(tables_kernel, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tables_weights(TableArgs a, hipStream_t s) {
    a.row0 = 0;
    hipLaunchKernelGGL(tables_kernel, dim3(a.Ti + a.Td), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Persistent grids: as many 256-thread blocks as fit on the device at once, at most
// max_per_cu per compute unit (fewer when there are fewer rays). A block is one wave
// per SIMD.
static int persistent_blocks(const void *kernel, int device, int64_t rays, int max_per_cu) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess)
        per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        cus = 1;
    per_cu = std::max(1, std::min(per_cu, max_per_cu));
    const int64_t resident = (int64_t)per_cu * (cus > 0 ? cus : 1);
    const int64_t needed = blocks_for(rays, 256);
    return (int)(needed < resident ? needed : resident);
}

// The trace kernels are bound by how often the SDF lines of the rays in flight are
// found in the L2 (each XCD's 4 MB serves its own CUs): more resident waves hide more
// latency but evict each other's lines. Measured on the open scene at 16384 x 256
// rays, in both precisions, the primary trace is fastest with 4 waves per SIMD (of
// the 7 that fit) and the hit shading with 2 (of 4) when it runs alone,
// 1 when it runs beside the next frame's primary trace. Beside the other frames'
// work the primary trace also does best with 4 waves per SIMD: with the hit shading
// split (its atlas-independent half beside the trace), frame period 0.692 ms vs
// 0.704 with 3 and 0.802 with 2 (binary32), 0.574 ms vs 0.618 with 3 (binary16);
// before that split the binary32 trace had preferred 3 (0.742 vs 0.770 ms).
constexpr int kPrimaryBlocksPerCu = 4;
constexpr int kPrimaryBlocksPerCuOverlapped[2] = {4, 4};  // binary32, binary16 SDF
constexpr int kHitsBlocksPerCu = 2;
constexpr int kHitsBlocksPerCuOverlapped = 1;

TraceGrid trace_grid(int device, int64_t rays, bool half, bool analytic) {
    TraceGrid g;
    const void *pk = analytic ? (const void *)primary_kernel<kSdfAnalytic>
                     : half   ? (const void *)primary_kernel<kSdfGrid16>
                              : (const void *)primary_kernel<kSdfGrid32>;
    g.primary_blocks = persistent_blocks(pk, device, rays, kPrimaryBlocksPerCu);
    g.primary_blocks_overlapped =
        persistent_blocks(pk, device, rays, kPrimaryBlocksPerCuOverlapped[half ? 1 : 0]);
    const void *hk = analytic ? (const void *)hits_kernel<kSdfAnalytic>
                     : half   ? (const void *)hits_kernel<kSdfGrid16>
                              : (const void *)hits_kernel<kSdfGrid32>;
    g.hits_blocks = persistent_blocks(hk, device, rays, kHitsBlocksPerCu);
    g.hits_blocks_overlapped = persistent_blocks(hk, device, rays, kHitsBlocksPerCuOverlapped);
    return g;
}

hipError_t launch_primary(const TraceArgs &a, const TraceGrid &g, hipStream_t s) {
    if ((int64_t)a.P * a.R == 0) return hipSuccess;
    if (a.analytic)
        hipLaunchKernelGGL(primary_kernel<kSdfAnalytic>, dim3(g.primary_blocks), dim3(256), 0, s,
                           a);
    else if (a.half_sdf)
        hipLaunchKernelGGL(primary_kernel<kSdfGrid16>, dim3(g.primary_blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(primary_kernel<kSdfGrid32>, dim3(g.primary_blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_hits(const TraceArgs &a, const TraceGrid &g, hipStream_t s) {
    if ((int64_t)a.P * a.R == 0) return hipSuccess;
    if (a.analytic)
        hipLaunchKernelGGL(hits_kernel<kSdfAnalytic>, dim3(g.hits_blocks), dim3(256), 0, s, a);
    else if (a.half_sdf)
        hipLaunchKernelGGL(hits_kernel<kSdfGrid16>, dim3(g.hits_blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(hits_kernel<kSdfGrid32>, dim3(g.hits_blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_shade(const TraceArgs &a, hipStream_t s) {
    if ((int64_t)a.P * a.R == 0) return hipSuccess;
    const int64_t threads = (int64_t)a.P * a.R;
    // four workgroups per CU of the 256-CU part, striding over the queue
    const int blocks = (int)std::min<int64_t>((threads + 255) / 256, 1024);
    hipLaunchKernelGGL(shade_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_blend(const BlendArgs &a, hipStream_t s) {
    const dim3 grid(blocks_for(a.P, kBlendProbes)), block(256);
    if (a.w16_i) {
        if (a.irr_res == 8 && a.depth_res == 16)
            hipLaunchKernelGGL(blend16_kernel<true>, grid, block, 0, s, a);
        else
            hipLaunchKernelGGL(blend16_kernel<false>, grid, block, 0, s, a);
        return hipGetLastError();
    }
    if (a.irr_res == 8 && a.depth_res == 16)
        hipLaunchKernelGGL(blend_kernel<true>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(blend_kernel<false>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_relocate(const TraceArgs &a, const RelocateArgs &r, hipStream_t s) {
    if (a.half_sdf)
        hipLaunchKernelGGL(relocate_kernel<true>, dim3(blocks_for(a.P, 256)), dim3(256), 0, s, a, r);
    else
        hipLaunchKernelGGL(relocate_kernel<false>, dim3(blocks_for(a.P, 256)), dim3(256), 0, s, a, r);
    return hipGetLastError();
}

hipError_t launch_probe_sdf(const TraceArgs &a, float *out, hipStream_t s) {
    if (a.half_sdf)
        hipLaunchKernelGGL(probe_sdf_kernel<true>, dim3(blocks_for(a.P, 256)), dim3(256), 0, s, a, out);
    else
        hipLaunchKernelGGL(probe_sdf_kernel<false>, dim3(blocks_for(a.P, 256)), dim3(256), 0, s, a, out);
    return hipGetLastError();
}

hipError_t launch_probe_first(const TraceArgs &a, int2 *out, hipStream_t s) {
    if (a.analytic)
        hipLaunchKernelGGL(probe_first_analytic_kernel, dim3(blocks_for(a.P, 256)), dim3(256), 0,
                           s, a, out);
    else if (a.half_sdf)
        hipLaunchKernelGGL(probe_first_kernel<true>, dim3(blocks_for(a.P, 256)), dim3(256), 0, s, a,
                           out);
    else
        hipLaunchKernelGGL(probe_first_kernel<false>, dim3(blocks_for(a.P, 256)), dim3(256), 0, s,
                           a, out);
    return hipGetLastError();
}

hipError_t launch_sample(const SampleArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(sample_kernel, dim3(blocks_for(a.n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pack_quads(const float *g, int n0, int n1, int n2, bool half, void *quad,
                             hipStream_t s) {
    const int64_t total = (int64_t)n0 * (n1 - 1) * (n2 - 1);
    if (half)
        hipLaunchKernelGGL(pack_quads_half_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, g,
                           n0, n1, n2, static_cast<half4_t *>(quad));
    else
        hipLaunchKernelGGL(pack_quads_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, g, n0,
                           n1, n2, static_cast<float4 *>(quad));
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *dst, uint8_t value, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u8_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, dst, value, n);
    return hipGetLastError();
}

}  // namespace sdfddgi
