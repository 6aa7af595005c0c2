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
#include "internal.h"
#include "octahedral.h"

#pragma clang fp contract(off)

namespace sdfddgi {

enum : int { kMissTmax = 0, kMissExit = 1, kHit = 2, kHitExhausted = 3, kInside = 4 };

__device__ __forceinline__ float clampf(float v, float lo, float hi) { return fminf(fmaxf(v, lo), hi); }

// ------------------------------------------------------------- geometry -----

// A cascade level as the trace loops read it, copied to LDS once per block. The
// binary32 constants were computed once in binary64 on the host.
struct LevelLds {
    const void *quad;              // corner quads [n2-1][n1-1][n0], float4 or half4
    const float *alb;              // albedo [n2][n1][n0][3] or nullptr
    float org0, org1, org2, inv;   // (float)origin, (float)(1/spacing)
    float cmax0, cmax1, cmax2;     // (float)(n-2): last cell index per axis
    float half;                    // (float)(spacing/2)
    uint32_t row, slice;           // quad strides: n0, n0*(n1-1)
    uint32_t arow, aslice;         // albedo strides: n0, n0*n1
};

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

// Cell and fraction of grid coordinate u along one axis (cell clamped to [0, cmax],
// cmax = vertices - 2). The int overload is deleted so a vertex count cannot be
// passed by mistake.
__device__ void cell_of(float u, int cmax, int &i, float &f) = delete;
__device__ __forceinline__ void cell_of(float u, float cmax, int &i, float &f) {
    const float fl = clampf(floorf(u), 0.0f, cmax);
    i = (int)fl;
    f = clampf(u - fl, 0.0f, 1.0f);
}

// Trilinear sample at grid coordinates (u0,u1,u2): lerps along x, then y, then z.
// The grid is stored as corner quads: quad (i,j,k) = the values at (i,j,k),
// (i,j+1,k), (i,j,k+1), (i,j+1,k+1), so a cell's eight corners are the two
// adjacent quads (i,j,k) and (i+1,j,k) -- usually one cache line.
// With kHalf the quads hold binary16 values (the precision form); they are widened
// exactly to binary32 and the arithmetic is unchanged.
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

template <bool kHalf>
__device__ __forceinline__ void load_quads(const void *base, uint32_t idx, float4 &a, float4 &b) {
    if (kHalf) {
        const half4_t *q = static_cast<const half4_t *>(base) + idx;
        const half4_t ha = q[0], hb = q[1];
        a = make_float4((float)ha.x, (float)ha.y, (float)ha.z, (float)ha.w);
        b = make_float4((float)hb.x, (float)hb.y, (float)hb.z, (float)hb.w);
    } else {
        const float4 *q = static_cast<const float4 *>(base) + idx;
        a = q[0];
        b = q[1];
    }
}

template <bool kHalf>
__device__ __forceinline__ float trilinear(const LevelLds &d, float u0, float u1, float u2) {
    int i0, i1, i2;
    float f0, f1, f2;
    cell_of(u0, d.cmax0, i0, f0);
    cell_of(u1, d.cmax1, i1, f1);
    cell_of(u2, d.cmax2, i2, f2);
    float4 a, b;
    load_quads<kHalf>(d.quad, (uint32_t)i2 * d.slice + (uint32_t)i1 * d.row + (uint32_t)i0, a, b);
    const float v000 = a.x, v010 = a.y, v001 = a.z, v011 = a.w;
    const float v100 = b.x, v110 = b.y, v101 = b.z, v111 = b.w;
    const float c00 = fmaf(f0, v100 - v000, v000);
    const float c10 = fmaf(f0, v110 - v010, v010);
    const float c01 = fmaf(f0, v101 - v001, v001);
    const float c11 = fmaf(f0, v111 - v011, v011);
    const float c0 = fmaf(f1, c10 - c00, c00);
    const float c1 = fmaf(f1, c11 - c01, c01);
    return fmaf(f2, c1 - c0, c0);
}

template <bool kHalf>
__device__ __forceinline__ float sample_at(const LevelLds &d, float p0, float p1, float p2) {
    return trilinear<kHalf>(d, (p0 - d.org0) * d.inv, (p1 - d.org1) * d.inv, (p2 - d.org2) * d.inv);
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

// Central differences at +-spacing/2 on the hit's level, normalised.
template <bool kHalf>
__device__ __forceinline__ void hit_normal(const LevelLds &d, float x0, float x1, float x2,
                                           float w0, float w1, float w2,
                                           float &n0, float &n1, float &n2) {
    const float h = d.half;
    float g[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const float p0 = x0 + (ax == 0 ? h : 0.0f), m0 = x0 - (ax == 0 ? h : 0.0f);
        const float p1 = x1 + (ax == 1 ? h : 0.0f), m1 = x1 - (ax == 1 ? h : 0.0f);
        const float p2 = x2 + (ax == 2 ? h : 0.0f), m2 = x2 - (ax == 2 ? h : 0.0f);
        g[ax] = sample_at<kHalf>(d, p0, p1, p2) - sample_at<kHalf>(d, m0, m1, m2);
    }
    const float g0 = g[0], g1 = g[1], g2 = g[2];
    const float len2 = fmaf(g2, g2, fmaf(g1, g1, g0 * g0));
    if (!(len2 >= 1e-24f)) { n0 = -w0; n1 = -w1; n2 = -w2; return; }
    const float inv = 1.0f / sqrtf(len2);
    n0 = g0 * inv; n1 = g1 * inv; n2 = g2 * inv;
}

// One sample of the fixed sphere-trace sequence for a ray o + t w at sample k.
// Returns the outcome code when the ray stops here (steps in *steps), -1 otherwise
// (t and k are then advanced). x and the level of the sample are returned too.
template <bool kPrimary, bool kHalf>
__device__ __forceinline__ int trace_step(const TraceArgs &a, const LevelLds *s_lv, float o0,
                                          float o1, float o2, float w0, float w1, float w2,
                                          float &t, int &k, float &x0, float &x1, float &x2,
                                          int &level, int &steps) {
    if (t > a.t_max) { steps = k; return kMissTmax; }
    x0 = fmaf(t, w0, o0); x1 = fmaf(t, w1, o1); x2 = fmaf(t, w2, o2);
    level = select_level(a, x0, x1, x2);
    if (level < 0) { steps = k; return kMissExit; }
    const LevelLds &d = s_lv[level];
    const float dist = trilinear<kHalf>(d, (x0 - d.org0) * d.inv, (x1 - d.org1) * d.inv,
                                        (x2 - d.org2) * d.inv);
    if (kPrimary && k == 0 && dist < 0.0f) { steps = 1; return kInside; }
    if (dist < a.eps) { steps = k + 1; return kHit; }
    t = fmaf(a.relax, dist, t);
    ++k;
    if (k == a.max_steps) { steps = k; return kHitExhausted; }
    return -1;
}

// ----------------------------------------------------------- radiometry -----

__device__ __forceinline__ float sgnf(float v) { return v >= 0.0f ? 1.0f : -1.0f; }

// Probe interpolation: trilinear over the 8 probes of x's cell, bilinear in each
// probe's padded octahedral tile at direction n.
__device__ __forceinline__ float3 interp_irradiance(const float *__restrict__ atlas, int res,
                                                   const ProbeGridDev &pg, float x0, float x1,
                                                   float x2, float n0, float n1, float n2) {
    int b0, b1, b2;
    float f0, f1, f2;
    cell_of((x0 - pg.org0) * pg.inv0, (float)(pg.n0 - 2), b0, f0);
    cell_of((x1 - pg.org1) * pg.inv1, (float)(pg.n1 - 2), b1, f1);
    cell_of((x2 - pg.org2) * pg.inv2, (float)(pg.n2 - 2), b2, f2);
    float l1 = fabsf(n0) + fabsf(n1) + fabsf(n2);
    float u = n0 / l1, v = n1 / l1;
    if (n2 < 0.0f) {
        float fu = (1.0f - fabsf(v)) * sgnf(u);
        float fv = (1.0f - fabsf(u)) * sgnf(v);
        u = fu; v = fv;
    }
    const float fres = (float)res;
    float su = (fres * (u + 1.0f) + 1.0f) * 0.5f;
    float sv = (fres * (v + 1.0f) + 1.0f) * 0.5f;
    float au = clampf(floorf(su), 0.0f, fres), av = clampf(floorf(sv), 0.0f, fres);
    float fu = clampf(su - au, 0.0f, 1.0f), fv = clampf(sv - av, 0.0f, 1.0f);
    const int side = res + 2;
    const int t00 = ((int)av * side + (int)au) * 3;
    const int tile = side * side * 3;
    const float w00 = (1.0f - fu) * (1.0f - fv), w10 = fu * (1.0f - fv);
    const float w01 = (1.0f - fu) * fv, w11 = fu * fv;
    float3 acc = make_float3(0.0f, 0.0f, 0.0f);
    // four probes per iteration: 48 loads in flight, a quarter of the registers of a
    // full unroll
#pragma unroll 4
    for (int c8 = 0; c8 < 8; ++c8) {
        const int dx = c8 & 1, dy = (c8 >> 1) & 1, dz = c8 >> 2;
        const float wp = (dx ? f0 : 1.0f - f0) * (dy ? f1 : 1.0f - f1) * (dz ? f2 : 1.0f - f2);
        const int p = (b0 + dx) + pg.n0 * ((b1 + dy) + pg.n1 * (b2 + dz));
        const float *tx = atlas + (size_t)p * tile + t00;
        const float *ty = tx + side * 3;
        acc.x += wp * (w00 * tx[0] + w10 * tx[3] + w01 * ty[0] + w11 * ty[3]);
        acc.y += wp * (w00 * tx[1] + w10 * tx[4] + w01 * ty[1] + w11 * ty[4]);
        acc.z += wp * (w00 * tx[2] + w10 * tx[5] + w01 * ty[2] + w11 * ty[5]);
    }
    return acc;
}

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

__device__ __forceinline__ void write_ray(const TraceArgs &a, int ray, float4 out, int kind,
                                          int level, int steps, int vis, int shadow_steps,
                                          float n0, float n1, float n2) {
    a.payload[ray] = out;
    if (a.records) {
        int4 *rec = reinterpret_cast<int4 *>(a.records) + 2 * (int64_t)ray;
        rec[0] = make_int4(kind | (level << 8), steps, vis, shadow_steps);
        rec[1] = make_int4(__float_as_int(out.w), __float_as_int(n0), __float_as_int(n1),
                           __float_as_int(n2));
    }
}

// Primary-ray hit record packing: outcome | level << 4 | steps << 8.
__device__ __forceinline__ int pack_hit(int kind, int level, int steps) {
    return kind | (level << 4) | (steps << 8);
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
constexpr int kRefillBelow = 40;  // refill / run batched work when fewer lanes are stepping

// Wave-level work feeder: claims `chunk` consecutive items per atomic and hands them
// to idle lanes in order. All members are wave-uniform.
template <int kChunkSize>
struct Feeder {
    int next = 0, end = 0;
    bool exhausted = false;
    // Returns the number of items given out; the rank-th idle lane takes first + rank.
    __device__ __forceinline__ int claim(int *counter, int total, int want, int &first) {
        if (next >= end) {
            int base = 0;
            if (__lane_id() == 0) base = atomicAdd(counter, kChunkSize);
            base = __builtin_amdgcn_readfirstlane(base);
            if (base >= total) { exhausted = true; return 0; }
            next = base;
            end = min(base + kChunkSize, total);
        }
        const int n = min(want, end - next);
        first = next;
        next += n;
        return n;
    }
};

// Primary sphere trace, persistent and wave-compacted: each lane owns one ray and
// takes one sample per iteration; when fewer than kRefillBelow lanes are stepping,
// idle lanes take the next rays (kChunk per global atomic: the rays of one probe,
// probes visited in Morton order of their grid cell). Misses and probes inside geometry write their payload here; hits are
// appended to a compact queue (ray, t, outcome, level, steps) for hits_kernel, staged
// per wave in LDS. Each ray's arithmetic is the fixed sequence of trace_step,
// whatever lane or wave runs it. Every wave exits once the counter has passed the
// last ray and its lanes are idle, after flushing its staged hits.
template <bool kHalf>
__global__ __launch_bounds__(256) void primary_kernel(TraceArgs a) {
    __shared__ LevelLds s_lv[kMaxLevels];
    __shared__ int4 s_hits[4][64];
    load_levels(a, s_lv);
    const int lane = (int)__lane_id();
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    int staged = 0;  // wave-uniform count of entries in s_hits[wave]
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int total = (a.probe_count ? *a.probe_count : a.P) * a.R;
    Feeder<kChunk> feed;
    bool active = false;
    int ray = 0, k = 0;
    float o0 = 0, o1 = 0, o2 = 0, w0 = 0, w1 = 0, w2 = 0, t = 0;
    while (true) {
        uint64_t stepping = __ballot(active);
        if (__popcll(stepping) < kRefillBelow) {
            uint64_t idle = ~stepping;
            while (idle != 0 && !feed.exhausted) {
                int first = 0;
                const int n = feed.claim(a.counter, total, __popcll(idle), first);
                const int rank = __popcll(idle & below);
                if (!active && rank < n) {
                    // slot -> (probe in Morton order, ray): neighbouring slots trace
                    // neighbouring probes, so the rays in flight share cache lines
                    const int slot = first + rank;
                    const int q = slot / a.R, i = slot - (slot / a.R) * a.R;
                    const int p = a.probe_order[q];
                    ray = p * a.R + i;
                    o0 = a.probe_pos[3 * p]; o1 = a.probe_pos[3 * p + 1]; o2 = a.probe_pos[3 * p + 2];
                    w0 = a.dirs[3 * i]; w1 = a.dirs[3 * i + 1]; w2 = a.dirs[3 * i + 2];
                    t = 0.0f;
                    k = 0;
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
            const int kind = trace_step<true, kHalf>(a, s_lv, o0, o1, o2, w0, w1, w2, t, k, x0,
                                                     x1, x2, level, steps);
            if (kind >= 0) {
                if (kind == kHit || kind == kHitExhausted) {
                    hit_now = true;
                    entry = make_int4(ray, __float_as_int(tt), pack_hit(kind, level, steps), 0);
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
template <bool kHalf>
__global__ __launch_bounds__(256) void hits_kernel(TraceArgs a) {
    __shared__ LevelLds s_lv[kMaxLevels];
    load_levels(a, s_lv);
    const int lane = (int)__lane_id();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int total = a.counter[2];  // queue length, final once primary_kernel has finished
    Feeder<kHitChunk> feed;

    int mode = kIdle, ray = 0, info = 0, k = 0, vis = -1;
    float ht = 0, hx0 = 0, hx1 = 0, hx2 = 0, n0 = 0, n1 = 0, n2 = 0;
    float o0 = 0, o1 = 0, o2 = 0, t = 0;
    while (true) {
        uint64_t stepping = __ballot(mode == kShadow);
        const int waiting = __popcll(__ballot(mode == kPendShade));
        if (__popcll(stepping) < kRefillBelow || waiting >= kShadeBatch) {
            for (int round = 0; round < 2; ++round) {
                if (__ballot(mode == kPendShade)) {
                    if (mode == kPendShade) {
                        // k holds the shadow ray's step count here
                        const LevelLds &d = s_lv[(info >> 4) & 15];
                        const float ndl = fmaf(n2, a.l2, fmaf(n1, a.l1, n0 * a.l0));
                        const float lit = vis == 1 ? ndl : 0.0f;
                        const float3 alb = albedo_at(a, d, hx0, hx1, hx2);
                        float3 ind = make_float3(0.0f, 0.0f, 0.0f);
                        if (a.gain != 0.0f)
                            ind = interp_irradiance(a.prev_irr, a.irr_res, a.pg, hx0, hx1, hx2, n0,
                                                    n1, n2);
                        const float inv_pi = 0.318309886183790671538f;
                        float4 out;
                        out.x = alb.x * inv_pi * (a.rad0 * lit + a.gain * ind.x);
                        out.y = alb.y * inv_pi * (a.rad1 * lit + a.gain * ind.y);
                        out.z = alb.z * inv_pi * (a.rad2 * lit + a.gain * ind.z);
                        out.w = ht;
                        write_ray(a, ray, out, info & 15, (info >> 4) & 15, info >> 8, vis, k, n0,
                                  n1, n2);
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
                        const int4 e = a.hitq[first + rank];
                        ray = e.x;
                        ht = __int_as_float(e.y);
                        info = e.z;
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
                        hit_normal<kHalf>(s_lv[(info >> 4) & 15], hx0, hx1, hx2, w0, w1, w2, n0, n1,
                                          n2);
                        const float ndl = fmaf(n2, a.l2, fmaf(n1, a.l1, n0 * a.l0));
                        if (ndl > 0.0f) {
                            o0 = fmaf(n0, a.bias, hx0);
                            o1 = fmaf(n1, a.bias, hx1);
                            o2 = fmaf(n2, a.bias, hx2);
                            t = 0.0f;
                            k = 0;
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
            const int kind = trace_step<false, kHalf>(a, s_lv, o0, o1, o2, a.l0, a.l1, a.l2, t,
                                                      k, x0, x1, x2, level, steps);
            if (kind >= 0) {
                vis = (kind == kHit || kind == kHitExhausted) ? 0 : 1;
                k = steps;
                mode = kPendShade;
            }
        }
    }
}

// One block per texel row of the weight matrices (irradiance rows, then depth
// rows), plus one block that writes the binary32 directions.
__global__ __launch_bounds__(256) void tables_kernel(TableArgs a) {
    __shared__ double red[256];
    const int row = blockIdx.x;
    const int tid = threadIdx.x;
    const bool is_dirs = row == a.Ti + a.Td;
    const bool is_depth = row >= a.Ti && !is_dirs;
    const int t = is_depth ? row - a.Ti : row;
    double nt0 = 0, nt1 = 0, nt2 = 0;
    if (!is_dirs) {
        const double *nt = is_depth ? a.texel_d + 3 * t : a.texel_i + 3 * t;
        nt0 = nt[0]; nt1 = nt[1]; nt2 = nt[2];
    }
    double part = 0.0;
    for (int i = tid; i < a.R; i += 256) {
        const double s0 = a.base[3 * i], s1 = a.base[3 * i + 1], s2 = a.base[3 * i + 2];
        const double w0 = a.q[0] * s0 + a.q[1] * s1 + a.q[2] * s2;
        const double w1 = a.q[3] * s0 + a.q[4] * s1 + a.q[5] * s2;
        const double w2 = a.q[6] * s0 + a.q[7] * s1 + a.q[8] * s2;
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
        if (tid < a.ncounter && a.counter) a.counter[tid] = 0;  // trace (and fallback) counters
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

constexpr int kBlendProbes = 16;  // probes per workgroup: the N extent of a tile row
typedef float floatx4 __attribute__((ext_vector_type(4)));

// The probes of one blend workgroup (slots pb .. pb+np-1 of the probe list, or of
// 0..P-1) and their hysteresis: none where the history is rejected. The first
// __syncthreads of the caller's ray loop publishes them.
__device__ __forceinline__ void load_blend_probes(const BlendArgs &a, int pb, int np, int *s_pid,
                                                  float *s_h) {
    const int tid = threadIdx.x;
    if (tid < kBlendProbes) {
        const int pid = tid < np ? (a.probe_list ? a.probe_list[pb + tid] : pb + tid) : 0;
        s_pid[tid] = pid;
        s_h[tid] = (tid < np && !(a.reject && a.reject[pid])) ? a.hysteresis : 0.0f;
    }
}

constexpr int kBlendChunk = 64;   // rays staged in LDS at a time
constexpr int kBlendPitch = kBlendChunk + 1;
constexpr int kMSlots = 5;        // 16-texel M-tiles per wave per pass

// Eq. 3 for 16 probes as a matrix product on MFMA (v_mfma_f32_16x16x4f32):
//   irradiance  U_i[t][(q,c)] = sum_k w_tk   * L[q][k][c]      (M = texels, N = 16 x RGB)
//   depth       U_d[t][(q,m)] = sum_k w_tk^s * t[q][k]^(m+1)   (M = texels, N = 16 x 2)
// with K = rays. The weights (shared by every probe of the frame) are the A operand,
// read from the transposed [R][T] tables; the probes' payload is the B operand,
// staged in LDS 64 rays at a time. M-tiles are dealt round-robin to the 4 waves, up
// to kMSlots per wave per pass (one pass covers 8x8 + 16x16 maps). The epilogue
// normalises, mixes with the previous interior (hysteresis, or none for rejected
// probes) and writes interior and border texels.
// Epilogue of both blend kernels for one 16x16 accumulator tile: lane holds
// D[4*krow + r][row]. Normalises, mixes with the previous interior (hysteresis, or
// none for rejected probes) and writes interior and border texels.
__device__ __forceinline__ void blend_epilogue(const BlendArgs &a, const float *s_h, const int *s_pid, int np,
                                               bool irr, int mtile, int n, int row, int krow,
                                               floatx4 acc) {
    const int res = irr ? a.irr_res : a.depth_res;
    const int T = res * res, comps = irr ? 3 : 2, side = res + 2;
    const int m0 = mtile * 16 + 4 * krow;
    const float *norm = irr ? a.norm_i : a.norm_d;
    const int col = n * 16 + row;
    const int q = irr ? col / 3 : col >> 1;
    const int c = irr ? col - 3 * q : col & 1;
    if (q >= np) return;
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
        const float u = acc[r] * nrm;
        const float v = nrm < 0.0f ? old : fmaf(h, old - u, u);
        store_with_border(new_tile, res, comps, i, j, c, v);
    }
}

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
constexpr int kPitch16 = kBlendChunk + 8;  // halves per LDS column (+8 spreads the banks)

// Precision form of the blend: the same tiling as blend_kernel, with the weights as
// FP16 (irradiance) / BF16 (depth) rows [T][Rpad] and the payload staged in LDS as
// FP16 radiance and BF16 (t, t^2) columns, contracted 32 rays at a time on
// v_mfma_f32_16x16x32_{f16,bf16} with FP32 accumulation.
template <bool kStd>
__global__ __launch_bounds__(256) void blend16_kernel(BlendArgs a) {
    __shared__ __attribute__((aligned(16))) _Float16 si[(kBlendProbes * 3 + 1) * kPitch16];
    __shared__ __attribute__((aligned(16))) __bf16 sd[(kBlendProbes * 2 + 1) * kPitch16];
    __shared__ float s_h[kBlendProbes];
    __shared__ int s_pid[kBlendProbes];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row = lane & 15, kgrp = lane >> 4;
    const int pb = blockIdx.x * kBlendProbes;
    const int count = a.probe_list ? min(*a.probe_count, a.P) : a.P;
    if (pb >= count) return;
    const int np = min(kBlendProbes, count - pb);
    const int Ti = a.irr_res * a.irr_res, Td = a.depth_res * a.depth_res;
    const int mti = (Ti + 15) >> 4, mtd = (Td + 15) >> 4;
    const int mtiles = mti + mtd;
    load_blend_probes(a, pb, np, s_pid, s_h);
    for (int e = tid; e < kPitch16; e += 256) {
        si[kBlendProbes * 3 * kPitch16 + e] = (_Float16)0.0f;
        sd[kBlendProbes * 2 * kPitch16 + e] = (__bf16)0.0f;
    }
    int bi_off[3], bd_off[2];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        const int col = n * 16 + row;
        bi_off[n] = (col / 3 < np ? col : kBlendProbes * 3) * kPitch16;
    }
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const int col = n * 16 + row;
        bd_off[n] = ((col >> 1) < np ? col : kBlendProbes * 2) * kPitch16;
    }
    const int passes = kStd ? 1 : (mtiles + 4 * kMSlots - 1) / (4 * kMSlots);
    for (int pass = 0; pass < passes; ++pass) {
        floatx4 acc[kMSlots][3];
        int mt[kMSlots];
        const _Float16 *wi[kMSlots];
        const __bf16 *wd[kMSlots];
#pragma unroll
        for (int s = 0; s < kMSlots; ++s) {
            mt[s] = pass * 4 * kMSlots + s * 4 + wave;
            const bool irr = kStd ? s == 0 : mt[s] < mti;
            wi[s] = a.w16_i + (size_t)(mt[s] * 16 + row) * a.Rpad;
            wd[s] = a.w16_d + (size_t)((irr ? 0 : mt[s] - mti) * 16 + row) * a.Rpad;
#pragma unroll
            for (int n = 0; n < 3; ++n) acc[s][n] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        }
        for (int k0 = 0; k0 < a.Rpad; k0 += kBlendChunk) {
            __syncthreads();
            const int kc = min(kBlendChunk, a.R - k0);  // rays present in this chunk
            for (int e = tid; e < kBlendProbes * kBlendChunk; e += 256) {
                const int q = e / kBlendChunk, kk = e - q * kBlendChunk;
                float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (q < np && kk < kc) v = a.payload[(size_t)s_pid[q] * a.R + k0 + kk];
                si[(q * 3 + 0) * kPitch16 + kk] = (_Float16)v.x;
                si[(q * 3 + 1) * kPitch16 + kk] = (_Float16)v.y;
                si[(q * 3 + 2) * kPitch16 + kk] = (_Float16)v.z;
                sd[(q * 2 + 0) * kPitch16 + kk] = (__bf16)v.w;
                sd[(q * 2 + 1) * kPitch16 + kk] = (__bf16)(v.w * v.w);
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < kBlendChunk; kk += 32) {
                const int kl = kk + 8 * kgrp;  // this lane's 8 rays within the chunk
                half8_t bi[3];
                bf16x8_t bd[2];
#pragma unroll
                for (int n = 0; n < 3; ++n)
                    bi[n] = *reinterpret_cast<const half8_t *>(&si[bi_off[n] + kl]);
#pragma unroll
                for (int n = 0; n < 2; ++n)
                    bd[n] = *reinterpret_cast<const bf16x8_t *>(&sd[bd_off[n] + kl]);
#pragma unroll
                for (int s = 0; s < kMSlots; ++s) {
                    if (kStd ? s == 0 : mt[s] < mti) {
                        const half8_t av = *reinterpret_cast<const half8_t *>(wi[s] + k0 + kl);
#pragma unroll
                        for (int n = 0; n < 3; ++n)
                            acc[s][n] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bi[n], acc[s][n], 0, 0, 0);
                    } else if (kStd || mt[s] < mtiles) {
                        const bf16x8_t av = *reinterpret_cast<const bf16x8_t *>(wd[s] + k0 + kl);
#pragma unroll
                        for (int n = 0; n < 2; ++n)
                            acc[s][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bd[n], acc[s][n], 0, 0, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < kMSlots; ++s) {
            if (!kStd && mt[s] >= mtiles) continue;
            const bool irr = kStd ? s == 0 : mt[s] < mti;
#pragma unroll
            for (int n = 0; n < 3; ++n) {
                if (!irr && n == 2) break;
                blend_epilogue(a, s_h, s_pid, np, irr, irr ? mt[s] : mt[s] - mti, n, row, kgrp,
                               acc[s][n]);
            }
        }
    }
    __syncthreads();
    if (tid < np && a.reject) a.reject[s_pid[tid]] = 0;
}

// kStd: the 8x8 irradiance + 16x16 depth layout (4 + 16 M-tiles, one pass), where
// slot 0 of every wave is an irradiance tile and slots 1..4 are depth tiles, known at
// compile time; other resolutions take the general instantiation.
template <bool kStd>
__global__ __launch_bounds__(256) void blend_kernel(BlendArgs a) {
    // payload of 16 probes x 4 channels x 64 rays, plus one zero row for absent probes
    __shared__ float sx[(kBlendProbes * 4 + 1) * kBlendPitch];
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
            for (int e = tid; e < kBlendProbes * kBlendChunk; e += 256) {
                const int q = e / kBlendChunk, kk = e - q * kBlendChunk;
                float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (q < np && kk < kc) v = a.payload[(size_t)s_pid[q] * a.R + k0 + kk];
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
    hipLaunchKernelGGL(tables_kernel, dim3(a.Ti + a.Td + 1), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Persistent grid: as many 256-thread blocks as fit on the device at once (fewer
// when there are fewer rays).
// Persistent grids: as many 256-thread blocks as fit on the device at once (fewer
// when there are fewer rays).
static int persistent_blocks(const void *kernel, int device, int64_t rays) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess)
        per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        cus = 1;
    const int64_t resident = (int64_t)(per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    const int64_t needed = blocks_for(rays, 256);
    return (int)(needed < resident ? needed : resident);
}

TraceGrid trace_grid(int device, int64_t rays, bool half) {
    TraceGrid g;
    g.primary_blocks = persistent_blocks(half ? (const void *)primary_kernel<true>
                                              : (const void *)primary_kernel<false>,
                                         device, rays);
    g.hits_blocks = persistent_blocks(half ? (const void *)hits_kernel<true>
                                           : (const void *)hits_kernel<false>,
                                      device, rays);
    return g;
}

hipError_t launch_primary(const TraceArgs &a, const TraceGrid &g, hipStream_t s) {
    if ((int64_t)a.P * a.R == 0) return hipSuccess;
    if (a.half_sdf)
        hipLaunchKernelGGL(primary_kernel<true>, dim3(g.primary_blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(primary_kernel<false>, dim3(g.primary_blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_hits(const TraceArgs &a, const TraceGrid &g, hipStream_t s) {
    if ((int64_t)a.P * a.R == 0) return hipSuccess;
    if (a.half_sdf)
        hipLaunchKernelGGL(hits_kernel<true>, dim3(g.hits_blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(hits_kernel<false>, dim3(g.hits_blocks), dim3(256), 0, s, a);
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

hipError_t launch_probe_sdf(const TraceArgs &a, float *out, hipStream_t s) {
    if (a.half_sdf)
        hipLaunchKernelGGL(probe_sdf_kernel<true>, dim3(blocks_for(a.P, 256)), dim3(256), 0, s, a, out);
    else
        hipLaunchKernelGGL(probe_sdf_kernel<false>, dim3(blocks_for(a.P, 256)), dim3(256), 0, s, a, out);
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
