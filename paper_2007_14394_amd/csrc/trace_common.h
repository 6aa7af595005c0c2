// Device code shared by the trace kernels of one scene (kernels.hip) and of a
// batch of scenes (batch.hip): the cascade level as the loops read it, the
// trilinear sampler and its fixed binary32 lerp sequence, the hit normal, the
// probe interpolation, and the wave-level work feeder.
#pragma once

#include "internal.h"

namespace sdfddgi {

enum : int { kMissTmax = 0, kMissExit = 1, kHit = 2, kHitExhausted = 3, kInside = 4 };

__device__ __forceinline__ float clampf(float v, float lo, float hi) { return fminf(fmaxf(v, lo), hi); }

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

// Primary-ray hit record packing: outcome | level << 4 | steps << 8.
__device__ __forceinline__ int pack_hit(int kind, int level, int steps) {
    return kind | (level << 4) | (steps << 8);
}

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

// The XCD (accelerator complex die) the calling wave runs on, from the hardware
// register that holds it; each XCD has its own L2.
__device__ __forceinline__ int xcd_id() {
    return __builtin_amdgcn_s_getreg((3 << 11) | 20) & (kXcds - 1);  // HW_REG_XCC_ID, 4 bits
}

// Work handed out so that every XCD walks the same region of the item order at the
// same time (the order is coherent in space, so the device-wide working set stays
// small) while each XCD's L2 sees runs of neighbouring items: the order is cut into
// blocks of kBlock chunks of kChunkSize items, block b belongs to XCD b mod kXcds,
// and each XCD claims the chunks of its blocks in order from a counter of its own
// (parts[x * kPartStride]). A wave starts on its XCD's counter and moves on to the
// next XCD's once that one is used up; a counter, once used up, stays so, so a wave
// that has found kXcds used up in a row has seen them all and reports exhausted.

template <int kChunkSize, int kBlock>
struct BlockFeeder {
    int next = 0, end = 0, part = 0, misses = 0;
    bool exhausted = false;
    __device__ __forceinline__ void start() { part = xcd_id(); }
    // Returns the number of items given out; the rank-th idle lane takes first + rank.
    __device__ __forceinline__ int claim(int *parts, int total, int want, int &first) {
        while (next >= end) {
            if (misses == kXcds) { exhausted = true; return 0; }
            int s = 0;
            if (__lane_id() == 0) s = atomicAdd(parts + part * kPartStride, 1);
            s = __builtin_amdgcn_readfirstlane(s);
            const int64_t chunk = ((int64_t)(s / kBlock) * kXcds + part) * kBlock + s % kBlock;
            const int64_t base = chunk * kChunkSize;
            if (base >= total) {
                part = part + 1 == kXcds ? 0 : part + 1;
                ++misses;
                continue;
            }
            next = (int)base;
            end = (int)min(base + kChunkSize, (int64_t)total);
        }
        const int n = min(want, end - next);
        first = next;
        next += n;
        return n;
    }
};

}  // namespace sdfddgi
