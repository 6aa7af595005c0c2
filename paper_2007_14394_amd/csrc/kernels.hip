// gfx950 kernels of the SDFDDGI per-frame probe update (paper Sec. 3.3).
//
//   tables_kernel   frame ray directions (binary64 rotation of the fixed
//                   spherical-Fibonacci set, rounded once) and the Eq. 3 texel-by-
//                   ray weight matrices w_ti = max(0, n_t . w_i) and w_ti^s with
//                   their reciprocal row sums
//   trace_kernel    per ray: sphere trace, hit normal, SDF shadow ray, albedo,
//                   multi-bounce lookup into the previous atlas, payload (R,G,B,t)
//   blend_kernel    per probe: Eq. 3 ratio estimate for every texel, depth
//                   moments, temporal mix, octahedral border
//   sample_kernel   probe interpolation at arbitrary points and normals
//
// The geometric part of the trace (everything that decides an integer) follows
// one fixed binary32 operation sequence, spelled out with fmaf; contraction of
// any other multiply-add is disabled for this file.
#include "internal.h"

#pragma clang fp contract(off)

namespace sdfddgi {

enum : int { kMissTmax = 0, kMissExit = 1, kHit = 2, kHitExhausted = 3, kInside = 4 };

__device__ __forceinline__ float clampf(float v, float lo, float hi) { return fminf(fmaxf(v, lo), hi); }

// ------------------------------------------------------------- geometry -----

struct LevelView {
    const float *sdf;
    const float *alb;
    int n0, n1, n2;
    float org0, org1, org2, inv, half;
};

__device__ __forceinline__ void level_view(const DevLevel &d, LevelView &v) {
    v.sdf = d.sdf; v.alb = d.alb; v.n0 = d.n0; v.n1 = d.n1; v.n2 = d.n2;
    v.org0 = d.org0; v.org1 = d.org1; v.org2 = d.org2; v.inv = d.inv; v.half = d.half;
}

// Cell and fraction of grid coordinate u along one axis with n vertices.
__device__ __forceinline__ void cell_of(float u, int n, int &i, float &f) {
    float fl = clampf(floorf(u), 0.0f, (float)(n - 2));
    i = (int)fl;
    f = clampf(u - fl, 0.0f, 1.0f);
}

// Trilinear sample at grid coordinates (u0,u1,u2): lerps along x, then y, then z.
__device__ __forceinline__ float trilinear(const float *__restrict__ g, int n0, int n1, int n2,
                                           float u0, float u1, float u2) {
    int i0, i1, i2;
    float f0, f1, f2;
    cell_of(u0, n0, i0, f0);
    cell_of(u1, n1, i1, f1);
    cell_of(u2, n2, i2, f2);
    const uint32_t sy = (uint32_t)n0, sz = (uint32_t)n0 * (uint32_t)n1;
    const float *p = g + ((uint32_t)i2 * sz + (uint32_t)i1 * sy + (uint32_t)i0);
    float v000 = p[0], v100 = p[1], v010 = p[sy], v110 = p[sy + 1];
    float v001 = p[sz], v101 = p[sz + 1], v011 = p[sz + sy], v111 = p[sz + sy + 1];
    float c00 = fmaf(f0, v100 - v000, v000);
    float c10 = fmaf(f0, v110 - v010, v010);
    float c01 = fmaf(f0, v101 - v001, v001);
    float c11 = fmaf(f0, v111 - v011, v011);
    float c0 = fmaf(f1, c10 - c00, c00);
    float c1 = fmaf(f1, c11 - c01, c01);
    return fmaf(f2, c1 - c0, c0);
}

// Finest level whose box shrunk by one voxel holds x (the coarsest level with its
// full box); returns -1 outside the coarsest box. Fills the level and x's grid
// coordinates on it.
__device__ __forceinline__ int select_level(const TraceArgs &a, float x0, float x1, float x2,
                                            LevelView &lv, float &u0, float &u1, float &u2) {
#pragma unroll
    for (int L = 0; L < kMaxLevels; ++L) {
        if (L < a.nl) {
            const DevLevel &d = a.lv[L];
            const bool inner = L < a.nl - 1;
            const float lo = inner ? 1.0f : 0.0f;
            const int shrink = inner ? 2 : 1;
            float v0 = (x0 - d.org0) * d.inv;
            float v1 = (x1 - d.org1) * d.inv;
            float v2 = (x2 - d.org2) * d.inv;
            bool in = v0 >= lo && v0 <= (float)(d.n0 - shrink) && v1 >= lo &&
                      v1 <= (float)(d.n1 - shrink) && v2 >= lo && v2 <= (float)(d.n2 - shrink);
            if (in) {
                level_view(d, lv);
                u0 = v0; u1 = v1; u2 = v2;
                return L;
            }
        }
    }
    return -1;
}

struct TraceHit {
    int kind, steps, level;
    float t, x0, x1, x2;
};

// Sphere tracing along o + t w (Hart 1996; paper Sec. 3.3).
template <bool kPrimary>
__device__ __forceinline__ TraceHit trace_ray(const TraceArgs &a, float o0, float o1, float o2,
                                              float w0, float w1, float w2, LevelView &hit_lv) {
    TraceHit r;
    r.kind = kHitExhausted; r.steps = a.max_steps; r.level = -1;
    r.t = 0.0f; r.x0 = r.x1 = r.x2 = 0.0f;
    float t = 0.0f;
    for (int k = 0; k < a.max_steps; ++k) {
        if (t > a.t_max) { r.kind = kMissTmax; r.steps = k; return r; }
        float x0 = fmaf(t, w0, o0), x1 = fmaf(t, w1, o1), x2 = fmaf(t, w2, o2);
        LevelView lv;
        float u0, u1, u2;
        int L = select_level(a, x0, x1, x2, lv, u0, u1, u2);
        if (L < 0) { r.kind = kMissExit; r.steps = k; return r; }
        float d = trilinear(lv.sdf, lv.n0, lv.n1, lv.n2, u0, u1, u2);
        r.t = t; r.level = L; r.x0 = x0; r.x1 = x1; r.x2 = x2;
        if (kPrimary) hit_lv = lv;
        if (kPrimary && k == 0 && d < 0.0f) { r.kind = kInside; r.steps = 1; return r; }
        if (d < a.eps) { r.kind = kHit; r.steps = k + 1; return r; }
        t = fmaf(a.relax, d, t);
    }
    return r;
}

__device__ __forceinline__ float sample_at(const LevelView &lv, float p0, float p1, float p2) {
    return trilinear(lv.sdf, lv.n0, lv.n1, lv.n2, (p0 - lv.org0) * lv.inv,
                     (p1 - lv.org1) * lv.inv, (p2 - lv.org2) * lv.inv);
}

// Central differences at +-spacing/2 on the hit's level, normalised.
__device__ __forceinline__ void hit_normal(const LevelView &lv, float x0, float x1, float x2,
                                           float w0, float w1, float w2,
                                           float &n0, float &n1, float &n2) {
    const float h = lv.half;
    float g0 = sample_at(lv, x0 + h, x1, x2) - sample_at(lv, x0 - h, x1, x2);
    float g1 = sample_at(lv, x0, x1 + h, x2) - sample_at(lv, x0, x1 - h, x2);
    float g2 = sample_at(lv, x0, x1, x2 + h) - sample_at(lv, x0, x1, x2 - h);
    float len2 = fmaf(g2, g2, fmaf(g1, g1, g0 * g0));
    if (!(len2 >= 1e-24f)) { n0 = -w0; n1 = -w1; n2 = -w2; return; }
    float inv = 1.0f / sqrtf(len2);
    n0 = g0 * inv; n1 = g1 * inv; n2 = g2 * inv;
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
    cell_of((x0 - pg.org0) * pg.inv0, pg.n0, b0, f0);
    cell_of((x1 - pg.org1) * pg.inv1, pg.n1, b1, f1);
    cell_of((x2 - pg.org2) * pg.inv2, pg.n2, b2, f2);
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
    float w00 = (1.0f - fu) * (1.0f - fv), w10 = fu * (1.0f - fv);
    float w01 = (1.0f - fu) * fv, w11 = fu * fv;
    float3 acc = make_float3(0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                float wp = (dx ? f0 : 1.0f - f0) * (dy ? f1 : 1.0f - f1) * (dz ? f2 : 1.0f - f2);
                int p = (b0 + dx) + pg.n0 * ((b1 + dy) + pg.n1 * (b2 + dz));
                const float *tx = atlas + (size_t)p * tile + t00;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float s = w00 * tx[c] + w10 * tx[3 + c] + w01 * tx[side * 3 + c] +
                              w11 * tx[side * 3 + 3 + c];
                    if (c == 0) acc.x += wp * s;
                    if (c == 1) acc.y += wp * s;
                    if (c == 2) acc.z += wp * s;
                }
            }
    return acc;
}

__device__ __forceinline__ float3 albedo_at(const TraceArgs &a, const LevelView &lv, float x0,
                                            float x1, float x2) {
    if (!lv.alb) return make_float3(a.alb0, a.alb1, a.alb2);
    int i0, i1, i2;
    float f0, f1, f2;
    cell_of((x0 - lv.org0) * lv.inv, lv.n0, i0, f0);
    cell_of((x1 - lv.org1) * lv.inv, lv.n1, i1, f1);
    cell_of((x2 - lv.org2) * lv.inv, lv.n2, i2, f2);
    const uint32_t sy = (uint32_t)lv.n0, sz = (uint32_t)lv.n0 * (uint32_t)lv.n1;
    const float *p = lv.alb + 3u * ((uint32_t)i2 * sz + (uint32_t)i1 * sy + (uint32_t)i0);
    float out[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float v000 = p[c], v100 = p[3 + c], v010 = p[3 * sy + c], v110 = p[3 * (sy + 1) + c];
        float v001 = p[3 * sz + c], v101 = p[3 * (sz + 1) + c];
        float v011 = p[3 * (sz + sy) + c], v111 = p[3 * (sz + sy + 1) + c];
        float c00 = fmaf(f0, v100 - v000, v000), c10 = fmaf(f0, v110 - v010, v010);
        float c01 = fmaf(f0, v101 - v001, v001), c11 = fmaf(f0, v111 - v011, v011);
        float c0 = fmaf(f1, c10 - c00, c00), c1 = fmaf(f1, c11 - c01, c01);
        out[c] = fmaf(f2, c1 - c0, c0);
    }
    return make_float3(out[0], out[1], out[2]);
}

// ------------------------------------------------------------- kernels ------

__global__ __launch_bounds__(256) void trace_kernel(TraceArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)a.P * a.R;
    if (gid >= total) return;
    const int p = (int)(gid / a.R);
    const int i = (int)(gid - (int64_t)p * a.R);
    const float o0 = a.probe_pos[3 * p], o1 = a.probe_pos[3 * p + 1], o2 = a.probe_pos[3 * p + 2];
    const float w0 = a.dirs[3 * i], w1 = a.dirs[3 * i + 1], w2 = a.dirs[3 * i + 2];

    LevelView lv;
    TraceHit h = trace_ray<true>(a, o0, o1, o2, w0, w1, w2, lv);
    float n0 = 0.0f, n1 = 0.0f, n2 = 0.0f;
    int vis = -1, shadow_steps = 0;
    float4 out;
    const bool hit = h.kind == kHit || h.kind == kHitExhausted;
    if (hit) {
        hit_normal(lv, h.x0, h.x1, h.x2, w0, w1, w2, n0, n1, n2);
        float ndl = fmaf(n2, a.l2, fmaf(n1, a.l1, n0 * a.l0));
        if (ndl > 0.0f) {
            LevelView unused;
            TraceHit s = trace_ray<false>(a, fmaf(n0, a.bias, h.x0), fmaf(n1, a.bias, h.x1),
                                          fmaf(n2, a.bias, h.x2), a.l0, a.l1, a.l2, unused);
            vis = (s.kind == kHit || s.kind == kHitExhausted) ? 0 : 1;
            shadow_steps = s.steps;
        }
        float lit = vis == 1 ? ndl : 0.0f;
        float3 alb = albedo_at(a, lv, h.x0, h.x1, h.x2);
        float3 ind = make_float3(0.0f, 0.0f, 0.0f);
        if (a.gain != 0.0f)
            ind = interp_irradiance(a.prev_irr, a.irr_res, a.pg, h.x0, h.x1, h.x2, n0, n1, n2);
        const float inv_pi = 0.318309886183790671538f;
        out.x = alb.x * inv_pi * (a.rad0 * lit + a.gain * ind.x);
        out.y = alb.y * inv_pi * (a.rad1 * lit + a.gain * ind.y);
        out.z = alb.z * inv_pi * (a.rad2 * lit + a.gain * ind.z);
        out.w = h.t;
    } else if (h.kind == kInside) {
        out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    } else {
        out = make_float4(a.sky0, a.sky1, a.sky2, a.t_max);
    }
    a.payload[gid] = out;
    if (a.records) {
        int4 r0 = make_int4(h.kind | ((hit ? h.level : 0) << 8), h.steps, vis, shadow_steps);
        int4 r1 = make_int4(__float_as_int(out.w), __float_as_int(n0), __float_as_int(n1),
                            __float_as_int(n2));
        int4 *rec = reinterpret_cast<int4 *>(a.records) + 2 * gid;
        rec[0] = r0;
        rec[1] = r1;
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
            a.wt_d[(size_t)i * a.Td + t] = (float)w;
        } else {
            a.wt_i[(size_t)i * a.Ti + t] = (float)w;
        }
        part += w;
    }
    if (is_dirs) return;
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

// Source interior texel of padded texel (col a, row b) of an n x n map.
__device__ __forceinline__ void border_source(int n, int a, int b, int &i, int &j) {
    const bool left = a == 0, right = a == n + 1, top = b == 0, bottom = b == n + 1;
    if ((left || right) && (top || bottom)) { i = left ? n - 1 : 0; j = top ? n - 1 : 0; }
    else if (top || bottom) { i = n - a; j = top ? 0 : n - 1; }
    else if (left || right) { i = left ? 0 : n - 1; j = n - b; }
    else { i = a - 1; j = b - 1; }
}

// One block per probe: Eq. 3 for every texel from the probe's ray payload staged in
// LDS, temporal mix with the previous interior, border fill from LDS.
__global__ __launch_bounds__(256) void blend_kernel(BlendArgs a) {
    __shared__ float4 pl[kMaxRays];
    __shared__ float ti[kMaxRes * kMaxRes * 3];
    __shared__ float td[kMaxRes * kMaxRes * 2];
    const int p = blockIdx.x;
    const int tid = threadIdx.x;
    for (int i = tid; i < a.R; i += 256) pl[i] = a.payload[(size_t)p * a.R + i];
    __syncthreads();
    const float h = a.reject[p] ? 0.0f : a.hysteresis;
    const int ri = a.irr_res, rd = a.depth_res;
    const int Ti = ri * ri, Td = rd * rd;
    const int si = ri + 2, sd = rd + 2;
    const float *old_i = a.prev_irr + (size_t)p * si * si * 3;
    const float *old_d = a.prev_depth + (size_t)p * sd * sd * 2;
    for (int t = tid; t < Ti; t += 256) {
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
        for (int i = 0; i < a.R; ++i) {
            const float w = a.wt_i[(size_t)i * Ti + t];
            const float4 v = pl[i];
            s0 = fmaf(w, v.x, s0); s1 = fmaf(w, v.y, s1); s2 = fmaf(w, v.z, s2);
        }
        const float nrm = a.norm_i[t];
        const int at = ((t / ri + 1) * si + (t % ri + 1)) * 3;
        const float o0 = old_i[at], o1 = old_i[at + 1], o2 = old_i[at + 2];
        if (nrm < 0.0f) {
            ti[3 * t] = o0; ti[3 * t + 1] = o1; ti[3 * t + 2] = o2;
        } else {
            const float u0 = s0 * nrm, u1 = s1 * nrm, u2 = s2 * nrm;
            ti[3 * t] = fmaf(h, o0 - u0, u0);
            ti[3 * t + 1] = fmaf(h, o1 - u1, u1);
            ti[3 * t + 2] = fmaf(h, o2 - u2, u2);
        }
    }
    for (int t = tid; t < Td; t += 256) {
        float m1 = 0.0f, m2 = 0.0f;
        for (int i = 0; i < a.R; ++i) {
            const float w = a.wt_d[(size_t)i * Td + t];
            const float d = pl[i].w;
            m1 = fmaf(w, d, m1);
            m2 = fmaf(w, d * d, m2);
        }
        const float nrm = a.norm_d[t];
        const int at = ((t / rd + 1) * sd + (t % rd + 1)) * 2;
        const float o0 = old_d[at], o1 = old_d[at + 1];
        if (nrm < 0.0f) {
            td[2 * t] = o0; td[2 * t + 1] = o1;
        } else {
            const float u0 = m1 * nrm, u1 = m2 * nrm;
            td[2 * t] = fmaf(h, o0 - u0, u0);
            td[2 * t + 1] = fmaf(h, o1 - u1, u1);
        }
    }
    __syncthreads();
    float *out_i = a.new_irr + (size_t)p * si * si * 3;
    for (int k = tid; k < si * si; k += 256) {
        int i, j;
        border_source(ri, k % si, k / si, i, j);
        const int src = (j * ri + i) * 3;
        out_i[3 * k] = ti[src]; out_i[3 * k + 1] = ti[src + 1]; out_i[3 * k + 2] = ti[src + 2];
    }
    float *out_d = a.new_depth + (size_t)p * sd * sd * 2;
    for (int k = tid; k < sd * sd; k += 256) {
        int i, j;
        border_source(rd, k % sd, k / sd, i, j);
        const int src = (j * rd + i) * 2;
        out_d[2 * k] = td[src]; out_d[2 * k + 1] = td[src + 1];
    }
    if (tid == 0) a.reject[p] = 0;
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

hipError_t launch_trace(const TraceArgs &a, hipStream_t s) {
    const int64_t total = (int64_t)a.P * a.R;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(trace_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_blend(const BlendArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(blend_kernel, dim3(a.P), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sample(const SampleArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(sample_kernel, dim3(blocks_for(a.n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *dst, uint8_t value, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u8_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, dst, value, n);
    return hipGetLastError();
}

}  // namespace sdfddgi
