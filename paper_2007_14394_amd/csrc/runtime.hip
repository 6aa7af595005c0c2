// Host runtime of libsdfddgi: argument validation, device memory, per-frame
// constants and stream-ordered launches behind the C ABI of include/sdfddgi.h.
//
// Per-frame host work is one binary64 rotation matrix (SplitMix64 + Shoemake);
// the fixed spherical-Fibonacci set, the texel directions and the probe
// positions are computed once at create, in binary64, and uploaded.
#include "sdfddgi.h"
#include "internal.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

using namespace sdfddgi;

namespace {

thread_local std::string g_create_error;

constexpr double kPi = 3.14159265358979323846;
constexpr int kTimingRing = 256;
constexpr int kEvents = 5;

// ---------------------------------------------------------- frame constants --

// SplitMix64 (Steele, Lea, Flood 2014): Weyl increment then a 64-bit finaliser.
uint64_t splitmix_next(uint64_t &state) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double unit_from(uint64_t &state) { return (double)(splitmix_next(state) >> 11) * 0x1.0p-53; }

// Shoemake's uniform random rotation: quaternion (x,y,z,w) from three uniforms,
// then its row-major rotation matrix.
void rotation_matrix(uint64_t seed, double m[9]) {
    uint64_t st = seed;
    const double u1 = unit_from(st);
    const double u2 = unit_from(st);
    const double u3 = unit_from(st);
    const double two_pi = 2.0 * kPi;
    const double r1 = std::sqrt(1.0 - u1), r2 = std::sqrt(u1);
    const double a1 = two_pi * u2, a2 = two_pi * u3;
    const double x = r1 * std::sin(a1), y = r1 * std::cos(a1);
    const double z = r2 * std::sin(a2), w = r2 * std::cos(a2);
    m[0] = 1.0 - 2.0 * (y * y + z * z);
    m[1] = 2.0 * (x * y - z * w);
    m[2] = 2.0 * (x * z + y * w);
    m[3] = 2.0 * (x * y + z * w);
    m[4] = 1.0 - 2.0 * (x * x + z * z);
    m[5] = 2.0 * (y * z - x * w);
    m[6] = 2.0 * (x * z - y * w);
    m[7] = 2.0 * (y * z + x * w);
    m[8] = 1.0 - 2.0 * (x * x + y * y);
}

// Unrotated spherical-Fibonacci point k of R (binary64).
void fibonacci_point(int k, int R, double s[3]) {
    const double golden_conj = (std::sqrt(5.0) - 1.0) * 0.5;
    const double two_pi = 2.0 * kPi;
    const double z = 1.0 - (2.0 * (double)k + 1.0) / (double)R;
    const double r = std::sqrt(1.0 - z * z);
    const double g = (double)k * golden_conj;
    const double phi = two_pi * (g - std::floor(g));
    s[0] = r * std::cos(phi);
    s[1] = r * std::sin(phi);
    s[2] = z;
}

double sign_of(double v) { return v >= 0.0 ? 1.0 : -1.0; }

// Centre direction of interior texel (i, j) of an n x n octahedral map (binary64).
void texel_direction(int n, int i, int j, double d[3]) {
    double u = ((double)i + 0.5) / (double)n * 2.0 - 1.0;
    double v = ((double)j + 0.5) / (double)n * 2.0 - 1.0;
    double z = 1.0 - std::fabs(u) - std::fabs(v);
    if (z < 0.0) {
        const double fu = (1.0 - std::fabs(v)) * sign_of(u);
        const double fv = (1.0 - std::fabs(u)) * sign_of(v);
        u = fu;
        v = fv;
    }
    const double len = std::sqrt(u * u + v * v + z * z);
    d[0] = u / len;
    d[1] = v / len;
    d[2] = z / len;
}

bool finite_all(const float *v, int n) {
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(v[k])) return false;
    return true;
}

}  // namespace

struct sdfddgi_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    sdfddgi_params prm{};
    int nl = 0;
    int n[kMaxLevels][3]{};
    double origin[kMaxLevels][3]{};
    double spacing[kMaxLevels]{};
    void *quad[kMaxLevels]{};    // corner-quad repacking of each level's grid
    bool half = false;           // precision form: quads in binary16
    float *alb[kMaxLevels]{};
    sdfddgi_probe_grid pg{};
    int64_t P = 0;
    int R = 0, Ti = 0, Td = 0, Tpi = 0, Tpd = 0;
    int64_t irr_floats = 0, depth_floats = 0;
    float *probe_pos = nullptr;
    int *probe_order = nullptr;
    double *base_dirs = nullptr, *texel_i = nullptr, *texel_d = nullptr;
    float *dirs = nullptr, *wt_i = nullptr, *wt_d = nullptr, *norm_i = nullptr, *norm_d = nullptr;
    _Float16 *w16_i = nullptr;   // precision-form weight tables [T][Rpad]
    __bf16 *w16_d = nullptr;
    int Rpad = 0;
    float *irr[2]{}, *depth[2]{};
    int cur = 0;
    uint8_t *reject = nullptr;
    int *counter = nullptr;
    int4 *hitq = nullptr;
    TraceGrid grid;
    float4 *payload = nullptr;
    int *records = nullptr;
    bool have_frame = false, have_records = false;
    // Timing: kEvents events per frame (before tables, after tables, after the
    // primary trace, after the hit kernel, after the blend) in a ring;
    // sdfddgi_get_kernel_times averages the frames recorded since its previous call.
    hipEvent_t *ev_ring = nullptr;
    int ring_head = 0;
    int64_t timed_frames = 0;
    std::string err;
};

namespace {

sdfddgi_status fail(sdfddgi_ctx *c, sdfddgi_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_create_error = buf;
    return s;
}

sdfddgi_status hip_fail(sdfddgi_ctx *c, hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory)
        return fail(c, SDFDDGI_ENOMEM, "%s: out of device memory", what);
    return fail(c, SDFDDGI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

template <typename T>
hipError_t dev_alloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return hipSuccess;
    return hipMalloc((void **)p, count * sizeof(T));
}

void free_all(sdfddgi_ctx *c) {
    for (int L = 0; L < kMaxLevels; ++L) {
        if (c->quad[L]) (void)hipFree(c->quad[L]);
        if (c->alb[L]) (void)hipFree(c->alb[L]);
    }
    void *bufs[] = {c->probe_pos, c->probe_order, c->base_dirs, c->texel_i, c->texel_d, c->dirs, c->wt_i,
                    c->wt_d, c->norm_i, c->norm_d, c->w16_i, c->w16_d, c->irr[0], c->irr[1], c->depth[0],
                    c->depth[1], c->reject, c->counter, c->hitq, c->payload, c->records};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (c->ev_ring) {
        for (int k = 0; k < kEvents * kTimingRing; ++k)
            if (c->ev_ring[k]) (void)hipEventDestroy(c->ev_ring[k]);
        delete[] c->ev_ring;
    }
}

sdfddgi_status validate(const sdfddgi_sdf_grid *sdf, const sdfddgi_probe_grid *pg,
                        const sdfddgi_params *p) {
    if (!sdf || !pg || !p) return fail(nullptr, SDFDDGI_EINVAL, "null argument");
    if (sdf->num_levels < 1 || sdf->num_levels > kMaxLevels)
        return fail(nullptr, SDFDDGI_EINVAL, "num_levels %d not in 1..%d", sdf->num_levels,
                    kMaxLevels);
    for (int L = 0; L < sdf->num_levels; ++L) {
        const sdfddgi_sdf_level &lv = sdf->level[L];
        int64_t cnt = 1;
        for (int c = 0; c < 3; ++c) {
            if (lv.n[c] < 2) return fail(nullptr, SDFDDGI_EINVAL, "level %d: n[%d] < 2", L, c);
            if (!std::isfinite(lv.origin[c]))
                return fail(nullptr, SDFDDGI_EINVAL, "level %d: non-finite origin", L);
            cnt *= lv.n[c];
        }
        if (cnt * 4 >= (int64_t)1 << 31)
            return fail(nullptr, SDFDDGI_EINVAL, "level %d: grid too large", L);
        if (!(lv.spacing > 0.0) || !std::isfinite(lv.spacing))
            return fail(nullptr, SDFDDGI_EINVAL, "level %d: spacing must be finite and > 0", L);
        if (!lv.sdf) return fail(nullptr, SDFDDGI_EINVAL, "level %d: sdf is NULL", L);
    }
    int64_t P = 1;
    for (int c = 0; c < 3; ++c) {
        if (pg->n[c] < 2) return fail(nullptr, SDFDDGI_EINVAL, "probe grid n[%d] < 2", c);
        if (!(pg->spacing[c] > 0.0) || !std::isfinite(pg->spacing[c]) ||
            !std::isfinite(pg->origin[c]))
            return fail(nullptr, SDFDDGI_EINVAL, "probe grid spacing/origin invalid");
        P *= pg->n[c];
    }
    const int R = p->rays_per_probe;
    if (R < 16 || R > kMaxRays || R % 16)
        return fail(nullptr, SDFDDGI_EINVAL, "rays_per_probe %d: need a multiple of 16 in 16..%d",
                    R, kMaxRays);
    if (P * R >= (int64_t)1 << 31) return fail(nullptr, SDFDDGI_EINVAL, "probes x rays too large");
    if (p->max_steps < 1 || p->max_steps > 4096)
        return fail(nullptr, SDFDDGI_EINVAL, "max_steps %d not in 1..4096", p->max_steps);
    if (p->irr_res < 2 || p->irr_res > kMaxRes || p->depth_res < 2 || p->depth_res > kMaxRes)
        return fail(nullptr, SDFDDGI_EINVAL, "map resolution not in 2..%d", kMaxRes);
    const float scalars[] = {p->hit_eps, p->t_max, p->hysteresis, p->bounce_gain,
                             p->depth_sharpness, p->shadow_bias, p->relax};
    if (!finite_all(scalars, 7) || !finite_all(p->sky_rgb, 3) || !finite_all(p->albedo, 3))
        return fail(nullptr, SDFDDGI_EINVAL, "non-finite parameter");
    if (!(p->hit_eps > 0) || !(p->t_max > 0))
        return fail(nullptr, SDFDDGI_EINVAL, "hit_eps and t_max must be > 0");
    if (!(p->hysteresis >= 0 && p->hysteresis < 1))
        return fail(nullptr, SDFDDGI_EINVAL, "hysteresis must be in [0,1)");
    if (!(p->bounce_gain >= 0 && p->bounce_gain <= 1))
        return fail(nullptr, SDFDDGI_EINVAL, "bounce_gain must be in [0,1]");
    if (!(p->depth_sharpness >= 0) || !(p->shadow_bias >= 0))
        return fail(nullptr, SDFDDGI_EINVAL, "depth_sharpness and shadow_bias must be >= 0");
    if (!(p->relax > 0 && p->relax <= 2))
        return fail(nullptr, SDFDDGI_EINVAL, "relax must be in (0,2]");
    for (int c = 0; c < 3; ++c)
        if (p->sky_rgb[c] < 0 || p->albedo[c] < 0)
            return fail(nullptr, SDFDDGI_EINVAL, "sky and albedo must be >= 0");
    return SDFDDGI_OK;
}

// Monotone integer key of a binary32 value (orders all finite floats).
int32_t float_key(float f) {
    int32_t b;
    std::memcpy(&b, &f, 4);
    return b >= 0 ? b : -(b & 0x7fffffff);
}

float key_float(int32_t k) {
    int32_t b = k >= 0 ? k : (int32_t)(0x80000000u | (uint32_t)(-k));
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

// Grid coordinate of x exactly as the kernels compute it.
float grid_coord(float x, float org, float inv) {
    volatile float d = x - org;  // one binary32 subtraction, then one multiplication
    return d * inv;
}

// Smallest float x with grid_coord(x) >= lo (the map is monotone in x); -inf / +inf
// when every / no finite float qualifies.
float lower_bound_x(float org, float inv, float lo) {
    int64_t a = float_key(-FLT_MAX), b = float_key(FLT_MAX);
    if (grid_coord(key_float((int32_t)a), org, inv) >= lo) return -INFINITY;
    if (!(grid_coord(key_float((int32_t)b), org, inv) >= lo)) return INFINITY;
    while (b - a > 1) {
        const int32_t m = (int32_t)(a + (b - a) / 2);
        if (grid_coord(key_float(m), org, inv) >= lo) b = m;
        else a = m;
    }
    return key_float((int32_t)b);
}

// Largest float x with grid_coord(x) <= hi.
float upper_bound_x(float org, float inv, float hi) {
    int64_t a = float_key(-FLT_MAX), b = float_key(FLT_MAX);
    if (grid_coord(key_float((int32_t)b), org, inv) <= hi) return INFINITY;
    if (!(grid_coord(key_float((int32_t)a), org, inv) <= hi)) return -INFINITY;
    while (b - a > 1) {
        const int32_t m = (int32_t)(a + (b - a) / 2);
        if (grid_coord(key_float(m), org, inv) <= hi) a = m;
        else b = m;
    }
    return key_float((int32_t)a);
}

DevLevel dev_level(const sdfddgi_ctx *c, int L) {
    DevLevel d{};
    d.quad = c->quad[L];
    d.alb = c->alb[L];
    d.n0 = c->n[L][0];
    d.n1 = c->n[L][1];
    d.n2 = c->n[L][2];
    d.org0 = (float)c->origin[L][0];
    d.org1 = (float)c->origin[L][1];
    d.org2 = (float)c->origin[L][2];
    d.inv = (float)(1.0 / c->spacing[L]);
    d.half = (float)(0.5 * c->spacing[L]);
    const bool inner = L < c->nl - 1;
    const float org[3] = {d.org0, d.org1, d.org2};
    float lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        const float ulo = inner ? 1.0f : 0.0f;
        const float uhi = (float)(c->n[L][k] - (inner ? 2 : 1));
        lo[k] = lower_bound_x(org[k], d.inv, ulo);
        hi[k] = upper_bound_x(org[k], d.inv, uhi);
    }
    d.xlo0 = lo[0]; d.xlo1 = lo[1]; d.xlo2 = lo[2];
    d.xhi0 = hi[0]; d.xhi1 = hi[1]; d.xhi2 = hi[2];
    return d;
}

ProbeGridDev dev_probes(const sdfddgi_ctx *c) {
    ProbeGridDev g{};
    g.n0 = c->pg.n[0];
    g.n1 = c->pg.n[1];
    g.n2 = c->pg.n[2];
    g.org0 = (float)c->pg.origin[0];
    g.org1 = (float)c->pg.origin[1];
    g.org2 = (float)c->pg.origin[2];
    g.inv0 = (float)(1.0 / c->pg.spacing[0]);
    g.inv1 = (float)(1.0 / c->pg.spacing[1]);
    g.inv2 = (float)(1.0 / c->pg.spacing[2]);
    return g;
}

TableArgs table_args(const sdfddgi_ctx *c, uint64_t seed) {
    TableArgs t{};
    t.R = c->R;
    t.Ti = c->Ti;
    t.Td = c->Td;
    t.Tpi = c->Tpi;
    t.Tpd = c->Tpd;
    rotation_matrix(seed, t.q);
    t.sharp = (double)c->prm.depth_sharpness;
    t.base = c->base_dirs;
    t.texel_i = c->texel_i;
    t.texel_d = c->texel_d;
    t.dirs = c->dirs;
    t.wt_i = c->wt_i;
    t.wt_d = c->wt_d;
    t.norm_i = c->norm_i;
    t.norm_d = c->norm_d;
    t.counter = c->counter;
    t.Rpad = c->Rpad;
    t.w16_i = c->w16_i;
    t.w16_d = c->w16_d;
    return t;
}

BlendArgs blend_args(const sdfddgi_ctx *c, const float4 *payload) {
    BlendArgs b{};
    b.P = (int)c->P;
    b.R = c->R;
    b.irr_res = c->prm.irr_res;
    b.depth_res = c->prm.depth_res;
    b.hysteresis = c->prm.hysteresis;
    b.payload = payload;
    b.wt_i = c->wt_i;
    b.wt_d = c->wt_d;
    b.norm_i = c->norm_i;
    b.norm_d = c->norm_d;
    b.Rpad = c->Rpad;
    b.w16_i = c->w16_i;
    b.w16_d = c->w16_d;
    b.prev_irr = c->irr[c->cur];
    b.prev_depth = c->depth[c->cur];
    b.new_irr = c->irr[1 - c->cur];
    b.new_depth = c->depth[1 - c->cur];
    b.reject = c->reject;
    return b;
}

sdfddgi_status check_ctx(sdfddgi_ctx *c) {
    if (!c) return SDFDDGI_EINVAL;
    c->err.clear();
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    return SDFDDGI_OK;
}

}  // namespace

extern "C" {

void sdfddgi_default_params(sdfddgi_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->rays_per_probe = 144;
    p->max_steps = 64;
    p->irr_res = 8;
    p->depth_res = 16;
    p->hit_eps = 1e-3f;
    p->t_max = (float)(2.0 * std::sqrt(3.0));
    p->hysteresis = 0.97f;
    p->bounce_gain = 1.0f;
    p->depth_sharpness = 50.0f;
    p->shadow_bias = 4e-3f;
    p->relax = 1.0f;
    for (int c = 0; c < 3; ++c) p->albedo[c] = 0.5f;
}

sdfddgi_status sdfddgi_create(const sdfddgi_sdf_grid *sdf, const sdfddgi_probe_grid *probes,
                              const sdfddgi_params *params, void *hip_stream, sdfddgi_ctx **out) {
    g_create_error.clear();
    if (!out) return fail(nullptr, SDFDDGI_EINVAL, "out is NULL");
    *out = nullptr;
    sdfddgi_status st = validate(sdf, probes, params);
    if (st != SDFDDGI_OK) return st;

    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) return fail(nullptr, SDFDDGI_EDEVICE, "no HIP device visible");
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess)
        return hip_fail(nullptr, e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, SDFDDGI_EDEVICE, "library built for gfx950, device is %s",
                    prop.gcnArchName);

    sdfddgi_ctx *c = new (std::nothrow) sdfddgi_ctx();
    if (!c) return fail(nullptr, SDFDDGI_ENOMEM, "host allocation failed");
    c->device = dev;
    c->stream = (hipStream_t)hip_stream;
    c->prm = *params;
    c->half = (params->flags & SDFDDGI_FLAG_FP16) != 0;
    c->nl = sdf->num_levels;
    c->pg = *probes;
    c->P = (int64_t)probes->n[0] * probes->n[1] * probes->n[2];
    c->R = params->rays_per_probe;
    c->Ti = params->irr_res * params->irr_res;
    c->Td = params->depth_res * params->depth_res;
    c->Tpi = (c->Ti + 15) / 16 * 16;
    c->Tpd = (c->Td + 15) / 16 * 16;
    c->irr_floats = c->P * (params->irr_res + 2) * (params->irr_res + 2) * 3;
    c->depth_floats = c->P * (params->depth_res + 2) * (params->depth_res + 2) * 2;

    auto bail = [&](sdfddgi_status s) {
        (void)hipStreamSynchronize(c->stream);
        free_all(c);
        delete c;
        return s;
    };
#define SDF_TRY(expr, what)                                                     \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess) return bail(hip_fail(nullptr, e_, what));         \
    } while (0)

    for (int L = 0; L < c->nl; ++L) {
        const sdfddgi_sdf_level &lv = sdf->level[L];
        const size_t cnt = (size_t)lv.n[0] * lv.n[1] * lv.n[2];
        for (int k = 0; k < 3; ++k) {
            c->n[L][k] = lv.n[k];
            c->origin[L][k] = lv.origin[k];
        }
        c->spacing[L] = lv.spacing;
        const size_t nquad = (size_t)lv.n[0] * (lv.n[1] - 1) * (lv.n[2] - 1);
        SDF_TRY(hipMalloc(&c->quad[L], nquad * (c->half ? 8 : 16)), "allocating sdf level");
        SDF_TRY(launch_pack_quads(lv.sdf, lv.n[0], lv.n[1], lv.n[2], c->half, c->quad[L],
                                  c->stream),
                "packing sdf level");
        if (lv.albedo_rgb) {
            SDF_TRY(dev_alloc(&c->alb[L], 3 * cnt), "allocating albedo level");
            SDF_TRY(hipMemcpyAsync(c->alb[L], lv.albedo_rgb, 3 * cnt * sizeof(float),
                                   hipMemcpyDeviceToDevice, c->stream), "copying albedo level");
        }
    }

    // Host constants in binary64: probe positions (rounded once), the fixed
    // spherical-Fibonacci set and the texel directions of both maps.
    const int64_t P = c->P;
    float *h_pos = new (std::nothrow) float[3 * P];
    double *h_base = new (std::nothrow) double[3 * c->R];
    double *h_ti = new (std::nothrow) double[3 * c->Ti];
    double *h_td = new (std::nothrow) double[3 * c->Td];
    if (!h_pos || !h_base || !h_ti || !h_td) {
        delete[] h_pos; delete[] h_base; delete[] h_ti; delete[] h_td;
        return bail(fail(nullptr, SDFDDGI_ENOMEM, "host allocation failed"));
    }
    const int nx = probes->n[0], ny = probes->n[1];
    for (int64_t p = 0; p < P; ++p) {
        const int64_t idx[3] = {p % nx, (p / nx) % ny, p / ((int64_t)nx * ny)};
        for (int k = 0; k < 3; ++k)
            h_pos[3 * p + k] = (float)(probes->origin[k] + probes->spacing[k] * (double)idx[k]);
    }
    for (int i = 0; i < c->R; ++i) fibonacci_point(i, c->R, h_base + 3 * i);
    // tracing order of the probes: Morton order of their (x, y, z) grid index
    std::vector<std::pair<uint64_t, int32_t>> morton((size_t)P);
    for (int64_t p = 0; p < P; ++p) {
        const uint64_t x = (uint64_t)(p % nx), y = (uint64_t)((p / nx) % ny);
        const uint64_t z = (uint64_t)(p / ((int64_t)nx * ny));
        uint64_t m = 0;
        for (int b = 0; b < 21; ++b)
            m |= (((x >> b) & 1) << (3 * b)) | (((y >> b) & 1) << (3 * b + 1)) |
                 (((z >> b) & 1) << (3 * b + 2));
        morton[(size_t)p] = {m, (int32_t)p};
    }
    std::sort(morton.begin(), morton.end());
    std::vector<int32_t> h_order((size_t)P);
    for (int64_t j = 0; j < P; ++j) h_order[(size_t)j] = morton[(size_t)j].second;
    for (int t = 0; t < c->Ti; ++t)
        texel_direction(params->irr_res, t % params->irr_res, t / params->irr_res, h_ti + 3 * t);
    for (int t = 0; t < c->Td; ++t)
        texel_direction(params->depth_res, t % params->depth_res, t / params->depth_res,
                        h_td + 3 * t);

    hipError_t ce = hipSuccess;
    auto chk = [&](hipError_t x) { if (ce == hipSuccess) ce = x; };
    chk(dev_alloc(&c->probe_pos, 3 * P));
    chk(dev_alloc(&c->probe_order, P));
    chk(dev_alloc(&c->base_dirs, 3 * c->R));
    chk(dev_alloc(&c->texel_i, 3 * c->Ti));
    chk(dev_alloc(&c->texel_d, 3 * c->Td));
    if (ce == hipSuccess) {
        chk(hipMemcpy(c->probe_pos, h_pos, 3 * P * sizeof(float), hipMemcpyHostToDevice));
        chk(hipMemcpy(c->probe_order, h_order.data(), P * sizeof(int32_t), hipMemcpyHostToDevice));
        chk(hipMemcpy(c->base_dirs, h_base, 3 * c->R * sizeof(double), hipMemcpyHostToDevice));
        chk(hipMemcpy(c->texel_i, h_ti, 3 * c->Ti * sizeof(double), hipMemcpyHostToDevice));
        chk(hipMemcpy(c->texel_d, h_td, 3 * c->Td * sizeof(double), hipMemcpyHostToDevice));
    }
    delete[] h_pos; delete[] h_base; delete[] h_ti; delete[] h_td;
    SDF_TRY(ce, "uploading constants");

    SDF_TRY(dev_alloc(&c->dirs, 3 * c->R), "allocating tables");
    SDF_TRY(dev_alloc(&c->wt_i, (size_t)c->R * c->Tpi), "allocating tables");
    SDF_TRY(dev_alloc(&c->wt_d, (size_t)c->R * c->Tpd), "allocating tables");
    SDF_TRY(hipMemsetAsync(c->wt_i, 0, (size_t)c->R * c->Tpi * sizeof(float), c->stream),
            "clearing tables");
    SDF_TRY(hipMemsetAsync(c->wt_d, 0, (size_t)c->R * c->Tpd * sizeof(float), c->stream),
            "clearing tables");
    if (c->half) {
        c->Rpad = (c->R + 63) / 64 * 64;
        SDF_TRY(dev_alloc(&c->w16_i, (size_t)c->Tpi * c->Rpad), "allocating tables");
        SDF_TRY(dev_alloc(&c->w16_d, (size_t)c->Tpd * c->Rpad), "allocating tables");
        SDF_TRY(hipMemsetAsync(c->w16_i, 0, (size_t)c->Tpi * c->Rpad * 2, c->stream),
                "clearing tables");
        SDF_TRY(hipMemsetAsync(c->w16_d, 0, (size_t)c->Tpd * c->Rpad * 2, c->stream),
                "clearing tables");
    }
    SDF_TRY(dev_alloc(&c->norm_i, c->Ti), "allocating tables");
    SDF_TRY(dev_alloc(&c->norm_d, c->Td), "allocating tables");
    for (int k = 0; k < 2; ++k) {
        SDF_TRY(dev_alloc(&c->irr[k], c->irr_floats), "allocating irradiance atlas");
        SDF_TRY(dev_alloc(&c->depth[k], c->depth_floats), "allocating depth atlas");
        SDF_TRY(hipMemsetAsync(c->irr[k], 0, c->irr_floats * sizeof(float), c->stream),
                "clearing atlas");
        SDF_TRY(hipMemsetAsync(c->depth[k], 0, c->depth_floats * sizeof(float), c->stream),
                "clearing atlas");
    }
    SDF_TRY(dev_alloc(&c->reject, P), "allocating reject flags");
    SDF_TRY(launch_fill_u8(c->reject, 1, P, c->stream), "launching fill");
    SDF_TRY(dev_alloc(&c->counter, 3), "allocating ray counters");
    SDF_TRY(dev_alloc(&c->hitq, (size_t)P * c->R), "allocating the hit queue");
    SDF_TRY(dev_alloc(&c->payload, (size_t)P * c->R), "allocating payload");
    c->grid = trace_grid(dev, P * c->R, c->half);
    if (params->flags & SDFDDGI_FLAG_RECORD_RAYS)
        SDF_TRY(dev_alloc(&c->records, (size_t)P * c->R * 8), "allocating ray records");
    if (params->flags & SDFDDGI_FLAG_TIMING) {
        c->ev_ring = new (std::nothrow) hipEvent_t[kEvents * kTimingRing]();
        if (!c->ev_ring) return bail(fail(nullptr, SDFDDGI_ENOMEM, "host allocation failed"));
        for (int k = 0; k < kEvents * kTimingRing; ++k)
            SDF_TRY(hipEventCreate(&c->ev_ring[k]), "creating events");
    }
    SDF_TRY(hipStreamSynchronize(c->stream), "waiting for create");
#undef SDF_TRY
    *out = c;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_update_frame(sdfddgi_ctx *c, const sdfddgi_light *light,
                                    uint64_t rotation_seed) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!light) return fail(c, SDFDDGI_EINVAL, "light is NULL");
    if (!finite_all(light->dir_to_light, 3) || !finite_all(light->radiance_rgb, 3))
        return fail(c, SDFDDGI_EINVAL, "non-finite light");
    const double d0 = light->dir_to_light[0], d1 = light->dir_to_light[1],
                 d2 = light->dir_to_light[2];
    const double len = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    if (!(len > 0.0)) return fail(c, SDFDDGI_EINVAL, "light direction has zero length");
    for (int k = 0; k < 3; ++k)
        if (light->radiance_rgb[k] < 0) return fail(c, SDFDDGI_EINVAL, "negative radiance");

    TraceArgs t{};
    for (int L = 0; L < c->nl; ++L) t.lv[L] = dev_level(c, L);
    t.nl = c->nl;
    t.half_sdf = c->half ? 1 : 0;
    t.P = (int)c->P;
    t.R = c->R;
    t.max_steps = c->prm.max_steps;
    t.irr_res = c->prm.irr_res;
    t.pg = dev_probes(c);
    t.eps = c->prm.hit_eps;
    t.t_max = c->prm.t_max;
    t.relax = c->prm.relax;
    t.bias = c->prm.shadow_bias;
    t.gain = c->prm.bounce_gain;
    t.l0 = (float)(d0 / len);
    t.l1 = (float)(d1 / len);
    t.l2 = (float)(d2 / len);
    t.rad0 = light->radiance_rgb[0];
    t.rad1 = light->radiance_rgb[1];
    t.rad2 = light->radiance_rgb[2];
    t.sky0 = c->prm.sky_rgb[0];
    t.sky1 = c->prm.sky_rgb[1];
    t.sky2 = c->prm.sky_rgb[2];
    t.alb0 = c->prm.albedo[0];
    t.alb1 = c->prm.albedo[1];
    t.alb2 = c->prm.albedo[2];
    t.probe_pos = c->probe_pos;
    t.probe_order = c->probe_order;
    t.dirs = c->dirs;
    t.prev_irr = c->irr[c->cur];
    t.payload = c->payload;
    t.records = c->records;
    t.counter = c->counter;
    t.hitq = c->hitq;

    hipEvent_t *ev = c->ev_ring ? c->ev_ring + kEvents * c->ring_head : nullptr;
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], c->stream)) != hipSuccess)
        return hip_fail(c, e, "event");
    if ((e = launch_tables(table_args(c, rotation_seed), c->stream)) != hipSuccess)
        return hip_fail(c, e, "launching tables_kernel");
    if (ev && (e = hipEventRecord(ev[1], c->stream)) != hipSuccess)
        return hip_fail(c, e, "event");
    if ((e = launch_primary(t, c->grid, c->stream)) != hipSuccess)
        return hip_fail(c, e, "launching primary_kernel");
    if (ev && (e = hipEventRecord(ev[2], c->stream)) != hipSuccess)
        return hip_fail(c, e, "event");
    if ((e = launch_hits(t, c->grid, c->stream)) != hipSuccess)
        return hip_fail(c, e, "launching hits_kernel");
    if (ev && (e = hipEventRecord(ev[3], c->stream)) != hipSuccess)
        return hip_fail(c, e, "event");
    if ((e = launch_blend(blend_args(c, c->payload), c->stream)) != hipSuccess)
        return hip_fail(c, e, "launching blend_kernel");
    if (ev && (e = hipEventRecord(ev[4], c->stream)) != hipSuccess)
        return hip_fail(c, e, "event");
    if (ev) {
        c->ring_head = (c->ring_head + 1) % kTimingRing;
        ++c->timed_frames;
    }
    c->cur = 1 - c->cur;
    c->have_frame = true;
    c->have_records = c->records != nullptr;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_blend(sdfddgi_ctx *c, const float *payload, uint64_t rotation_seed) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!payload) return fail(c, SDFDDGI_EINVAL, "payload is NULL");
    hipError_t e;
    if ((e = launch_tables(table_args(c, rotation_seed), c->stream)) != hipSuccess)
        return hip_fail(c, e, "launching tables_kernel");
    if ((e = launch_blend(blend_args(c, (const float4 *)payload), c->stream)) != hipSuccess)
        return hip_fail(c, e, "launching blend_kernel");
    c->cur = 1 - c->cur;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_sample_irradiance(sdfddgi_ctx *c, const float *points,
                                         const float *normals, int64_t n, float *out_rgb) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (n < 0) return fail(c, SDFDDGI_EINVAL, "negative count");
    if (n == 0) return SDFDDGI_OK;
    if (!points || !normals || !out_rgb) return fail(c, SDFDDGI_EINVAL, "null array");
    SampleArgs a{};
    a.n = n;
    a.irr_res = c->prm.irr_res;
    a.pg = dev_probes(c);
    a.atlas = c->irr[c->cur];
    a.points = points;
    a.normals = normals;
    a.out = out_rgb;
    hipError_t e = launch_sample(a, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "launching sample_kernel");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_get_maps(sdfddgi_ctx *c, float *irr, float *depth) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    hipError_t e;
    if (irr && (e = hipMemcpyAsync(irr, c->irr[c->cur], c->irr_floats * sizeof(float),
                                   hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
        return hip_fail(c, e, "copying irradiance atlas");
    if (depth && (e = hipMemcpyAsync(depth, c->depth[c->cur], c->depth_floats * sizeof(float),
                                     hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
        return hip_fail(c, e, "copying depth atlas");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_set_maps(sdfddgi_ctx *c, const float *irr, const float *depth) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!irr || !depth) return fail(c, SDFDDGI_EINVAL, "both maps are required");
    hipError_t e;
    if ((e = hipMemcpyAsync(c->irr[c->cur], irr, c->irr_floats * sizeof(float),
                            hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
        return hip_fail(c, e, "copying irradiance atlas");
    if ((e = hipMemcpyAsync(c->depth[c->cur], depth, c->depth_floats * sizeof(float),
                            hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
        return hip_fail(c, e, "copying depth atlas");
    if ((e = launch_fill_u8(c->reject, 0, c->P, c->stream)) != hipSuccess)
        return hip_fail(c, e, "launching fill");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_reset_history(sdfddgi_ctx *c) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    hipError_t e = launch_fill_u8(c->reject, 1, c->P, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "launching fill");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_get_payload(sdfddgi_ctx *c, float *out) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!out) return fail(c, SDFDDGI_EINVAL, "out is NULL");
    if (!c->have_frame) return fail(c, SDFDDGI_ESTATE, "no frame has been traced yet");
    hipError_t e = hipMemcpyAsync(out, c->payload, (size_t)c->P * c->R * sizeof(float4),
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copying payload");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_get_ray_records(sdfddgi_ctx *c, int32_t *out) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!out) return fail(c, SDFDDGI_EINVAL, "out is NULL");
    if (!c->records) return fail(c, SDFDDGI_ESTATE, "created without SDFDDGI_FLAG_RECORD_RAYS");
    if (!c->have_records) return fail(c, SDFDDGI_ESTATE, "no frame has been traced yet");
    hipError_t e = hipMemcpyAsync(out, c->records, (size_t)c->P * c->R * 8 * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copying records");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_get_ray_directions(sdfddgi_ctx *c, float *out) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!out) return fail(c, SDFDDGI_EINVAL, "out is NULL");
    hipError_t e = hipMemcpyAsync(out, c->dirs, (size_t)c->R * 3 * sizeof(float),
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copying directions");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_ray_directions(uint64_t rotation_seed, int32_t rays, float *out) {
    if (!out || rays < 1 || rays > kMaxRays) return SDFDDGI_EINVAL;
    double q[9];
    rotation_matrix(rotation_seed, q);
    for (int i = 0; i < rays; ++i) {
        double s[3];
        fibonacci_point(i, rays, s);
        for (int a = 0; a < 3; ++a)
            out[3 * i + a] = (float)(q[3 * a] * s[0] + q[3 * a + 1] * s[1] + q[3 * a + 2] * s[2]);
    }
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_get_kernel_times(sdfddgi_ctx *c, float *ms, int32_t count) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!ms || count < 0 || count > kEvents) return fail(c, SDFDDGI_EINVAL, "bad output array");
    if (!c->ev_ring) return fail(c, SDFDDGI_ESTATE, "created without SDFDDGI_FLAG_TIMING");
    if (c->timed_frames == 0) return fail(c, SDFDDGI_ESTATE, "no timed frame since the last call");
    const int frames = (int)(c->timed_frames < kTimingRing ? c->timed_frames : kTimingRing);
    const int last = (c->ring_head + kTimingRing - 1) % kTimingRing;
    hipError_t e = hipEventSynchronize(c->ev_ring[kEvents * last + kEvents - 1]);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
    const int pairs[kEvents][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 4}, {0, 4}};
    double sum[kEvents] = {0, 0, 0, 0, 0};
    for (int f = 0; f < frames; ++f) {
        const hipEvent_t *ev = c->ev_ring + kEvents * ((last - f + kTimingRing) % kTimingRing);
        for (int k = 0; k < kEvents; ++k) {
            float v = 0.0f;
            e = hipEventElapsedTime(&v, ev[pairs[k][0]], ev[pairs[k][1]]);
            if (e != hipSuccess) return hip_fail(c, e, "hipEventElapsedTime");
            sum[k] += v;
        }
    }
    for (int k = 0; k < count; ++k) ms[k] = (float)(sum[k] / frames);
    c->timed_frames = 0;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_get_sizes(const sdfddgi_ctx *c, int64_t *probes, int32_t *rays,
                                 int64_t *irr_floats, int64_t *depth_floats) {
    if (!c) return SDFDDGI_EINVAL;
    if (probes) *probes = c->P;
    if (rays) *rays = c->R;
    if (irr_floats) *irr_floats = c->irr_floats;
    if (depth_floats) *depth_floats = c->depth_floats;
    return SDFDDGI_OK;
}

const char *sdfddgi_last_error(const sdfddgi_ctx *c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

sdfddgi_status sdfddgi_destroy(sdfddgi_ctx *c) {
    if (!c) return SDFDDGI_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
    return SDFDDGI_OK;
}

}  // extern "C"
