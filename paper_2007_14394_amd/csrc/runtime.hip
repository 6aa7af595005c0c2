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
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

using namespace sdfddgi;

namespace {

thread_local std::string g_create_error;

constexpr double kPi = 3.14159265358979323846;
constexpr int kTimingRing = 256;
constexpr int kEvents = 14;

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

// One set of ray directions with its tables and per-ray buffers: the frame's
// rays (rays_per_probe) and the learned form's low ray count.
struct RaySet {
    int R = 0, Rpad = 0;
    double *base = nullptr;          // [R][3] unrotated spherical-Fibonacci set
    float *dirs = nullptr, *wt_i = nullptr, *wt_d = nullptr, *norm_i = nullptr, *norm_d = nullptr;
    _Float16 *w16_i = nullptr;       // precision-form weight tables [T][Rpad]
    __bf16 *w16_d = nullptr;
    float4 *payload = nullptr;       // [P][R]
    int4 *hitq = nullptr;            // [P][R]
    int *counter = nullptr;          // [kSetCounters] counters of the set's trace (see TraceArgs);
                                     //     [6] the length of `list`
    float4 *geo = nullptr;           // learned form: [P][R][2] split hit shading (TraceArgs::geo)
    int *list = nullptr;             // learned form's fallback sets: [P] the frame's fallback list
    TraceGrid grid;
    hipEvent_t done = nullptr;       // main / spare: recorded on the caller's stream once the
                                     //     last plain frame that traced into this set is blended;
                                     //     learned sets: once the last frame that used it is done
                                     //     with it (see the context)
    hipEvent_t ready = nullptr;      // learned sets: the set's pass is done (see the context)
    hipEvent_t sel = nullptr;        // fallback sets: the frame's list is built
};

// Counters of one learned frame: [0..2] the trace pass over all probes (unused,
// queue entries claimed, queue length), [3..5] the second pass (its fallback
// probes), [6] fallback count; from [kPartStride] the two passes' per-XCD chunk
// counters, kXcds * kPartStride ints each.
constexpr int kCounters = kPartStride + 2 * kXcds * kPartStride;
// A ray set's own counters (plain frames): [0..2] as above, per-XCD ones from
// [kPartStride].
constexpr int kSetCounters = kPartStride + kXcds * kPartStride;

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
    int Ti = 0, Td = 0, Tpi = 0, Tpd = 0;
    int64_t irr_floats = 0, depth_floats = 0;
    float *probe_pos = nullptr;
    float *grid_pos = nullptr;   // the grid positions (probe_pos differs after relocation)
    int2 *probe_first = nullptr; // each probe's first sample (see TraceArgs)
    int *probe_order = nullptr;
    double *texel_i = nullptr, *texel_d = nullptr;
    // main: the ray set of the last plain frame; spare: the one the next plain frame
    // traces into while the last one's hit shading and blend may still run
    RaySet main, spare;
    // The learned form's ray sets, used in turn by consecutive learned frames so that
    // a frame's traces need not wait for the frame before it: for learned frame n of
    // parity k = n % 2, low[k] holds learned_rays rays over every probe and fbs[k]
    // rays_per_probe rays over the frame's fallback list. fb_flag[k]: per probe,
    // the plain update in the frames of parity k; each frame's denoiser replaces it by
    // its decision for the learned frame after next.
    RaySet low[2], fbs[2];
    uint8_t *fb_flag[2]{};
    int last_learned = 0;        // parity of the last learned frame
    // Plain frames are pipelined: the tables and primary trace of frame f run on the
    // side stream, and on grids the atlas-independent half of its hit shading
    // (normal, shadow ray, albedo) on side2 after them, so both may overlap frame
    // f-1's lookups and blend on the caller's stream (neither reads the atlas or
    // anything frame f-1 writes); the caller's stream then takes frame f's lookup
    // half and blend. A frame's side work waits for the done event of the ray set it
    // traces into (recorded after the blend of the frame before the previous one);
    // ev_primary joins the side stream to side2 (or, unsplit, to the caller's
    // stream) and the set's ready event side2 to the caller's. Any other call in
    // between makes the next frame wait for everything before it (serialize_next).
    hipStream_t side = nullptr;
    hipEvent_t ev_primary = nullptr, ev_tail = nullptr;
    bool serialize_next = true;
    // Learned frames overlap among themselves; a switch between plain and learned
    // frames waits for everything before it. Learned frame n (parity k = n % 2, low
    // set lo = low[k]) has two side chains, dealt in turn to the three side streams
    // (side, side2, side3), so that the chains of consecutive frames overlap:
    //   low chain, after lo.done (learned frame n - 2 is done with that set): the low
    //     set's tables, primary trace and the atlas-independent half of its hit
    //     shading, then lo.ready;
    //   fallback chain, after fbs[k].done (learned frame n - 2 is done: its denoiser
    //     has written the flags of parity k, its fallback blend has read the set's
    //     list and payload): the fallback set's tables, the list (fbs[k].sel), its primary
    //     trace and atlas-independent half; after ev_end (the previous frame is done,
    //     its atlas complete) the lookup half and the blend with hysteresis into the
    //     fallback probes' tiles of the new atlas, then fbs[k].ready.
    // The caller's stream, after the previous frame: the low-ray lookup half and Eq. 3
    // without hysteresis (lo.done), the denoiser after fbs[k].sel, then it joins
    // fbs[k].ready (fbs[k].done) and records ev_end.
    bool learned_chain = false;
    hipStream_t side2 = nullptr, side3 = nullptr;
    hipEvent_t ev_end = nullptr;
    int64_t learned_index = 0;   // learned frames so far: deals the side chains
    float *irr[2]{}, *depth[2]{};
    int cur = 0;
    uint8_t *reject = nullptr;
    int *counter = nullptr;      // [kCounters]
    int *records = nullptr;
    bool have_frame = false, have_records = false, have_learned = false;
    // learned form
    float *u_irr = nullptr, *u_depth = nullptr;      // low-ray estimates (no hysteresis)
    float *probe_sdf = nullptr;                      // [P]
    float *texel_dir = nullptr;                      // [Ti][3] binary32
    float *mean_error = nullptr;                     // [P]
    // analytic scene (sdfddgi_create_analytic): the primitives in cluster order
    bool analytic = false;
    int an_nprims = 0, an_nclusters = 0;
    int *an_kind = nullptr, *an_orig = nullptr, *an_first = nullptr;
    float *an_center = nullptr, *an_half = nullptr, *an_lo = nullptr, *an_hi = nullptr;
    float *an_alb = nullptr;
    // Timing: kEvents events per frame in a ring (see sdfddgi_get_kernel_times);
    // sdfddgi_get_kernel_times averages the frames recorded since its previous call.
    hipEvent_t *ev_ring = nullptr;
    bool ring_learned[kTimingRing]{};   // the frame in that slot was learned (else only
                                        // marks 0-5 and 10 were recorded)
    int ring_head = 0;
    int64_t timed_frames = 0;
    std::string err;
};

struct sdfddgi_denoiser {
    int device = 0;
    hipStream_t stream = nullptr;
    float S = 1.0f, D = 1.0f;
    float *theta = nullptr;
    uint4 *fwd = nullptr, *bwd = nullptr;
    float *bias = nullptr;
};

struct sdfddgi_trainer {
    int device = 0;
    hipStream_t stream = nullptr;
    sdfddgi_train_config cfg{};
    int64_t step = 0;
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr;
    uint4 *fwd = nullptr, *bwd = nullptr;
    float *bias = nullptr;
};

namespace {

thread_local std::string g_learned_error;

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

sdfddgi_status lfail(sdfddgi_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_learned_error = buf;
    return s;
}

sdfddgi_status lhip_fail(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory) return lfail(SDFDDGI_ENOMEM, "%s: out of device memory", what);
    return lfail(SDFDDGI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

template <typename T>
hipError_t dev_alloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return hipSuccess;
    return hipMalloc((void **)p, count * sizeof(T));
}

template <typename T>
void dev_free(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

void free_set(RaySet &r) {
    dev_free(r.base); dev_free(r.dirs); dev_free(r.wt_i); dev_free(r.wt_d);
    dev_free(r.norm_i); dev_free(r.norm_d); dev_free(r.w16_i); dev_free(r.w16_d);
    dev_free(r.payload); dev_free(r.hitq); dev_free(r.counter); dev_free(r.geo); dev_free(r.list);
    r.R = r.Rpad = 0;
}

void free_all(sdfddgi_ctx *c) {
    for (int L = 0; L < kMaxLevels; ++L) {
        dev_free(c->quad[L]);
        dev_free(c->alb[L]);
    }
    free_set(c->main);
    free_set(c->spare);
    for (RaySet *r : {&c->low[0], &c->low[1], &c->fbs[0], &c->fbs[1]}) {
        free_set(*r);
        if (r->done) (void)hipEventDestroy(r->done);
        if (r->ready) (void)hipEventDestroy(r->ready);
        if (r->sel) (void)hipEventDestroy(r->sel);
    }
    for (RaySet *r : {&c->main, &c->spare}) {
        if (r->done) (void)hipEventDestroy(r->done);
        if (r->ready) (void)hipEventDestroy(r->ready);
    }
    if (c->ev_primary) (void)hipEventDestroy(c->ev_primary);
    if (c->ev_tail) (void)hipEventDestroy(c->ev_tail);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->side2) (void)hipStreamDestroy(c->side2);
    if (c->side3) (void)hipStreamDestroy(c->side3);
    if (c->ev_end) (void)hipEventDestroy(c->ev_end);
    dev_free(c->probe_pos); dev_free(c->grid_pos); dev_free(c->probe_first); dev_free(c->probe_order); dev_free(c->texel_i); dev_free(c->texel_d);
    dev_free(c->irr[0]); dev_free(c->irr[1]); dev_free(c->depth[0]); dev_free(c->depth[1]);
    dev_free(c->reject); dev_free(c->counter); dev_free(c->records);
    dev_free(c->u_irr); dev_free(c->u_depth);
    dev_free(c->probe_sdf); dev_free(c->texel_dir); dev_free(c->mean_error);
    dev_free(c->fb_flag[0]); dev_free(c->fb_flag[1]);
    dev_free(c->an_kind); dev_free(c->an_orig); dev_free(c->an_first); dev_free(c->an_center);
    dev_free(c->an_half); dev_free(c->an_lo); dev_free(c->an_hi); dev_free(c->an_alb);
    if (c->ev_ring) {
        for (int k = 0; k < kEvents * kTimingRing; ++k)
            if (c->ev_ring[k]) (void)hipEventDestroy(c->ev_ring[k]);
        delete[] c->ev_ring;
    }
}

bool valid_rays(int R) { return R >= 16 && R <= kMaxRays && R % 16 == 0; }

sdfddgi_status validate_probes_params(const sdfddgi_probe_grid *pg, const sdfddgi_params *p);

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
    return validate_probes_params(pg, p);
}

sdfddgi_status validate_probes_params(const sdfddgi_probe_grid *pg, const sdfddgi_params *p) {
    if (!pg || !p) return fail(nullptr, SDFDDGI_EINVAL, "null argument");
    int64_t P = 1;
    for (int c = 0; c < 3; ++c) {
        if (pg->n[c] < 2) return fail(nullptr, SDFDDGI_EINVAL, "probe grid n[%d] < 2", c);
        if (!(pg->spacing[c] > 0.0) || !std::isfinite(pg->spacing[c]) ||
            !std::isfinite(pg->origin[c]))
            return fail(nullptr, SDFDDGI_EINVAL, "probe grid spacing/origin invalid");
        P *= pg->n[c];
    }
    const int R = p->rays_per_probe;
    if (!valid_rays(R))
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
    if (!(p->fallback_error >= 0))  // +inf allowed: no probe falls back on its prediction
        return fail(nullptr, SDFDDGI_EINVAL, "fallback_error must be >= 0");
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
    if (p->learned_rays != 0) {
        if (!valid_rays(p->learned_rays) || p->learned_rays > R)
            return fail(nullptr, SDFDDGI_EINVAL,
                        "learned_rays %d: need 0 or a multiple of 16 in 16..rays_per_probe",
                        p->learned_rays);
        if (p->irr_res > kMaxLearnedRes || p->depth_res % p->irr_res != 0 || p->depth_res % 2)
            return fail(nullptr, SDFDDGI_EINVAL,
                        "learned form needs irr_res <= %d and depth_res an even multiple of "
                        "irr_res", kMaxLearnedRes);
    }
    return SDFDDGI_OK;
}

// An analytic scene's primitives packed into clusters for the culled query of
// Sec. 3.3: primitives in Morton order of their centres, cluster_size at a time;
// each cluster's bounding box is widened by 1e-4 (1 + the scene's reach) and
// rounded outward, so its binary32 distance stays below every member's.
struct HostClusters {
    int nprims = 0, nclusters = 0;
    std::vector<int> kind, orig, first;
    std::vector<float> cen, half, lo, hi, alb;
};

// Empty on success, else why the primitives are refused. albedo may be null.
std::string build_clusters(int nprims, const int32_t *kind, const double *center,
                           const double *half, const double *albedo, int cluster_size,
                           HostClusters &h) {
    char msg[160];
    if (nprims < 1 || nprims > kMaxAnalyticPrims || !kind || !center || !half) {
        std::snprintf(msg, sizeof msg, "need 1..%d primitives", kMaxAnalyticPrims);
        return msg;
    }
    if (cluster_size < 1 || cluster_size > 64) return "cluster_size must be in 1..64";
    const int nclusters = (nprims + cluster_size - 1) / cluster_size;
    if (nclusters > kMaxClusters) {
        std::snprintf(msg, sizeof msg, "more than %d clusters", kMaxClusters);
        return msg;
    }
    double lo_s[3] = {INFINITY, INFINITY, INFINITY}, hi_s[3] = {-INFINITY, -INFINITY, -INFINITY};
    double reach = 0.0;
    for (int m = 0; m < nprims; ++m) {
        if (kind[m] != 0 && kind[m] != 1) {
            std::snprintf(msg, sizeof msg, "primitive kind %d", kind[m]);
            return msg;
        }
        for (int c = 0; c < 3; ++c) {
            const double hc = kind[m] == 0 ? half[3 * m] : half[3 * m + c];
            if (!std::isfinite(center[3 * m + c]) || !std::isfinite(hc) || hc < 0) {
                std::snprintf(msg, sizeof msg, "primitive %d: bad centre or size", m);
                return msg;
            }
            if (albedo && !(albedo[3 * m + c] >= 0 && std::isfinite(albedo[3 * m + c]))) {
                std::snprintf(msg, sizeof msg, "primitive %d: bad albedo", m);
                return msg;
            }
            lo_s[c] = std::min(lo_s[c], center[3 * m + c]);
            hi_s[c] = std::max(hi_s[c], center[3 * m + c]);
            reach = std::max(reach, std::fabs(center[3 * m + c]) + hc);
        }
    }
    std::vector<std::pair<uint64_t, int>> order((size_t)nprims);
    for (int m = 0; m < nprims; ++m) {
        uint64_t code = 0;
        for (int c = 0; c < 3; ++c) {
            const double ext = hi_s[c] - lo_s[c];
            const double u = ext > 0 ? (center[3 * m + c] - lo_s[c]) / ext : 0.0;
            const uint64_t q = (uint64_t)std::min(1023.0, std::max(0.0, std::floor(u * 1024.0)));
            for (int bit = 0; bit < 10; ++bit) code |= ((q >> bit) & 1ull) << (3 * bit + c);
        }
        order[(size_t)m] = {code, m};
    }
    std::sort(order.begin(), order.end());
    h.nprims = nprims;
    h.nclusters = nclusters;
    h.kind.assign(nprims, 0);
    h.orig.assign(nprims, 0);
    h.first.assign(nclusters + 1, 0);
    h.cen.assign(3 * (size_t)nprims, 0.0f);
    h.half.assign(3 * (size_t)nprims, 0.0f);
    h.alb.assign(3 * (size_t)nprims, 0.0f);
    h.lo.assign(3 * (size_t)nclusters, 0.0f);
    h.hi.assign(3 * (size_t)nclusters, 0.0f);
    const double widen = 1e-4 * (1.0 + reach);
    for (int k = 0; k < nclusters; ++k) {
        h.first[k] = k * cluster_size;
        double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int j = k * cluster_size; j < std::min(nprims, (k + 1) * cluster_size); ++j) {
            const int m = order[(size_t)j].second;
            h.kind[j] = kind[m];
            h.orig[j] = m;
            for (int c = 0; c < 3; ++c) {
                const double hc = kind[m] == 0 ? half[3 * m] : half[3 * m + c];
                h.cen[3 * j + c] = (float)center[3 * m + c];
                h.half[3 * j + c] = (float)half[3 * m + c];
                if (albedo) h.alb[3 * j + c] = (float)albedo[3 * m + c];
                blo[c] = std::min(blo[c], center[3 * m + c] - hc);
                bhi[c] = std::max(bhi[c], center[3 * m + c] + hc);
            }
        }
        for (int c = 0; c < 3; ++c) {   // widened, then rounded outward
            h.lo[3 * k + c] = std::nextafter((float)(blo[c] - widen), -INFINITY);
            h.hi[3 * k + c] = std::nextafter((float)(bhi[c] + widen), INFINITY);
        }
    }
    h.first[nclusters] = nprims;
    return std::string();
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


// Allocate a ray set of R rays: the fixed spherical-Fibonacci set (binary64,
// uploaded), zeroed weight tables and the per-ray buffers.
hipError_t alloc_set(sdfddgi_ctx *c, RaySet &r, int R, bool split = false) {
    free_set(r);
    r.R = R;
    std::vector<double> h_base(3 * (size_t)R);
    for (int i = 0; i < R; ++i) fibonacci_point(i, R, h_base.data() + 3 * i);
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(dev_alloc(&r.base, 3 * (size_t)R));
    chk(dev_alloc(&r.dirs, 3 * (size_t)R));
    chk(dev_alloc(&r.wt_i, (size_t)R * c->Tpi));
    chk(dev_alloc(&r.wt_d, (size_t)R * c->Tpd));
    chk(dev_alloc(&r.norm_i, c->Ti));
    chk(dev_alloc(&r.norm_d, c->Td));
    chk(dev_alloc(&r.payload, (size_t)c->P * R));
    chk(dev_alloc(&r.hitq, (size_t)c->P * R));
    chk(dev_alloc(&r.counter, kSetCounters));
    if (split) {
        chk(dev_alloc(&r.geo, 2 * (size_t)c->P * R));
        chk(dev_alloc(&r.list, (size_t)c->P));
    }
    if (e != hipSuccess) return e;
    chk(hipMemcpy(r.base, h_base.data(), 3 * (size_t)R * sizeof(double), hipMemcpyHostToDevice));
    chk(hipMemsetAsync(r.wt_i, 0, (size_t)R * c->Tpi * sizeof(float), c->stream));
    chk(hipMemsetAsync(r.wt_d, 0, (size_t)R * c->Tpd * sizeof(float), c->stream));
    if (c->half) {
        r.Rpad = (R + 63) / 64 * 64;
        chk(dev_alloc(&r.w16_i, (size_t)c->Tpi * r.Rpad));
        chk(dev_alloc(&r.w16_d, (size_t)c->Tpd * r.Rpad));
        if (e != hipSuccess) return e;
        chk(hipMemsetAsync(r.w16_i, 0, (size_t)c->Tpi * r.Rpad * 2, c->stream));
        chk(hipMemsetAsync(r.w16_d, 0, (size_t)c->Tpd * r.Rpad * 2, c->stream));
    }
    r.grid = trace_grid(c->device, c->P * R, c->half, c->analytic);
    return e;
}

TableArgs table_args(const sdfddgi_ctx *c, const RaySet &r, uint64_t seed, int ncounter,
                     int *counter = nullptr) {
    TableArgs t{};
    t.R = r.R;
    t.Ti = c->Ti;
    t.Td = c->Td;
    t.Tpi = c->Tpi;
    t.Tpd = c->Tpd;
    rotation_matrix(seed, t.q);
    t.sharp = (double)c->prm.depth_sharpness;
    t.base = r.base;
    t.texel_i = c->texel_i;
    t.texel_d = c->texel_d;
    t.dirs = r.dirs;
    t.wt_i = r.wt_i;
    t.wt_d = r.wt_d;
    t.norm_i = r.norm_i;
    t.norm_d = r.norm_d;
    t.counter = ncounter > 0 ? (counter ? counter : c->counter) : nullptr;
    t.ncounter = ncounter;
    t.Rpad = r.Rpad;
    t.w16_i = r.w16_i;
    t.w16_d = r.w16_d;
    return t;
}

// Blend of ray set r's payload: reads prev maps, writes new ones (hysteresis h,
// none where reject is set; reject may be null), optionally for a probe list.
BlendArgs blend_args(const sdfddgi_ctx *c, const RaySet &r, const float4 *payload, float h,
                     const float *prev_irr, const float *prev_depth, float *new_irr,
                     float *new_depth, uint8_t *reject, const int *list, const int *count) {
    BlendArgs b{};
    b.P = (int)c->P;
    b.R = r.R;
    b.irr_res = c->prm.irr_res;
    b.depth_res = c->prm.depth_res;
    b.hysteresis = h;
    b.payload = payload;
    b.wt_i = r.wt_i;
    b.wt_d = r.wt_d;
    b.norm_i = r.norm_i;
    b.norm_d = r.norm_d;
    b.Rpad = r.Rpad;
    b.w16_i = r.w16_i;
    b.w16_d = r.w16_d;
    b.prev_irr = prev_irr;
    b.prev_depth = prev_depth;
    b.new_irr = new_irr;
    b.new_depth = new_depth;
    b.reject = reject;
    b.probe_list = list;
    b.probe_count = count;
    return b;
}

// Trace arguments shared by every pass of a frame (levels, probes, light, params).
TraceArgs trace_base(const sdfddgi_ctx *c, const float l[3], const float rad[3]) {
    TraceArgs t{};
    for (int L = 0; L < c->nl; ++L) t.lv[L] = dev_level(c, L);
    t.nl = c->nl;
    t.half_sdf = c->half ? 1 : 0;
    t.P = (int)c->P;
    t.max_steps = c->prm.max_steps;
    t.irr_res = c->prm.irr_res;
    t.pg = dev_probes(c);
    t.eps = c->prm.hit_eps;
    t.t_max = c->prm.t_max;
    t.relax = c->prm.relax;
    t.bias = c->prm.shadow_bias;
    t.gain = c->prm.bounce_gain;
    t.l0 = l[0]; t.l1 = l[1]; t.l2 = l[2];
    t.rad0 = rad[0]; t.rad1 = rad[1]; t.rad2 = rad[2];
    t.sky0 = c->prm.sky_rgb[0];
    t.sky1 = c->prm.sky_rgb[1];
    t.sky2 = c->prm.sky_rgb[2];
    t.alb0 = c->prm.albedo[0];
    t.alb1 = c->prm.albedo[1];
    t.alb2 = c->prm.albedo[2];
    t.probe_pos = c->probe_pos;
    t.probe_order = c->probe_order;
    t.probe_first = c->probe_first;
    t.prev_irr = c->irr[c->cur];
    if (c->analytic) {
        t.analytic = 1;
        t.an.nprims = c->an_nprims;
        t.an.nclusters = c->an_nclusters;
        t.an.kind = c->an_kind;
        t.an.orig = c->an_orig;
        t.an.center = c->an_center;
        t.an.half = c->an_half;
        t.an.lo = c->an_lo;
        t.an.hi = c->an_hi;
        t.an.first = c->an_first;
        t.prim_alb = c->an_alb;
    }
    return t;
}

// The pass of ray set r: all probes (list == null) or the device-side list.
TraceArgs trace_pass(const TraceArgs &base, const RaySet &r, int *counters, int *parts,
                     const int *list, const int *count, int *records) {
    TraceArgs t = base;
    t.parts = parts;
    t.R = r.R;
    t.dirs = r.dirs;
    t.payload = r.payload;
    t.hitq = r.hitq;
    t.counter = counters;
    t.records = records;
    if (list) {
        t.probe_order = list;
        t.probe_count = count;
    }
    return t;
}

sdfddgi_status check_ctx(sdfddgi_ctx *c) {
    if (!c) return SDFDDGI_EINVAL;
    c->err.clear();
    // launch status is read with hipGetLastError: drop a failure some other code left
    (void)hipGetLastError();
    // the next plain frame waits for whatever this call enqueues
    c->serialize_next = true;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    return SDFDDGI_OK;
}

// Light direction normalised in binary64 and rounded once; EINVAL on bad input.
sdfddgi_status light_of(sdfddgi_ctx *c, const sdfddgi_light *light, float l[3], float rad[3]) {
    if (!light) return fail(c, SDFDDGI_EINVAL, "light is NULL");
    if (!finite_all(light->dir_to_light, 3) || !finite_all(light->radiance_rgb, 3))
        return fail(c, SDFDDGI_EINVAL, "non-finite light");
    const double d0 = light->dir_to_light[0], d1 = light->dir_to_light[1],
                 d2 = light->dir_to_light[2];
    const double len = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    if (!(len > 0.0)) return fail(c, SDFDDGI_EINVAL, "light direction has zero length");
    for (int k = 0; k < 3; ++k)
        if (light->radiance_rgb[k] < 0) return fail(c, SDFDDGI_EINVAL, "negative radiance");
    l[0] = (float)(d0 / len);
    l[1] = (float)(d1 / len);
    l[2] = (float)(d2 / len);
    for (int k = 0; k < 3; ++k) rad[k] = light->radiance_rgb[k];
    return SDFDDGI_OK;
}

// Timing events of one frame, each recorded when its step is done: [0] start,
// [1] tables, [2] primary trace, [3] hit shading may start, [4] hit shading,
// [5] blend, [6] denoiser, [7] fallback pass starts, [8] fallback trace (tables,
// list, primary, atlas-independent hit shading), [9] fallback blend, [10] frame,
// [11] fallback lookup half may start, [12] tables start, [13] tables done. Split
// hit shading (learned frames, and pipelined plain frames on grids) runs from [3]
// on a side stream to [4] on the caller's; such plain frames run the tables' weight
// rows on that side stream too ([12] to [13]), beside their primary trace.
struct FrameEvents {
    hipEvent_t *ev = nullptr;
    hipStream_t s = nullptr;
    hipError_t mark(int k) { return mark_on(k, s); }
    hipError_t mark_on(int k, hipStream_t on) {
        return ev ? hipEventRecord(ev[k], on) : hipSuccess;
    }
};

FrameEvents frame_events(sdfddgi_ctx *c) {
    FrameEvents f;
    f.ev = c->ev_ring ? c->ev_ring + kEvents * c->ring_head : nullptr;
    f.s = c->stream;
    return f;
}

void frame_done(sdfddgi_ctx *c, bool learned) {
    if (c->ev_ring) {
        c->ring_learned[c->ring_head] = learned;
        c->ring_head = (c->ring_head + 1) % kTimingRing;
        ++c->timed_frames;
    }
}

#define TRY_HIP(c, expr, what)                                                  \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess) return hip_fail((c), e_, (what));                 \
    } while (0)

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
    p->learned_rays = 0;
    p->fallback_error = 0.02f;
}

}  // extern "C"

// The body of both create entry points, after their checks: the scene is either the
// grid levels (sdf) or the clustered primitives (hc).
static sdfddgi_status create_ctx(const sdfddgi_sdf_grid *sdf, const HostClusters *hc,
                                 const sdfddgi_probe_grid *probes, const sdfddgi_params *params,
                                 void *hip_stream, sdfddgi_ctx **out) {
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
    c->nl = sdf ? sdf->num_levels : 0;
    c->analytic = hc != nullptr;
    c->pg = *probes;
    c->P = (int64_t)probes->n[0] * probes->n[1] * probes->n[2];
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
    if (hc) {
        c->an_nprims = hc->nprims;
        c->an_nclusters = hc->nclusters;
        const size_t n3 = 3 * (size_t)hc->nprims, k3 = 3 * (size_t)hc->nclusters;
        SDF_TRY(dev_alloc(&c->an_kind, hc->nprims), "allocating primitives");
        SDF_TRY(dev_alloc(&c->an_orig, hc->nprims), "allocating primitives");
        SDF_TRY(dev_alloc(&c->an_first, hc->nclusters + 1), "allocating primitives");
        SDF_TRY(dev_alloc(&c->an_center, n3), "allocating primitives");
        SDF_TRY(dev_alloc(&c->an_half, n3), "allocating primitives");
        SDF_TRY(dev_alloc(&c->an_alb, n3), "allocating primitives");
        SDF_TRY(dev_alloc(&c->an_lo, k3), "allocating primitives");
        SDF_TRY(dev_alloc(&c->an_hi, k3), "allocating primitives");
        SDF_TRY(hipMemcpy(c->an_kind, hc->kind.data(), hc->nprims * sizeof(int),
                          hipMemcpyHostToDevice), "uploading primitives");
        SDF_TRY(hipMemcpy(c->an_orig, hc->orig.data(), hc->nprims * sizeof(int),
                          hipMemcpyHostToDevice), "uploading primitives");
        SDF_TRY(hipMemcpy(c->an_first, hc->first.data(), (hc->nclusters + 1) * sizeof(int),
                          hipMemcpyHostToDevice), "uploading primitives");
        SDF_TRY(hipMemcpy(c->an_center, hc->cen.data(), n3 * sizeof(float), hipMemcpyHostToDevice),
                "uploading primitives");
        SDF_TRY(hipMemcpy(c->an_half, hc->half.data(), n3 * sizeof(float), hipMemcpyHostToDevice),
                "uploading primitives");
        SDF_TRY(hipMemcpy(c->an_alb, hc->alb.data(), n3 * sizeof(float), hipMemcpyHostToDevice),
                "uploading primitives");
        SDF_TRY(hipMemcpy(c->an_lo, hc->lo.data(), k3 * sizeof(float), hipMemcpyHostToDevice),
                "uploading primitives");
        SDF_TRY(hipMemcpy(c->an_hi, hc->hi.data(), k3 * sizeof(float), hipMemcpyHostToDevice),
                "uploading primitives");
    }

    // Host constants in binary64: probe positions (rounded once), the probes'
    // tracing order and the texel directions of both maps.
    const int64_t P = c->P;
    std::vector<float> h_pos(3 * (size_t)P);
    std::vector<double> h_ti(3 * (size_t)c->Ti), h_td(3 * (size_t)c->Td);
    std::vector<float> h_tif(3 * (size_t)c->Ti);
    const int nx = probes->n[0], ny = probes->n[1];
    for (int64_t p = 0; p < P; ++p) {
        const int64_t idx[3] = {p % nx, (p / nx) % ny, p / ((int64_t)nx * ny)};
        for (int k = 0; k < 3; ++k)
            h_pos[3 * p + k] = (float)(probes->origin[k] + probes->spacing[k] * (double)idx[k]);
    }
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
    for (int t = 0; t < c->Ti; ++t) {
        texel_direction(params->irr_res, t % params->irr_res, t / params->irr_res, &h_ti[3 * t]);
        for (int k = 0; k < 3; ++k) h_tif[3 * t + k] = (float)h_ti[3 * t + k];
    }
    for (int t = 0; t < c->Td; ++t)
        texel_direction(params->depth_res, t % params->depth_res, t / params->depth_res,
                        &h_td[3 * t]);

    hipError_t ce = hipSuccess;
    auto chk = [&](hipError_t x) { if (ce == hipSuccess) ce = x; };
    chk(dev_alloc(&c->probe_pos, 3 * P));
    chk(dev_alloc(&c->grid_pos, 3 * P));
    chk(dev_alloc(&c->probe_order, P));
    chk(dev_alloc(&c->texel_i, 3 * c->Ti));
    chk(dev_alloc(&c->texel_d, 3 * c->Td));
    if (ce == hipSuccess) {
        chk(hipMemcpy(c->probe_pos, h_pos.data(), 3 * P * sizeof(float), hipMemcpyHostToDevice));
        chk(hipMemcpy(c->grid_pos, h_pos.data(), 3 * P * sizeof(float), hipMemcpyHostToDevice));
        chk(hipMemcpy(c->probe_order, h_order.data(), P * sizeof(int32_t), hipMemcpyHostToDevice));
        chk(hipMemcpy(c->texel_i, h_ti.data(), 3 * c->Ti * sizeof(double), hipMemcpyHostToDevice));
        chk(hipMemcpy(c->texel_d, h_td.data(), 3 * c->Td * sizeof(double), hipMemcpyHostToDevice));
    }
    SDF_TRY(ce, "uploading constants");

    // the grid backends split the pipelined frames' hit shading (geometry records)
    SDF_TRY(alloc_set(c, c->main, params->rays_per_probe, !c->analytic),
            "allocating the ray set");
    SDF_TRY(alloc_set(c, c->spare, params->rays_per_probe, !c->analytic),
            "allocating the ray set");
    SDF_TRY(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking), "creating a stream");
    SDF_TRY(hipEventCreateWithFlags(&c->ev_primary, hipEventDisableTiming), "creating events");
    SDF_TRY(hipEventCreateWithFlags(&c->ev_tail, hipEventDisableTiming), "creating events");
    SDF_TRY(hipStreamCreateWithFlags(&c->side2, hipStreamNonBlocking), "creating a stream");
    SDF_TRY(hipStreamCreateWithFlags(&c->side3, hipStreamNonBlocking), "creating a stream");
    SDF_TRY(hipEventCreateWithFlags(&c->ev_end, hipEventDisableTiming), "creating events");
    SDF_TRY(hipEventRecord(c->ev_end, c->stream), "event");
    for (RaySet *r : {&c->main, &c->spare}) {
        SDF_TRY(hipEventCreateWithFlags(&r->done, hipEventDisableTiming), "creating events");
        SDF_TRY(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming), "creating events");
        SDF_TRY(hipEventRecord(r->done, c->stream), "event");
    }
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
    SDF_TRY(dev_alloc(&c->counter, kCounters), "allocating ray counters");
    SDF_TRY(hipMemsetAsync(c->counter, 0, kCounters * sizeof(int), c->stream),
            "clearing counters");
    if (params->flags & SDFDDGI_FLAG_RECORD_RAYS)
        SDF_TRY(dev_alloc(&c->records, (size_t)P * c->main.R * 8), "allocating ray records");
    if (params->learned_rays > 0) {
        for (int k = 0; k < 2; ++k) {
            SDF_TRY(alloc_set(c, c->low[k], params->learned_rays, true),
                    "allocating the learned ray sets");
            SDF_TRY(alloc_set(c, c->fbs[k], params->rays_per_probe, true),
                    "allocating the learned ray sets");
        }
        for (RaySet *r : {&c->low[0], &c->low[1], &c->fbs[0], &c->fbs[1]}) {
            SDF_TRY(hipEventCreateWithFlags(&r->done, hipEventDisableTiming), "creating events");
            SDF_TRY(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming), "creating events");
            SDF_TRY(hipEventCreateWithFlags(&r->sel, hipEventDisableTiming), "creating events");
            SDF_TRY(hipEventRecord(r->done, c->stream), "event");
        }
        for (int k = 0; k < 2; ++k) {
            SDF_TRY(dev_alloc(&c->fb_flag[k], P), "allocating learned buffers");
            SDF_TRY(launch_fill_u8(c->fb_flag[k], 1, P, c->stream), "launching fill");
        }
        SDF_TRY(dev_alloc(&c->u_irr, c->irr_floats), "allocating learned buffers");
        SDF_TRY(dev_alloc(&c->u_depth, c->depth_floats), "allocating learned buffers");
        SDF_TRY(dev_alloc(&c->probe_sdf, P), "allocating learned buffers");
        SDF_TRY(dev_alloc(&c->texel_dir, 3 * c->Ti), "allocating learned buffers");
        SDF_TRY(dev_alloc(&c->mean_error, P), "allocating learned buffers");
        SDF_TRY(hipMemcpy(c->texel_dir, h_tif.data(), 3 * c->Ti * sizeof(float),
                          hipMemcpyHostToDevice),
                "uploading texel directions");
        const float l[3] = {0.0f, 1.0f, 0.0f}, rad[3] = {0.0f, 0.0f, 0.0f};
        SDF_TRY(launch_probe_sdf(trace_base(c, l, rad), c->probe_sdf, c->stream),
                "launching probe_sdf_kernel");
    }
    {
        // every ray of a probe takes its first sample at the probe
        const float l[3] = {0.0f, 1.0f, 0.0f}, rad[3] = {0.0f, 0.0f, 0.0f};
        SDF_TRY(dev_alloc(&c->probe_first, P), "allocating probe samples");
        SDF_TRY(launch_probe_first(trace_base(c, l, rad), c->probe_first, c->stream),
                "launching probe_first_kernel");
    }
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

extern "C" {

sdfddgi_status sdfddgi_create(const sdfddgi_sdf_grid *sdf, const sdfddgi_probe_grid *probes,
                              const sdfddgi_params *params, void *hip_stream, sdfddgi_ctx **out) {
    g_create_error.clear();
    if (!out) return fail(nullptr, SDFDDGI_EINVAL, "out is NULL");
    *out = nullptr;
    sdfddgi_status st = validate(sdf, probes, params);
    if (st != SDFDDGI_OK) return st;
    return create_ctx(sdf, nullptr, probes, params, hip_stream, out);
}

sdfddgi_status sdfddgi_create_analytic(int32_t nprims, const int32_t *kind, const double *center,
                                       const double *half, const double *albedo,
                                       int32_t cluster_size, const sdfddgi_probe_grid *probes,
                                       const sdfddgi_params *params, void *hip_stream,
                                       sdfddgi_ctx **out) {
    g_create_error.clear();
    if (!out) return fail(nullptr, SDFDDGI_EINVAL, "out is NULL");
    *out = nullptr;
    sdfddgi_status st = validate_probes_params(probes, params);
    if (st != SDFDDGI_OK) return st;
    if (params->flags & SDFDDGI_FLAG_FP16)
        return fail(nullptr, SDFDDGI_EINVAL, "the precision form stores a grid: not analytic");
    if (params->learned_rays != 0)
        return fail(nullptr, SDFDDGI_EINVAL, "the learned form needs a grid: learned_rays must be 0");
    if (!albedo) return fail(nullptr, SDFDDGI_EINVAL, "albedo is NULL");
    HostClusters hc;
    const std::string why = build_clusters(nprims, kind, center, half, albedo, cluster_size, hc);
    if (!why.empty()) return fail(nullptr, SDFDDGI_EINVAL, "%s", why.c_str());
    return create_ctx(nullptr, &hc, probes, params, hip_stream, out);
}

sdfddgi_status sdfddgi_update_frame(sdfddgi_ctx *c, const sdfddgi_light *light,
                                    uint64_t rotation_seed) {
    // overlap with the previous frame only when nothing else came in between and no
    // per-ray records are kept (they are one buffer for both frames)
    const bool serial = !c || c->serialize_next || c->records || c->learned_chain;
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    c->learned_chain = false;
    float l[3], rad[3];
    if ((st = light_of(c, light, l, rad)) != SDFDDGI_OK) return st;
    RaySet &r = c->spare;  // becomes main once every launch has gone in
    const TraceArgs t = trace_pass(trace_base(c, l, rad), r, r.counter, r.counter + kPartStride,
                                   nullptr, nullptr, c->records);
    FrameEvents ev = frame_events(c);
    const int nxt = 1 - c->cur;
    // Split hit shading when pipelined on a grid: the atlas-independent half on side2
    // right after the trace, only the lookups behind the previous frame's blend
    // (16384 x 256, ms per frame, FP32 / FP16: 0.7275 / 0.590 unsplit, 0.719 /
    // 0.576 split; that half's grid halved 0.736, not overlapped 0.734 in FP32)
    const bool split = !serial && r.geo != nullptr;
    // side stream: tables and primary trace. This set was last used by the frame
    // before the previous one, whose hit shading and blend ran before that set's
    // done event; so wait for that (the trace then starts as soon as its set is
    // free), or, when serial, for everything enqueued so far
    if (serial) {
        TRY_HIP(c, hipEventRecord(c->ev_tail, c->stream), "event");
        TRY_HIP(c, hipStreamWaitEvent(c->side, c->ev_tail, 0), "stream wait");
    } else {
        TRY_HIP(c, hipStreamWaitEvent(c->side, r.done, 0), "stream wait");
    }
    TRY_HIP(c, ev.mark_on(0, c->side), "event");
    const TableArgs ta = table_args(c, r, rotation_seed, kSetCounters, r.counter);
    if (split) {
        // only the directions block (which also resets the counters) ahead of the
        // trace; the weight rows, which only the blend reads, on side2 beside it
        // (16384 x 256: 0.692 -> 0.680 ms per FP32 frame, 0.574 -> 0.561 FP16)
        TRY_HIP(c, hipStreamWaitEvent(c->side2, r.done, 0), "stream wait");
        TRY_HIP(c, ev.mark_on(12, c->side2), "event");
        TRY_HIP(c, launch_tables_weights(ta, c->side2), "launching tables_kernel");
        TRY_HIP(c, ev.mark_on(13, c->side2), "event");
        TRY_HIP(c, launch_tables_dirs(ta, c->side), "launching tables_kernel");
    } else {
        TRY_HIP(c, ev.mark_on(12, c->side), "event");
        TRY_HIP(c, launch_tables(ta, c->side), "launching tables_kernel");
        TRY_HIP(c, ev.mark_on(13, c->side), "event");
    }
    TRY_HIP(c, ev.mark_on(1, c->side), "event");
    // overlapped frames share the GPU with the other stream's kernels: their own grids
    TraceGrid g = r.grid;
    if (!serial) {
        g.primary_blocks = r.grid.primary_blocks_overlapped;
        g.hits_blocks = r.grid.hits_blocks_overlapped;
    }
    TRY_HIP(c, launch_primary(t, g, c->side), "launching primary_kernel");
    TRY_HIP(c, ev.mark_on(2, c->side), "event");
    TRY_HIP(c, hipEventRecord(c->ev_primary, c->side), "event");
    if (split) {
        // side2, after the weight rows: the atlas-independent half of the hit
        // shading; then the caller's stream, after the previous frame's blend: the
        // lookups into its atlas
        TraceArgs tg = t;
        tg.geo = r.geo;
        TRY_HIP(c, hipStreamWaitEvent(c->side2, c->ev_primary, 0), "stream wait");
        TRY_HIP(c, ev.mark_on(3, c->side2), "event");
        TRY_HIP(c, launch_hits(tg, g, c->side2), "launching hits_kernel");
        TRY_HIP(c, hipEventRecord(r.ready, c->side2), "event");
        TRY_HIP(c, hipStreamWaitEvent(c->stream, r.ready, 0), "stream wait");
        TRY_HIP(c, launch_shade(tg, c->stream), "launching shade_kernel");
    } else {
        // caller's stream: hit shading (reads the previous atlas, so after the
        // previous frame's blend)
        TRY_HIP(c, hipStreamWaitEvent(c->stream, c->ev_primary, 0), "stream wait");
        TRY_HIP(c, ev.mark(3), "event");
        TRY_HIP(c, launch_hits(t, g, c->stream), "launching hits_kernel");
    }
    TRY_HIP(c, ev.mark(4), "event");
    TRY_HIP(c, launch_blend(blend_args(c, r, r.payload, c->prm.hysteresis, c->irr[c->cur],
                                       c->depth[c->cur], c->irr[nxt], c->depth[nxt], c->reject,
                                       nullptr, nullptr),
                            c->stream),
            "launching blend_kernel");
    // the learned form's marks are not recorded (their spans read as 0)
    TRY_HIP(c, ev.mark(5), "event");
    TRY_HIP(c, ev.mark(10), "event");
    TRY_HIP(c, hipEventRecord(r.done, c->stream), "event");
    frame_done(c, false);
    std::swap(c->main, c->spare);
    c->cur = nxt;
    c->have_frame = true;
    c->have_records = c->records != nullptr;
    c->serialize_next = false;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_blend(sdfddgi_ctx *c, const float *payload, uint64_t rotation_seed) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!payload) return fail(c, SDFDDGI_EINVAL, "payload is NULL");
    const int nxt = 1 - c->cur;
    TRY_HIP(c, launch_tables(table_args(c, c->main, rotation_seed, 0), c->stream),
            "launching tables_kernel");
    TRY_HIP(c, launch_blend(blend_args(c, c->main, (const float4 *)payload, c->prm.hysteresis,
                                       c->irr[c->cur], c->depth[c->cur], c->irr[nxt],
                                       c->depth[nxt], c->reject, nullptr, nullptr),
                            c->stream),
            "launching blend_kernel");
    c->cur = nxt;
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
    TRY_HIP(c, launch_sample(a, c->stream), "launching sample_kernel");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_get_maps(sdfddgi_ctx *c, float *irr, float *depth) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (irr)
        TRY_HIP(c, hipMemcpyAsync(irr, c->irr[c->cur], c->irr_floats * sizeof(float),
                                  hipMemcpyDeviceToDevice, c->stream),
                "copying irradiance atlas");
    if (depth)
        TRY_HIP(c, hipMemcpyAsync(depth, c->depth[c->cur], c->depth_floats * sizeof(float),
                                  hipMemcpyDeviceToDevice, c->stream),
                "copying depth atlas");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_set_maps(sdfddgi_ctx *c, const float *irr, const float *depth) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!irr || !depth) return fail(c, SDFDDGI_EINVAL, "both maps are required");
    TRY_HIP(c, hipMemcpyAsync(c->irr[c->cur], irr, c->irr_floats * sizeof(float),
                              hipMemcpyDeviceToDevice, c->stream),
            "copying irradiance atlas");
    TRY_HIP(c, hipMemcpyAsync(c->depth[c->cur], depth, c->depth_floats * sizeof(float),
                              hipMemcpyDeviceToDevice, c->stream),
            "copying depth atlas");
    TRY_HIP(c, launch_fill_u8(c->reject, 0, c->P, c->stream), "launching fill");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_reset_history(sdfddgi_ctx *c) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    TRY_HIP(c, launch_fill_u8(c->reject, 1, c->P, c->stream), "launching fill");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_get_payload(sdfddgi_ctx *c, float *out) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!out) return fail(c, SDFDDGI_EINVAL, "out is NULL");
    if (!c->have_frame) return fail(c, SDFDDGI_ESTATE, "no frame has been traced yet");
    TRY_HIP(c, hipMemcpyAsync(out, c->main.payload, (size_t)c->P * c->main.R * sizeof(float4),
                              hipMemcpyDeviceToDevice, c->stream),
            "copying payload");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_get_ray_records(sdfddgi_ctx *c, int32_t *out) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!out) return fail(c, SDFDDGI_EINVAL, "out is NULL");
    if (!c->records) return fail(c, SDFDDGI_ESTATE, "created without SDFDDGI_FLAG_RECORD_RAYS");
    if (!c->have_records) return fail(c, SDFDDGI_ESTATE, "no frame has been traced yet");
    TRY_HIP(c, hipMemcpyAsync(out, c->records, (size_t)c->P * c->main.R * 8 * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, c->stream),
            "copying records");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_get_ray_directions(sdfddgi_ctx *c, float *out) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!out) return fail(c, SDFDDGI_EINVAL, "out is NULL");
    TRY_HIP(c, hipMemcpyAsync(out, c->main.dirs, (size_t)c->main.R * 3 * sizeof(float),
                              hipMemcpyDeviceToDevice, c->stream),
            "copying directions");
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
    if (!ms || count < 0 || count > 8) return fail(c, SDFDDGI_EINVAL, "bad output array");
    if (!c->ev_ring) return fail(c, SDFDDGI_ESTATE, "created without SDFDDGI_FLAG_TIMING");
    if (c->timed_frames == 0) return fail(c, SDFDDGI_ESTATE, "no timed frame since the last call");
    const int frames = (int)(c->timed_frames < kTimingRing ? c->timed_frames : kTimingRing);
    const int last = (c->ring_head + kTimingRing - 1) % kTimingRing;
    // mark 10 ends a frame: every other mark of the frame is complete by then
    TRY_HIP(c, hipEventSynchronize(c->ev_ring[kEvents * last + 10]),
            "hipEventSynchronize");
    // tables, primary, hits, blend, frame, denoiser, fallback trace, fallback blend
    // (the marks of FrameEvents; the last three are learned-only)
    constexpr int kTimes = 8;
    const int pairs[kTimes][2] = {{12, 13}, {1, 2}, {3, 4}, {4, 5}, {0, 10}, {5, 6}, {7, 8}, {11, 9}};
    double sum[kTimes] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int f = 0; f < frames; ++f) {
        const int slot = (last - f + kTimingRing) % kTimingRing;
        const hipEvent_t *ev = c->ev_ring + kEvents * slot;
        for (int k = 0; k < kTimes; ++k) {
            if (k >= 5 && !c->ring_learned[slot]) continue;
            float v = 0.0f;
            TRY_HIP(c, hipEventElapsedTime(&v, ev[pairs[k][0]], ev[pairs[k][1]]),
                    "hipEventElapsedTime");
            sum[k] += v;
        }
    }
    for (int k = 0; k < count; ++k) ms[k] = (float)(sum[k] / frames);
    c->timed_frames = 0;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_relocate_probes(sdfddgi_ctx *c, float threshold1, float threshold2,
                                       int32_t iterations, float max_offset) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (c->analytic) return fail(c, SDFDDGI_ESTATE, "relocation walks a grid: analytic context");
    const float v[3] = {threshold1, threshold2, max_offset};
    if (!finite_all(v, 3) || !(threshold2 >= 0) || !(max_offset >= 0) || iterations < 0 ||
        iterations > 1024)
        return fail(c, SDFDDGI_EINVAL, "relocation parameters out of range");
    RelocateArgs r{};
    r.grid_pos = c->grid_pos;
    r.pos = c->probe_pos;
    r.reject = c->reject;
    r.t1 = threshold1;
    r.t2 = threshold2;
    r.iterations = iterations;
    r.off0 = (float)((double)max_offset * c->pg.spacing[0]);
    r.off1 = (float)((double)max_offset * c->pg.spacing[1]);
    r.off2 = (float)((double)max_offset * c->pg.spacing[2]);
    const float l[3] = {0.0f, 1.0f, 0.0f}, rad[3] = {0.0f, 0.0f, 0.0f};
    const TraceArgs t = trace_base(c, l, rad);
    TRY_HIP(c, launch_relocate(t, r, c->stream), "launching relocate_kernel");
    if (c->probe_sdf)   // the learned form's feature follows the probe
        TRY_HIP(c, launch_probe_sdf(t, c->probe_sdf, c->stream), "launching probe_sdf_kernel");
    // and so does the rays' first sample
    TRY_HIP(c, launch_probe_first(t, c->probe_first, c->stream), "launching probe_first_kernel");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_get_probe_positions(sdfddgi_ctx *c, float *out) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!out) return fail(c, SDFDDGI_EINVAL, "out is NULL");
    TRY_HIP(c, hipMemcpyAsync(out, c->probe_pos, (size_t)c->P * 3 * sizeof(float),
                              hipMemcpyDeviceToDevice, c->stream),
            "copying probe positions");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_get_sizes(const sdfddgi_ctx *c, int64_t *probes, int32_t *rays,
                                 int64_t *irr_floats, int64_t *depth_floats) {
    if (!c) return SDFDDGI_EINVAL;
    if (probes) *probes = c->P;
    if (rays) *rays = c->main.R;
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
    if (c->side) (void)hipStreamSynchronize(c->side);
    if (c->side2) (void)hipStreamSynchronize(c->side2);
    if (c->side3) (void)hipStreamSynchronize(c->side3);
    free_all(c);
    delete c;
    return SDFDDGI_OK;
}

// ------------------------------------------------------------ learned form --

sdfddgi_status sdfddgi_denoiser_create(const float *params, int32_t count, float irr_scale,
                                       float depth_scale, void *hip_stream,
                                       sdfddgi_denoiser **out) {
    g_learned_error.clear();
    if (!out) return lfail(SDFDDGI_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params || count != kMlpParams)
        return lfail(SDFDDGI_EINVAL, "need %d parameters, got %d", kMlpParams, count);
    if (!finite_all(params, kMlpParams)) return lfail(SDFDDGI_EINVAL, "non-finite parameter");
    (void)hipGetLastError();
    if (!(irr_scale > 0) || !(depth_scale > 0) || !std::isfinite(irr_scale) ||
        !std::isfinite(depth_scale))
        return lfail(SDFDDGI_EINVAL, "feature scales must be finite and > 0");
    sdfddgi_denoiser *d = new (std::nothrow) sdfddgi_denoiser();
    if (!d) return lfail(SDFDDGI_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&d->device);
    d->stream = (hipStream_t)hip_stream;
    d->S = irr_scale;
    d->D = depth_scale;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(dev_alloc(&d->theta, kMlpParams));
    chk(dev_alloc(&d->fwd, kFwdEntries * 64));
    chk(dev_alloc(&d->bwd, kBwdEntries * 64));
    chk(dev_alloc(&d->bias, kBiasFloats));
    if (e == hipSuccess)
        chk(hipMemcpy(d->theta, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice));
    if (e == hipSuccess) chk(launch_pack_mlp(d->theta, d->fwd, d->bwd, d->bias, d->stream));
    if (e == hipSuccess) chk(hipStreamSynchronize(d->stream));
    if (e != hipSuccess) {
        sdfddgi_denoiser_destroy(d);
        return lhip_fail(e, "creating the denoiser");
    }
    *out = d;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_denoiser_infer(sdfddgi_denoiser *d, const float *features, int64_t n,
                                      float *out) {
    g_learned_error.clear();
    if (!d) return lfail(SDFDDGI_EINVAL, "denoiser is NULL");
    if (n < 0) return lfail(SDFDDGI_EINVAL, "negative count");
    if (n == 0) return SDFDDGI_OK;
    if (!features || !out) return lfail(SDFDDGI_EINVAL, "null array");
    (void)hipGetLastError();
    hipError_t e = hipSetDevice(d->device);
    if (e != hipSuccess) return lhip_fail(e, "hipSetDevice");
    InferArgs a{};
    a.n = n;
    a.features = features;
    a.out = out;
    a.mlp = MlpPack{d->fwd, d->bwd, d->bias};
    if ((e = launch_infer(a, d->stream)) != hipSuccess) return lhip_fail(e, "launching infer_kernel");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_denoiser_destroy(sdfddgi_denoiser *d) {
    if (!d) return SDFDDGI_OK;
    (void)hipSetDevice(d->device);
    (void)hipStreamSynchronize(d->stream);
    dev_free(d->theta); dev_free(d->fwd); dev_free(d->bwd); dev_free(d->bias);
    delete d;
    return SDFDDGI_OK;
}

static FeatureArgs feature_args(const sdfddgi_ctx *c, const sdfddgi_denoiser *d) {
    FeatureArgs f{};
    f.irr_res = c->prm.irr_res;
    f.depth_res = c->prm.depth_res;
    f.inv_s = (float)(1.0 / (double)d->S);
    f.inv_d = (float)(1.0 / (double)d->D);
    f.u_irr = c->u_irr;
    f.prev_irr = c->irr[c->cur];
    f.prev_depth = c->depth[c->cur];
    f.probe_sdf = c->probe_sdf;
    f.texel_dir = c->texel_dir;
    return f;
}

static sdfddgi_status check_learned(sdfddgi_ctx *c, const sdfddgi_denoiser *d) {
    if (!c->low[0].R) return fail(c, SDFDDGI_ESTATE, "context created with learned_rays == 0");
    if (!d) return fail(c, SDFDDGI_EINVAL, "denoiser is NULL");
    if (d->device != c->device) return fail(c, SDFDDGI_EINVAL, "denoiser is on another device");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_update_frame_learned(sdfddgi_ctx *c, const sdfddgi_denoiser *d,
                                            const sdfddgi_light *light, uint64_t rotation_seed) {
    const bool serial = !c || c->serialize_next || c->records || !c->learned_chain;
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    c->learned_chain = false;
    if ((st = check_learned(c, d)) != SDFDDGI_OK) return st;
    float l[3], rad[3];
    if ((st = light_of(c, light, l, rad)) != SDFDDGI_OK) return st;
    const TraceArgs base = trace_base(c, l, rad);
    const int nxt = 1 - c->cur, k = (int)(c->learned_index % 2);
    FrameEvents ev = frame_events(c);
    RaySet &lo = c->low[k], &fb = c->fbs[k];
    hipStream_t sides[3] = {c->side, c->side2, c->side3};
    hipStream_t sl = sides[(2 * c->learned_index) % 3], sf = sides[(2 * c->learned_index + 1) % 3];
    if (serial) {
        // after everything so far, and then the reject flags join the flags
        TRY_HIP(c, hipEventRecord(c->ev_tail, c->stream), "event");
        TRY_HIP(c, hipStreamWaitEvent(sl, c->ev_tail, 0), "stream wait");
        TRY_HIP(c, hipStreamWaitEvent(sf, c->ev_tail, 0), "stream wait");
    } else {
        // back to back, no reject flag is set: the fallback blend of every frame clears
        // those of its probes, and a frame with a rejected history is serial
        TRY_HIP(c, hipStreamWaitEvent(sl, lo.done, 0), "stream wait");
        TRY_HIP(c, hipStreamWaitEvent(sf, fb.done, 0), "stream wait");
    }
    // low chain: the low-ray pass over every probe up to the atlas-independent half of
    // its hit shading
    TraceArgs tl = trace_pass(base, lo, lo.counter, lo.counter + kPartStride, nullptr, nullptr,
                              nullptr);
    tl.geo = lo.geo;
    TRY_HIP(c, ev.mark_on(0, sl), "event");
    // only the directions block (it also resets the counters) ahead of the low
    // trace; the weight rows, which only the low-ray blend reads, on the caller's
    // stream before it
    const TableArgs tal = table_args(c, lo, rotation_seed, kSetCounters, lo.counter);
    TRY_HIP(c, ev.mark_on(12, sl), "event");
    TRY_HIP(c, launch_tables_dirs(tal, sl), "launching tables_kernel");
    TRY_HIP(c, ev.mark_on(13, sl), "event");
    TRY_HIP(c, ev.mark_on(1, sl), "event");
    // The side chains run on small grids, so that the caller's stream -- the lookups,
    // Eq. 3 and the network, the frame's critical chain -- keeps most of the GPU:
    // measured at 16384 probes (FP16 / FP32 ms per frame, median of three 20-frame
    // windows), full and overlapped grids 0.323 / 0.346; low primary at half the
    // full grid and the rest at half the overlapped grids 0.275 / 0.298; the
    // fallback primary at a quarter 0.272 / 0.296; a quarter everywhere 0.289 / 0.319
    TraceGrid gl = lo.grid;
    gl.primary_blocks = std::max(1, gl.primary_blocks / 2);
    gl.hits_blocks = std::max(1, gl.hits_blocks_overlapped / 2);
    TRY_HIP(c, launch_primary(tl, gl, sl), "launching primary_kernel");
    TRY_HIP(c, ev.mark_on(2, sl), "event");
    TRY_HIP(c, ev.mark_on(3, sl), "event");
    TRY_HIP(c, launch_hits(tl, gl, sl), "launching hits_kernel");
    TRY_HIP(c, hipEventRecord(lo.ready, sl), "event");
    // fallback chain: the list -- probes whose flag of this parity asks for the plain
    // update (the decision of the learned frame before the previous one; set in every
    // probe until then) or, when serial, whose history is rejected -- then the
    // fallback probes' pass, on small grids (see the low chain)
    int *fb_count = fb.counter + 6;
    TraceArgs tf = trace_pass(base, fb, fb.counter, fb.counter + kPartStride, fb.list, fb_count,
                              nullptr);
    tf.geo = fb.geo;
    TraceGrid gf = fb.grid;
    gf.primary_blocks = std::max(1, gf.primary_blocks_overlapped / 4);
    gf.hits_blocks = std::max(1, gf.hits_blocks_overlapped / 2);
    TRY_HIP(c, ev.mark_on(7, sf), "event");
    // the fallback set's directions ahead of its trace, its weight rows (read by its
    // blend only) after it
    const TableArgs taf = table_args(c, fb, rotation_seed, kSetCounters, fb.counter);
    TRY_HIP(c, launch_tables_dirs(taf, sf), "launching tables_kernel");
    TRY_HIP(c, launch_select_fallback(serial ? c->reject : nullptr, c->fb_flag[k], (int)c->P,
                                      fb.list, fb_count, sf),
            "launching select_fallback_kernel");
    TRY_HIP(c, hipEventRecord(fb.sel, sf), "event");
    TRY_HIP(c, launch_primary(tf, gf, sf), "launching primary_kernel");
    TRY_HIP(c, launch_hits(tf, gf, sf), "launching hits_kernel");
    TRY_HIP(c, launch_tables_weights(taf, sf), "launching tables_kernel");
    TRY_HIP(c, ev.mark_on(8, sf), "event");
    TRY_HIP(c, hipStreamWaitEvent(sf, c->ev_end, 0), "stream wait");
    TRY_HIP(c, ev.mark_on(11, sf), "event");
    TRY_HIP(c, launch_shade(tf, sf), "launching shade_kernel");
    TRY_HIP(c, launch_blend(blend_args(c, fb, fb.payload, c->prm.hysteresis, c->irr[c->cur],
                                       c->depth[c->cur], c->irr[nxt], c->depth[nxt], c->reject,
                                       fb.list, fb_count),
                            sf),
            "launching blend_kernel");
    TRY_HIP(c, ev.mark_on(9, sf), "event");
    TRY_HIP(c, hipEventRecord(fb.ready, sf), "event");
    // caller's stream (the previous atlas is complete here): low-ray lookup half and
    // Eq. 3 without hysteresis
    TRY_HIP(c, hipStreamWaitEvent(c->stream, lo.ready, 0), "stream wait");
    TRY_HIP(c, launch_tables_weights(tal, c->stream), "launching tables_kernel");
    TRY_HIP(c, launch_shade(tl, c->stream), "launching shade_kernel");
    TRY_HIP(c, ev.mark(4), "event");
    TRY_HIP(c, launch_blend(blend_args(c, lo, lo.payload, 0.0f, c->irr[c->cur],
                                       c->depth[c->cur], c->u_irr, c->u_depth, nullptr, nullptr,
                                       nullptr),
                            c->stream),
            "launching blend_kernel");
    TRY_HIP(c, hipEventRecord(lo.done, c->stream), "event");
    TRY_HIP(c, ev.mark(5), "event");
    // the network over every probe once the flags of this parity name the frame's
    // fallback probes: maps of the others, every probe's prediction, and the flags
    // replaced by the decisions
    DenoiseArgs da{};
    da.f = feature_args(c, d);
    da.P = (int)c->P;
    da.hysteresis = c->prm.hysteresis;
    da.s = d->S;
    da.tau = c->prm.fallback_error;
    da.u_depth = c->u_depth;
    da.new_irr = c->irr[nxt];
    da.new_depth = c->depth[nxt];
    da.mlp = MlpPack{d->fwd, d->bwd, d->bias};
    da.fb_flag = c->fb_flag[k];
    da.mean_error = c->mean_error;
    TRY_HIP(c, hipStreamWaitEvent(c->stream, fb.sel, 0), "stream wait");
    TRY_HIP(c, launch_denoise(da, c->stream), "launching denoise_kernel");
    TRY_HIP(c, ev.mark(6), "event");
    // the fallback set is free again (its lookup half and blend read its list, counters
    // and payload) and the flags of this parity hold the decisions
    TRY_HIP(c, hipStreamWaitEvent(c->stream, fb.ready, 0), "stream wait");
    TRY_HIP(c, hipEventRecord(fb.done, c->stream), "event");
    TRY_HIP(c, ev.mark(10), "event");
    TRY_HIP(c, hipEventRecord(c->ev_end, c->stream), "event");
    ++c->learned_index;
    frame_done(c, true);
    c->last_learned = k;
    c->cur = nxt;
    c->have_learned = true;
    c->learned_chain = true;
    c->serialize_next = false;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_get_fallback(sdfddgi_ctx *c, int32_t *count, int32_t *probes,
                                    float *mean_error) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if (!count) return fail(c, SDFDDGI_EINVAL, "count is NULL");
    if (!c->have_learned) return fail(c, SDFDDGI_ESTATE, "no learned frame yet");
    const RaySet &fb = c->fbs[c->last_learned];
    TRY_HIP(c, hipMemcpyAsync(count, fb.counter + 6, sizeof(int32_t), hipMemcpyDeviceToHost,
                              c->stream),
            "copying the fallback count");
    if (probes)
        TRY_HIP(c, hipMemcpyAsync(probes, fb.list, c->P * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, c->stream),
                "copying the fallback list");
    if (mean_error)
        TRY_HIP(c, hipMemcpyAsync(mean_error, c->mean_error, c->P * sizeof(float),
                                  hipMemcpyDeviceToDevice, c->stream),
                "copying the mean errors");
    TRY_HIP(c, hipStreamSynchronize(c->stream), "waiting for the stream");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_learned_examples(sdfddgi_ctx *c, const sdfddgi_denoiser *d,
                                        const sdfddgi_light *light, uint64_t rotation_seed,
                                        const float *target_irr, float rel_floor,
                                        float *features, float *targets) {
    sdfddgi_status st = check_ctx(c);
    if (st != SDFDDGI_OK) return st;
    if ((st = check_learned(c, d)) != SDFDDGI_OK) return st;
    if (!target_irr || !features || !targets) return fail(c, SDFDDGI_EINVAL, "null array");
    if (!(rel_floor >= 0) || !std::isfinite(rel_floor))
        return fail(c, SDFDDGI_EINVAL, "rel_floor must be finite and >= 0");
    float l[3], rad[3];
    if ((st = light_of(c, light, l, rad)) != SDFDDGI_OK) return st;
    const TraceArgs base = trace_base(c, l, rad);
    RaySet &lo = c->low[0];
    TRY_HIP(c, launch_tables(table_args(c, lo, rotation_seed, kCounters), c->stream),
            "launching tables_kernel");
    const TraceArgs tl = trace_pass(base, lo, c->counter, c->counter + kPartStride, nullptr,
                                    nullptr, nullptr);
    TRY_HIP(c, launch_primary(tl, lo.grid, c->stream), "launching primary_kernel");
    TRY_HIP(c, launch_hits(tl, lo.grid, c->stream), "launching hits_kernel");
    TRY_HIP(c, launch_blend(blend_args(c, lo, lo.payload, 0.0f, c->irr[c->cur],
                                       c->depth[c->cur], c->u_irr, c->u_depth, nullptr, nullptr,
                                       nullptr),
                            c->stream),
            "launching blend_kernel");
    ExampleArgs ea{};
    ea.f = feature_args(c, d);
    ea.P = (int)c->P;
    ea.target_irr = target_irr;
    ea.rel_floor = rel_floor;
    ea.features = features;
    ea.targets = targets;
    TRY_HIP(c, launch_examples(ea, c->stream), "launching examples_kernel");
    return SDFDDGI_OK;
}

// ---------------------------------------------------------------- training --

sdfddgi_status sdfddgi_trainer_destroy(sdfddgi_trainer *t) {
    if (!t) return SDFDDGI_OK;
    (void)hipSetDevice(t->device);
    (void)hipStreamSynchronize(t->stream);
    t->loss = nullptr;  // the last element of the grad allocation, not an allocation
    dev_free(t->theta); dev_free(t->m); dev_free(t->v); dev_free(t->grad);
    dev_free(t->fwd); dev_free(t->bwd); dev_free(t->bias);
    delete t;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_trainer_create(const float *init, int32_t count,
                                      const sdfddgi_train_config *cfg, void *hip_stream,
                                      sdfddgi_trainer **out) {
    g_learned_error.clear();
    if (!out) return lfail(SDFDDGI_EINVAL, "out is NULL");
    *out = nullptr;
    if (!init || count != kMlpParams)
        return lfail(SDFDDGI_EINVAL, "need %d parameters, got %d", kMlpParams, count);
    if (!cfg) return lfail(SDFDDGI_EINVAL, "cfg is NULL");
    if (!finite_all(init, kMlpParams)) return lfail(SDFDDGI_EINVAL, "non-finite parameter");
    const float v[5] = {cfg->head_weight, cfg->min_error, cfg->beta1, cfg->beta2, cfg->eps};
    if (!finite_all(v, 5) || !(cfg->head_weight >= 0) || !(cfg->min_error > 0) ||
        !(cfg->beta1 >= 0 && cfg->beta1 < 1) || !(cfg->beta2 >= 0 && cfg->beta2 < 1) ||
        !(cfg->eps >= 0))
        return lfail(SDFDDGI_EINVAL, "bad training configuration");
    (void)hipGetLastError();
    sdfddgi_trainer *t = new (std::nothrow) sdfddgi_trainer();
    if (!t) return lfail(SDFDDGI_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&t->device);
    t->stream = (hipStream_t)hip_stream;
    t->cfg = *cfg;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(dev_alloc(&t->theta, kMlpParams));
    chk(dev_alloc(&t->m, kMlpParams));
    chk(dev_alloc(&t->v, kMlpParams));
    chk(dev_alloc(&t->grad, kMlpParams + 1));
    chk(dev_alloc(&t->fwd, kFwdEntries * 64));
    chk(dev_alloc(&t->bwd, kBwdEntries * 64));
    chk(dev_alloc(&t->bias, kBiasFloats));
    if (e == hipSuccess) {
        t->loss = t->grad + kMlpParams;
        chk(hipMemcpy(t->theta, init, kMlpParams * sizeof(float), hipMemcpyHostToDevice));
        chk(launch_zero_f32(t->m, kMlpParams, t->stream));
        chk(launch_zero_f32(t->v, kMlpParams, t->stream));
        chk(launch_pack_mlp(t->theta, t->fwd, t->bwd, t->bias, t->stream));
        chk(hipStreamSynchronize(t->stream));
    }
    if (e != hipSuccess) {
        t->loss = nullptr;
        sdfddgi_trainer_destroy(t);
        return lhip_fail(e, "creating the trainer");
    }
    *out = t;
    return SDFDDGI_OK;
}

static hipError_t run_train(sdfddgi_trainer *t, const float *features, const float *targets,
                            int64_t count, int32_t batch, uint64_t seed, int sequential) {
    (void)hipGetLastError();
    hipError_t e = launch_zero_f32(t->grad, kMlpParams + 1, t->stream);
    if (e != hipSuccess) return e;
    TrainArgs a{};
    a.features = features;
    a.targets = targets;
    a.count = count;
    a.batch = batch;
    a.seed = seed;
    a.sequential = sequential;
    a.mlp = MlpPack{t->fwd, t->bwd, t->bias};
    a.inv_n = (float)(1.0 / (double)batch);
    a.head_weight = t->cfg.head_weight;
    a.min_error = t->cfg.min_error;
    a.grad = t->grad;
    a.loss = t->loss;
    return launch_train(a, t->stream);
}

sdfddgi_status sdfddgi_trainer_gradient(sdfddgi_trainer *t, const float *features,
                                        const float *targets, int32_t n, float *grad,
                                        float *loss) {
    g_learned_error.clear();
    if (!t) return lfail(SDFDDGI_EINVAL, "trainer is NULL");
    if (n < 1 || !features || !targets) return lfail(SDFDDGI_EINVAL, "need n >= 1 samples");
    hipError_t e = hipSetDevice(t->device);
    if (e == hipSuccess) e = run_train(t, features, targets, n, n, 0, 1);
    if (e == hipSuccess && grad)
        e = hipMemcpyAsync(grad, t->grad, kMlpParams * sizeof(float), hipMemcpyDeviceToHost,
                           t->stream);
    if (e == hipSuccess && loss)
        e = hipMemcpyAsync(loss, t->loss, sizeof(float), hipMemcpyDeviceToHost, t->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(t->stream);
    if (e != hipSuccess) return lhip_fail(e, "computing the gradient");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_trainer_step(sdfddgi_trainer *t, const float *features,
                                    const float *targets, int64_t count, int32_t batch,
                                    uint64_t seed, float lr, float *loss) {
    g_learned_error.clear();
    if (!t) return lfail(SDFDDGI_EINVAL, "trainer is NULL");
    if (count < 1 || batch < 1 || !features || !targets)
        return lfail(SDFDDGI_EINVAL, "need count >= 1, batch >= 1 and both arrays");
    if (!(lr >= 0) || !std::isfinite(lr)) return lfail(SDFDDGI_EINVAL, "bad learning rate");
    hipError_t e = hipSetDevice(t->device);
    if (e == hipSuccess) e = run_train(t, features, targets, count, batch, seed, 0);
    if (e == hipSuccess) {
        ++t->step;
        AdamArgs a{};
        a.theta = t->theta;
        a.m = t->m;
        a.v = t->v;
        a.grad = t->grad;
        a.n = kMlpParams;
        a.lr = lr;
        a.beta1 = t->cfg.beta1;
        a.beta2 = t->cfg.beta2;
        a.eps = t->cfg.eps;
        a.c1 = (float)(1.0 / (1.0 - std::pow((double)t->cfg.beta1, (double)t->step)));
        a.c2 = (float)(1.0 / (1.0 - std::pow((double)t->cfg.beta2, (double)t->step)));
        e = launch_adam(a, t->stream);
    }
    if (e == hipSuccess) e = launch_pack_mlp(t->theta, t->fwd, t->bwd, t->bias, t->stream);
    if (e == hipSuccess && loss) {
        e = hipMemcpyAsync(loss, t->loss, sizeof(float), hipMemcpyDeviceToHost, t->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(t->stream);
    }
    if (e != hipSuccess) return lhip_fail(e, "training step");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_trainer_get_params(sdfddgi_trainer *t, float *params) {
    g_learned_error.clear();
    if (!t || !params) return lfail(SDFDDGI_EINVAL, "null argument");
    hipError_t e = hipSetDevice(t->device);
    if (e == hipSuccess)
        e = hipMemcpyAsync(params, t->theta, kMlpParams * sizeof(float), hipMemcpyDeviceToHost,
                           t->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(t->stream);
    if (e != hipSuccess) return lhip_fail(e, "copying parameters");
    return SDFDDGI_OK;
}

}  // extern "C"

// Argument checks shared by both bake entry points.
static sdfddgi_status check_bake_args(int32_t nprims, const int32_t *kind, const double *center,
                                      const double *half, const double *albedo, const int32_t n[3],
                                      const double origin[3], double spacing, const float *sdf) {
    if (nprims < 0 || !n || !origin || !sdf) return lfail(SDFDDGI_EINVAL, "null or negative argument");
    if (nprims > 0 && (!kind || !center || !half || !albedo))
        return lfail(SDFDDGI_EINVAL, "primitive arrays are NULL");
    if (n[0] < 2 || n[1] < 2 || n[2] < 2 || (int64_t)n[0] * n[1] * n[2] >= (int64_t)1 << 31)
        return lfail(SDFDDGI_EINVAL, "grid size out of range");
    if (!(spacing > 0) || !std::isfinite(spacing) || !std::isfinite(origin[0]) ||
        !std::isfinite(origin[1]) || !std::isfinite(origin[2]))
        return lfail(SDFDDGI_EINVAL, "spacing and origin must be finite, spacing > 0");
    for (int32_t m = 0; m < nprims; ++m)
        if (kind[m] != 0 && kind[m] != 1) return lfail(SDFDDGI_EINVAL, "primitive kind %d", kind[m]);
    return SDFDDGI_OK;
}

static BakeArgs bake_args(int32_t nprims, const int *d_kind, const double *d_prm, size_t stride,
                          const int32_t n[3], const double origin[3], double spacing,
                          float empty_value, float *sdf, float *albedo_out) {
    BakeArgs a{};
    a.nprims = nprims;
    a.kind = d_kind;
    a.center = d_prm;
    a.half = d_prm + 3 * stride;
    a.albedo = d_prm + 6 * stride;
    a.n0 = n[0]; a.n1 = n[1]; a.n2 = n[2];
    a.org0 = origin[0]; a.org1 = origin[1]; a.org2 = origin[2];
    a.spacing = spacing;
    a.empty_value = empty_value;
    a.sdf = sdf;
    a.alb = albedo_out;
    return a;
}

// Staging of sdfddgi_bake_sdf_noalloc's primitives: center | half | albedo
// (binary64, SDFDDGI_BAKE_NOALLOC_MAX_PRIMS x 3 each), then the kinds (int32).
// Each device holds its own copy for the life of the process; host code reaches it
// only through the address hipGetSymbolAddress gives for the current device.
constexpr size_t kBakeScratchDoubles = (size_t)9 * SDFDDGI_BAKE_NOALLOC_MAX_PRIMS;
constexpr size_t kBakeScratchBytes =
    kBakeScratchDoubles * sizeof(double) + (size_t)SDFDDGI_BAKE_NOALLOC_MAX_PRIMS * sizeof(int32_t);
static __device__ __align__(256) unsigned char scratch[kBakeScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices];   // device address of `scratch` per device, once known
}  // namespace

// The current device's address of `scratch`, looked up on the first call on that device.
static hipError_t bake_scratch(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

extern "C" {

sdfddgi_status sdfddgi_bake_sdf(int32_t nprims, const int32_t *kind, const double *center,
                                const double *half, const double *albedo, const int32_t n[3],
                                const double origin[3], double spacing, float empty_value,
                                float *sdf, float *albedo_out, void *hip_stream) {
    g_learned_error.clear();
    sdfddgi_status st0 = check_bake_args(nprims, kind, center, half, albedo, n, origin, spacing, sdf);
    if (st0 != SDFDDGI_OK) return st0;
    (void)hipGetLastError();
    hipStream_t st = (hipStream_t)hip_stream;
    int *d_kind = nullptr;
    double *d_prm = nullptr;   // center | half | albedo
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    const size_t np = (size_t)(nprims > 0 ? nprims : 1);
    chk(dev_alloc(&d_kind, np));
    chk(dev_alloc(&d_prm, 9 * np));
    if (e == hipSuccess && nprims > 0) {
        chk(hipMemcpy(d_kind, kind, nprims * sizeof(int), hipMemcpyHostToDevice));
        chk(hipMemcpy(d_prm, center, 3 * nprims * sizeof(double), hipMemcpyHostToDevice));
        chk(hipMemcpy(d_prm + 3 * np, half, 3 * nprims * sizeof(double), hipMemcpyHostToDevice));
        chk(hipMemcpy(d_prm + 6 * np, albedo, 3 * nprims * sizeof(double), hipMemcpyHostToDevice));
    }
    if (e == hipSuccess) {
        chk(launch_bake(bake_args(nprims, d_kind, d_prm, np, n, origin, spacing, empty_value,
                                  sdf, albedo_out), st));
        chk(hipStreamSynchronize(st));
    }
    dev_free(d_kind);
    dev_free(d_prm);
    if (e != hipSuccess) return lhip_fail(e, "baking");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_bake_sdf_noalloc(int32_t nprims, const int32_t *kind, const double *center,
                                        const double *half, const double *albedo,
                                        const int32_t n[3], const double origin[3], double spacing,
                                        float empty_value, float *sdf, float *albedo_out,
                                        void *hip_stream) {
    g_learned_error.clear();
    sdfddgi_status st0 = check_bake_args(nprims, kind, center, half, albedo, n, origin, spacing, sdf);
    if (st0 != SDFDDGI_OK) return st0;
    if (nprims > SDFDDGI_BAKE_NOALLOC_MAX_PRIMS)
        return lfail(SDFDDGI_EINVAL, "%d primitives: this entry point stages at most %d",
                     nprims, SDFDDGI_BAKE_NOALLOC_MAX_PRIMS);
    (void)hipGetLastError();
    hipStream_t st = (hipStream_t)hip_stream;
    void *base = nullptr;
    hipError_t e = bake_scratch(&base);
    if (e != hipSuccess) return lhip_fail(e, "looking up the staging buffer");
    double *d_prm = static_cast<double *>(base);
    int *d_kind = reinterpret_cast<int *>(d_prm + kBakeScratchDoubles);
    const size_t stride = (size_t)SDFDDGI_BAKE_NOALLOC_MAX_PRIMS;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    if (nprims > 0) {
        // every staged value is written before the kernel reads it: nothing to clear
        chk(hipMemcpyAsync(d_kind, kind, nprims * sizeof(int), hipMemcpyHostToDevice, st));
        chk(hipMemcpyAsync(d_prm, center, 3 * nprims * sizeof(double), hipMemcpyHostToDevice, st));
        chk(hipMemcpyAsync(d_prm + 3 * stride, half, 3 * nprims * sizeof(double),
                           hipMemcpyHostToDevice, st));
        chk(hipMemcpyAsync(d_prm + 6 * stride, albedo, 3 * nprims * sizeof(double),
                           hipMemcpyHostToDevice, st));
    }
    chk(launch_bake(bake_args(nprims, d_kind, d_prm, stride, n, origin, spacing, empty_value,
                              sdf, albedo_out), st));
    chk(hipStreamSynchronize(st));   // the host arrays and the staging are free again
    if (e != hipSuccess) return lhip_fail(e, "baking");
    return SDFDDGI_OK;
}

const char *sdfddgi_learned_last_error(void) { return g_learned_error.c_str(); }

sdfddgi_status sdfddgi_measure_gather(const void *buf, int64_t bytes, int64_t threads,
                                      int32_t reads, uint64_t seed, float *sink,
                                      void *hip_stream) {
    g_learned_error.clear();
    if (!buf || !sink) return lfail(SDFDDGI_EINVAL, "null buffer");
    const int64_t records = bytes / 32;
    if (bytes % 32 || records < 1 || (records & (records - 1)) || records > ((int64_t)1 << 31))
        return lfail(SDFDDGI_EINVAL, "bytes must be 32 times a power of two, at most 64 GiB");
    if (reads < 8 || reads > 4096 || reads % 8)
        return lfail(SDFDDGI_EINVAL, "reads must be a multiple of 8 in 8..4096");
    if (threads < 1 || threads > ((int64_t)1 << 30))
        return lfail(SDFDDGI_EINVAL, "threads must be in 1..2^30");
    (void)hipGetLastError();
    const hipError_t e = launch_gather(buf, records, threads, reads, (uint32_t)(seed ^ (seed >> 32)),
                                       sink, (hipStream_t)hip_stream);
    if (e != hipSuccess) return lhip_fail(e, "launching gather_kernel");
    return SDFDDGI_OK;
}

}  // extern "C"

// ------------------------------------------------------------ batched form --

namespace {

constexpr int kFrameSlots = 8;   // pinned staging slots of the per-frame constants

// One ray count's direction set and, per lane (see sdfddgi_batch), its tables.
struct BatchSet {
    int R = 0, dir_base = 0;
    double *base = nullptr;
    _Float16 *w16_i[2]{};
    __bf16 *w16_d[2]{};
    float *norm_i[2]{}, *norm_d[2]{};
};

}  // namespace

struct sdfddgi_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int S = 0;
    int64_t GP = 0, total_rays = 0;
    double sharp = 50.0;
    std::vector<sdfddgi_batch_scene> scenes;
    std::vector<BatchScene> host_scenes;
    std::vector<BatchSet> sets;
    void *quad[kMaxBatchScenes]{};
    float *alb[kMaxBatchScenes]{};
    // Frames are pipelined like the single-scene ones: the tables and primary trace
    // of frame f (the front graph, on the side stream) run beside frame f-1's hit
    // shading and blend (the back graph, on the caller's stream). Everything a
    // frame writes before its blend comes in two lanes; frame f uses lane f mod 2,
    // the same parity as the map pair it reads (cur).
    BatchScene *dev_scenes[2]{};              // per lane: the lane's table pointers
    float *probe_pos = nullptr, *dirs[2]{};
    int *probe_order = nullptr;
    double *texel_i = nullptr, *texel_d = nullptr;
    float *irr[2]{}, *depth[2]{};
    int cur = 0;
    uint8_t *reject = nullptr;
    float4 *payload[2]{};
    int4 *hitq[2]{};
    int *counter[2]{};
    unsigned long long *stamps[2]{};         // [1 + S] per lane
    int last_lane = 0;                       // lane of the last frame
    int2 *blocks = nullptr;
    int nblocks = 0;
    // per-frame constants on the device: rotation (9 doubles) then lights [S][6]
    char *frame_dev[2]{};
    char *frame_host[kFrameSlots]{};          // pinned
    hipEvent_t frame_ev[kFrameSlots]{};
    bool frame_used[kFrameSlots]{};
    int slot = 0;
    size_t frame_bytes = 0;
    BatchTuning tuning{};
    hipGraph_t front[2]{}, back[2]{};
    hipGraphExec_t front_exec[2]{}, back_exec[2]{};
    hipStream_t side = nullptr;
    hipEvent_t ev_gate = nullptr, ev_primary = nullptr, ev_tail = nullptr;
    bool serialize_next = true;              // the next frame waits for everything before it
    bool have_frame = false;
};

namespace {

void batch_drop_graphs(sdfddgi_batch *b) {
    for (int k = 0; k < 2; ++k) {
        if (b->front_exec[k]) (void)hipGraphExecDestroy(b->front_exec[k]);
        if (b->back_exec[k]) (void)hipGraphExecDestroy(b->back_exec[k]);
        if (b->front[k]) (void)hipGraphDestroy(b->front[k]);
        if (b->back[k]) (void)hipGraphDestroy(b->back[k]);
        b->front_exec[k] = b->back_exec[k] = nullptr;
        b->front[k] = b->back[k] = nullptr;
    }
}

void batch_free(sdfddgi_batch *b) {
    batch_drop_graphs(b);
    for (int s = 0; s < kMaxBatchScenes; ++s) {
        dev_free(b->quad[s]);
        dev_free(b->alb[s]);
    }
    for (BatchSet &r : b->sets) {
        dev_free(r.base);
        for (int k = 0; k < 2; ++k) {
            dev_free(r.w16_i[k]); dev_free(r.w16_d[k]); dev_free(r.norm_i[k]); dev_free(r.norm_d[k]);
        }
    }
    for (int k = 0; k < 2; ++k) {
        dev_free(b->dev_scenes[k]); dev_free(b->dirs[k]); dev_free(b->payload[k]);
        dev_free(b->hitq[k]); dev_free(b->counter[k]); dev_free(b->stamps[k]);
        dev_free(b->frame_dev[k]);
    }
    dev_free(b->probe_pos); dev_free(b->probe_order);
    dev_free(b->texel_i); dev_free(b->texel_d);
    dev_free(b->irr[0]); dev_free(b->irr[1]); dev_free(b->depth[0]); dev_free(b->depth[1]);
    dev_free(b->reject); dev_free(b->blocks);
    for (int k = 0; k < kFrameSlots; ++k) {
        if (b->frame_host[k]) (void)hipHostFree(b->frame_host[k]);
        if (b->frame_ev[k]) (void)hipEventDestroy(b->frame_ev[k]);
    }
    if (b->ev_gate) (void)hipEventDestroy(b->ev_gate);
    if (b->ev_primary) (void)hipEventDestroy(b->ev_primary);
    if (b->ev_tail) (void)hipEventDestroy(b->ev_tail);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

// Arguments of a frame reading map pair `cur` with lane `lane`'s buffers.
BatchArgs batch_args(const sdfddgi_batch *b, int cur, int lane) {
    BatchArgs a{};
    a.nscenes = b->S;
    a.scenes = b->dev_scenes[lane];
    a.lights = reinterpret_cast<const float *>(b->frame_dev[lane] + 9 * sizeof(double));
    a.total_rays = (int)b->total_rays;
    a.probe_pos = b->probe_pos;
    a.probe_order = b->probe_order;
    a.dirs = b->dirs[lane];
    a.prev_irr = b->irr[cur];
    a.payload = b->payload[lane];
    a.hitq = b->hitq[lane];
    a.counter = b->counter[lane];
    a.refill = b->tuning.refill;
    return a;
}

// The launches of one frame reading map pair `cur` and writing the other, with
// lane `lane`'s buffers (a frame normally uses lane cur), in two parts: the front
// (counters, tables, primary trace; reads no map) and the back (hit shading, blend).
// `ev` (may be null) receives events before the primary trace (front), and after
// it, after the hit shading and (when ev[3] is set) after the blend (back).
hipError_t batch_enqueue_front(sdfddgi_batch *b, int lane, const BatchTuning &t, hipStream_t st,
                               hipEvent_t *ev) {
    const int cur = lane;
    hipError_t e = launch_batch_begin(b->counter[lane], b->stamps[lane], b->S, st);
    for (const BatchSet &r : b->sets) {
        if (e != hipSuccess) return e;
        TableArgs ta{};
        ta.R = r.R;
        ta.Ti = 64;
        ta.Td = 256;
        ta.Tpi = 64;
        ta.Tpd = 256;
        ta.q_dev = reinterpret_cast<const double *>(b->frame_dev[cur]);
        ta.sharp = b->sharp;
        ta.base = r.base;
        ta.texel_i = b->texel_i;
        ta.texel_d = b->texel_d;
        ta.dirs = b->dirs[cur] + 3 * (size_t)r.dir_base;
        ta.norm_i = r.norm_i[cur];
        ta.norm_d = r.norm_d[cur];
        ta.Rpad = r.R;
        ta.w16_i = r.w16_i[cur];
        ta.w16_d = r.w16_d[cur];
        e = launch_tables(ta, st);
    }
    if (e != hipSuccess) return e;
    BatchArgs a = batch_args(b, cur, lane);
    a.refill = t.refill;
    if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
    return launch_batch_primary(a, t, st);
}

hipError_t batch_enqueue_back(sdfddgi_batch *b, int cur, int lane, const BatchTuning &t,
                              hipStream_t st, hipEvent_t *ev) {
    hipError_t e = hipSuccess;
    BatchArgs a = batch_args(b, cur, lane);
    a.refill = t.refill;
    if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
    if ((e = launch_batch_hits(a, t, st)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
    BatchBlendArgs bb{};
    bb.nscenes = b->S;
    bb.scenes = b->dev_scenes[lane];
    bb.blocks = b->blocks;
    bb.payload = b->payload[lane];
    bb.prev_irr = b->irr[cur];
    bb.prev_depth = b->depth[cur];
    bb.new_irr = b->irr[1 - cur];
    bb.new_depth = b->depth[1 - cur];
    bb.reject = b->reject;
    bb.done = b->stamps[lane] + 1;
    if ((e = launch_batch_blend(bb, b->nblocks, t, st)) != hipSuccess) return e;
    return ev && ev[3] ? hipEventRecord(ev[3], st) : hipSuccess;
}

// One whole frame on the caller's stream (the autotuner's candidates).
hipError_t batch_enqueue(sdfddgi_batch *b, int cur, const BatchTuning &t, hipEvent_t *ev) {
    hipError_t e = batch_enqueue_front(b, cur, t, b->stream, ev);
    return e != hipSuccess ? e : batch_enqueue_back(b, cur, cur, t, b->stream, ev);
}

// Graphs of both parts for both lanes: fronts captured on the side stream, backs on
// the caller's.
hipError_t batch_capture(sdfddgi_batch *b) {
    batch_drop_graphs(b);
    for (int k = 0; k < 2; ++k) {
        hipError_t e = hipStreamBeginCapture(b->side, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t le = batch_enqueue_front(b, k, b->tuning, b->side, nullptr);
        e = hipStreamEndCapture(b->side, &b->front[k]);
        if (le != hipSuccess) return le;
        if (e != hipSuccess) return e;
        if ((e = hipGraphInstantiate(&b->front_exec[k], b->front[k], nullptr, nullptr, 0)) !=
            hipSuccess)
            return e;
        if ((e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return e;
        le = batch_enqueue_back(b, k, k, b->tuning, b->stream, nullptr);
        e = hipStreamEndCapture(b->stream, &b->back[k]);
        if (le != hipSuccess) return le;
        if (e != hipSuccess) return e;
        if ((e = hipGraphInstantiate(&b->back_exec[k], b->back[k], nullptr, nullptr, 0)) !=
            hipSuccess)
            return e;
    }
    return hipSuccess;
}

// Stage the frame's rotation and lights through a pinned slot into lane `lane`'s
// constants, on stream `st`.
sdfddgi_status batch_stage_frame(sdfddgi_batch *b, const sdfddgi_light *lights, uint64_t seed,
                                 int lane, hipStream_t st) {
    if (!lights) return lfail(SDFDDGI_EINVAL, "lights is NULL");
    const int k = b->slot;
    hipError_t e = hipSuccess;
    if (b->frame_used[k] && (e = hipEventSynchronize(b->frame_ev[k])) != hipSuccess)
        return lhip_fail(e, "waiting for a staging slot");
    double *q = reinterpret_cast<double *>(b->frame_host[k]);
    rotation_matrix(seed, q);
    float *lt = reinterpret_cast<float *>(b->frame_host[k] + 9 * sizeof(double));
    for (int s = 0; s < b->S; ++s) {
        const sdfddgi_light &li = lights[s];
        if (!finite_all(li.dir_to_light, 3) || !finite_all(li.radiance_rgb, 3))
            return lfail(SDFDDGI_EINVAL, "scene %d: non-finite light", s);
        const double d0 = li.dir_to_light[0], d1 = li.dir_to_light[1], d2 = li.dir_to_light[2];
        const double len = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        if (!(len > 0.0)) return lfail(SDFDDGI_EINVAL, "scene %d: zero light direction", s);
        for (int c = 0; c < 3; ++c)
            if (li.radiance_rgb[c] < 0) return lfail(SDFDDGI_EINVAL, "scene %d: negative radiance", s);
        lt[6 * s + 0] = (float)(d0 / len);
        lt[6 * s + 1] = (float)(d1 / len);
        lt[6 * s + 2] = (float)(d2 / len);
        for (int c = 0; c < 3; ++c) lt[6 * s + 3 + c] = li.radiance_rgb[c];
    }
    if ((e = hipMemcpyAsync(b->frame_dev[lane], b->frame_host[k], b->frame_bytes,
                            hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipEventRecord(b->frame_ev[k], st)) != hipSuccess)
        return lhip_fail(e, "staging the frame");
    b->frame_used[k] = true;
    b->slot = (k + 1) % kFrameSlots;
    return SDFDDGI_OK;
}

}  // namespace

extern "C" {

sdfddgi_status sdfddgi_batch_destroy(sdfddgi_batch *b) {
    if (!b) return SDFDDGI_OK;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    if (b->side) (void)hipStreamSynchronize(b->side);
    batch_free(b);
    delete b;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_batch_create(const sdfddgi_batch_scene *scenes, int32_t count,
                                    void *hip_stream, sdfddgi_batch **out) {
    g_learned_error.clear();
    if (!out) return lfail(SDFDDGI_EINVAL, "out is NULL");
    *out = nullptr;
    if (!scenes || count < 1 || count > kMaxBatchScenes)
        return lfail(SDFDDGI_EINVAL, "need 1..%d scenes", kMaxBatchScenes);
    int64_t GP = 0, rays = 0;
    for (int s = 0; s < count; ++s) {
        const sdfddgi_batch_scene &sc = scenes[s];
        sdfddgi_sdf_grid g{};
        g.num_levels = 1;
        g.level[0] = sc.level;
        sdfddgi_params p = sc.params;
        p.learned_rays = 0;
        p.flags = 0;
        if (validate(&g, &sc.probes, &p) != SDFDDGI_OK)
            return lfail(SDFDDGI_EINVAL, "scene %d: %s", s, g_create_error.c_str());
        if (p.rays_per_probe % 64 || p.irr_res != 8 || p.depth_res != 16)
            return lfail(SDFDDGI_EINVAL,
                         "scene %d: batched scenes need rays a multiple of 64, 8x8 and 16x16 maps", s);
        if (p.depth_sharpness != scenes[0].params.depth_sharpness)
            return lfail(SDFDDGI_EINVAL, "scene %d: every scene needs the same depth_sharpness", s);
        const int64_t P = (int64_t)sc.probes.n[0] * sc.probes.n[1] * sc.probes.n[2];
        GP += P;
        rays += P * p.rays_per_probe;
    }
    if (rays >= (int64_t)1 << 31) return lfail(SDFDDGI_EINVAL, "too many rays in the batch");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return lhip_fail(e, "hipGetDevice");
    (void)hipGetLastError();
    sdfddgi_batch *b = new (std::nothrow) sdfddgi_batch();
    if (!b) return lfail(SDFDDGI_ENOMEM, "host allocation failed");
    b->device = dev;
    b->S = count;
    b->GP = GP;
    b->total_rays = rays;
    b->sharp = scenes[0].params.depth_sharpness;
    b->scenes.assign(scenes, scenes + count);
    auto bail = [&](sdfddgi_status st) {
        (void)hipStreamSynchronize(b->stream);
        batch_free(b);
        delete b;
        return st;
    };
#define B_TRY(expr, what)                                                       \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess) return bail(lhip_fail(e_, what));                 \
    } while (0)
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        B_TRY(hipStreamCreate(&b->stream), "creating a stream");
        b->own_stream = true;
    }
    // ray sets: one per distinct ray count, directions concatenated
    std::vector<int> set_of(count);
    int dir_total = 0;
    for (int s = 0; s < count; ++s) {
        const int R = scenes[s].params.rays_per_probe;
        int k = 0;
        while (k < (int)b->sets.size() && b->sets[k].R != R) ++k;
        if (k == (int)b->sets.size()) {
            BatchSet r;
            r.R = R;
            r.dir_base = dir_total;
            dir_total += R;
            b->sets.push_back(r);
        }
        set_of[s] = k;
    }
    for (BatchSet &r : b->sets) {
        std::vector<double> h(3 * (size_t)r.R);
        for (int i = 0; i < r.R; ++i) fibonacci_point(i, r.R, &h[3 * i]);
        B_TRY(dev_alloc(&r.base, h.size()), "allocating ray sets");
        B_TRY(hipMemcpy(r.base, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice),
              "uploading ray sets");
        for (int k = 0; k < 2; ++k) {
            B_TRY(dev_alloc(&r.w16_i[k], (size_t)64 * r.R), "allocating tables");
            B_TRY(dev_alloc(&r.w16_d[k], (size_t)256 * r.R), "allocating tables");
            B_TRY(dev_alloc(&r.norm_i[k], 64), "allocating tables");
            B_TRY(dev_alloc(&r.norm_d[k], 256), "allocating tables");
        }
    }
    for (int k = 0; k < 2; ++k)
        B_TRY(dev_alloc(&b->dirs[k], 3 * (size_t)dir_total), "allocating directions");
    {
        std::vector<double> ti(3 * 64), td(3 * 256);
        for (int t = 0; t < 64; ++t) texel_direction(8, t % 8, t / 8, &ti[3 * t]);
        for (int t = 0; t < 256; ++t) texel_direction(16, t % 16, t / 16, &td[3 * t]);
        B_TRY(dev_alloc(&b->texel_i, ti.size()), "allocating texel directions");
        B_TRY(dev_alloc(&b->texel_d, td.size()), "allocating texel directions");
        B_TRY(hipMemcpy(b->texel_i, ti.data(), ti.size() * sizeof(double), hipMemcpyHostToDevice),
              "uploading texel directions");
        B_TRY(hipMemcpy(b->texel_d, td.data(), td.size() * sizeof(double), hipMemcpyHostToDevice),
              "uploading texel directions");
    }
    // scenes: binary16 grids, descriptors, probe positions and tracing orders
    std::vector<float> h_pos(3 * (size_t)GP);
    std::vector<int32_t> h_order((size_t)GP);
    std::vector<int2> h_blocks;
    b->host_scenes.resize(count);
    int64_t pbase = 0, rbase = 0;
    for (int s = 0; s < count; ++s) {
        const sdfddgi_batch_scene &sc = scenes[s];
        const sdfddgi_sdf_level &lv = sc.level;
        const size_t nquad = (size_t)lv.n[0] * (lv.n[1] - 1) * (lv.n[2] - 1);
        B_TRY(hipMalloc(&b->quad[s], nquad * 8), "allocating a grid");
        B_TRY(launch_pack_quads(lv.sdf, lv.n[0], lv.n[1], lv.n[2], true, b->quad[s], b->stream),
              "packing a grid");
        const size_t cnt = (size_t)lv.n[0] * lv.n[1] * lv.n[2];
        if (lv.albedo_rgb) {
            B_TRY(dev_alloc(&b->alb[s], 3 * cnt), "allocating albedo");
            B_TRY(hipMemcpyAsync(b->alb[s], lv.albedo_rgb, 3 * cnt * sizeof(float),
                                 hipMemcpyDeviceToDevice, b->stream),
                  "copying albedo");
        }
        BatchScene &d = b->host_scenes[s];
        d = BatchScene{};
        d.lv.quad = b->quad[s];
        d.lv.alb = b->alb[s];
        d.lv.org0 = (float)lv.origin[0];
        d.lv.org1 = (float)lv.origin[1];
        d.lv.org2 = (float)lv.origin[2];
        d.lv.inv = (float)(1.0 / lv.spacing);
        d.lv.cmax0 = (float)(lv.n[0] - 2);
        d.lv.cmax1 = (float)(lv.n[1] - 2);
        d.lv.cmax2 = (float)(lv.n[2] - 2);
        d.lv.half = (float)(0.5 * lv.spacing);
        d.lv.row = (uint32_t)lv.n[0];
        d.lv.slice = (uint32_t)lv.n[0] * (uint32_t)(lv.n[1] - 1);
        d.lv.arow = (uint32_t)lv.n[0];
        d.lv.aslice = (uint32_t)lv.n[0] * (uint32_t)lv.n[1];
        const float org[3] = {d.lv.org0, d.lv.org1, d.lv.org2};
        float lo[3], hi[3];
        for (int k = 0; k < 3; ++k) {   // one level: the whole grid box, [0, n-1]
            lo[k] = lower_bound_x(org[k], d.lv.inv, 0.0f);
            hi[k] = upper_bound_x(org[k], d.lv.inv, (float)(lv.n[k] - 1));
        }
        d.xlo0 = lo[0]; d.xlo1 = lo[1]; d.xlo2 = lo[2];
        d.xhi0 = hi[0]; d.xhi1 = hi[1]; d.xhi2 = hi[2];
        const sdfddgi_probe_grid &pg = sc.probes;
        d.pg.n0 = pg.n[0]; d.pg.n1 = pg.n[1]; d.pg.n2 = pg.n[2];
        d.pg.org0 = (float)pg.origin[0];
        d.pg.org1 = (float)pg.origin[1];
        d.pg.org2 = (float)pg.origin[2];
        d.pg.inv0 = (float)(1.0 / pg.spacing[0]);
        d.pg.inv1 = (float)(1.0 / pg.spacing[1]);
        d.pg.inv2 = (float)(1.0 / pg.spacing[2]);
        const int64_t P = (int64_t)pg.n[0] * pg.n[1] * pg.n[2];
        const sdfddgi_params &p = sc.params;
        d.P = (int)P;
        d.R = p.rays_per_probe;
        d.ray_base = (int)rbase;
        d.probe_base = (int)pbase;
        const BatchSet &r = b->sets[set_of[s]];
        d.dir_base = r.dir_base;
        d.max_steps = p.max_steps;
        d.eps = p.hit_eps;
        d.t_max = p.t_max;
        d.relax = p.relax;
        d.bias = p.shadow_bias;
        d.gain = p.bounce_gain;
        d.hysteresis = p.hysteresis;
        d.sky0 = p.sky_rgb[0]; d.sky1 = p.sky_rgb[1]; d.sky2 = p.sky_rgb[2];
        d.alb0 = p.albedo[0]; d.alb1 = p.albedo[1]; d.alb2 = p.albedo[2];
        d.w16_i = r.w16_i[0];  // lane 0; lane 1's descriptors are patched below
        d.w16_d = r.w16_d[0];
        d.norm_i = r.norm_i[0];
        d.norm_d = r.norm_d[0];
        // positions (binary64, rounded once) and the Morton tracing order
        const int nx = pg.n[0], ny = pg.n[1];
        std::vector<std::pair<uint64_t, int32_t>> morton((size_t)P);
        for (int64_t q = 0; q < P; ++q) {
            const int64_t idx[3] = {q % nx, (q / nx) % ny, q / ((int64_t)nx * ny)};
            for (int k = 0; k < 3; ++k)
                h_pos[3 * (pbase + q) + k] =
                    (float)(pg.origin[k] + pg.spacing[k] * (double)idx[k]);
            uint64_t m = 0;
            for (int bit = 0; bit < 21; ++bit)
                m |= ((((uint64_t)idx[0] >> bit) & 1) << (3 * bit)) |
                     ((((uint64_t)idx[1] >> bit) & 1) << (3 * bit + 1)) |
                     ((((uint64_t)idx[2] >> bit) & 1) << (3 * bit + 2));
            morton[(size_t)q] = {m, (int32_t)q};
        }
        std::sort(morton.begin(), morton.end());
        for (int64_t q = 0; q < P; ++q) h_order[(size_t)(pbase + q)] = morton[(size_t)q].second;
        for (int pb = 0; pb < (int)P; pb += 16) h_blocks.push_back(make_int2(s, pb));
        pbase += P;
        rbase += P * p.rays_per_probe;
    }
    b->nblocks = (int)h_blocks.size();
    for (int k = 0; k < 2; ++k) {
        std::vector<BatchScene> lane = b->host_scenes;
        for (int s = 0; s < count; ++s) {
            const BatchSet &r = b->sets[set_of[s]];
            lane[s].w16_i = r.w16_i[k];
            lane[s].w16_d = r.w16_d[k];
            lane[s].norm_i = r.norm_i[k];
            lane[s].norm_d = r.norm_d[k];
        }
        B_TRY(dev_alloc(&b->dev_scenes[k], count), "allocating scene descriptors");
        B_TRY(hipMemcpy(b->dev_scenes[k], lane.data(), count * sizeof(BatchScene),
                        hipMemcpyHostToDevice),
              "uploading scene descriptors");
    }
    B_TRY(dev_alloc(&b->probe_pos, h_pos.size()), "allocating probes");
    B_TRY(dev_alloc(&b->probe_order, h_order.size()), "allocating probes");
    B_TRY(dev_alloc(&b->blocks, h_blocks.size()), "allocating the blend table");
    B_TRY(hipMemcpy(b->probe_pos, h_pos.data(), h_pos.size() * sizeof(float), hipMemcpyHostToDevice),
          "uploading probes");
    B_TRY(hipMemcpy(b->probe_order, h_order.data(), h_order.size() * sizeof(int32_t),
                    hipMemcpyHostToDevice),
          "uploading probes");
    B_TRY(hipMemcpy(b->blocks, h_blocks.data(), h_blocks.size() * sizeof(int2),
                    hipMemcpyHostToDevice),
          "uploading the blend table");
    const size_t irr_f = (size_t)GP * 10 * 10 * 3, dep_f = (size_t)GP * 18 * 18 * 2;
    for (int k = 0; k < 2; ++k) {
        B_TRY(dev_alloc(&b->irr[k], irr_f), "allocating maps");
        B_TRY(dev_alloc(&b->depth[k], dep_f), "allocating maps");
        B_TRY(hipMemsetAsync(b->irr[k], 0, irr_f * sizeof(float), b->stream), "clearing maps");
        B_TRY(hipMemsetAsync(b->depth[k], 0, dep_f * sizeof(float), b->stream), "clearing maps");
    }
    B_TRY(dev_alloc(&b->reject, (size_t)GP), "allocating history flags");
    B_TRY(launch_fill_u8(b->reject, 1, GP, b->stream), "launching fill");
    b->frame_bytes = 9 * sizeof(double) + 6 * sizeof(float) * (size_t)count;
    for (int k = 0; k < 2; ++k) {
        B_TRY(dev_alloc(&b->payload[k], (size_t)rays), "allocating payload");
        B_TRY(dev_alloc(&b->hitq[k], (size_t)rays), "allocating the hit queue");
        B_TRY(dev_alloc(&b->counter[k], kBatchCounters), "allocating counters");
        B_TRY(dev_alloc(&b->stamps[k], 1 + (size_t)count), "allocating stamps");
        B_TRY(dev_alloc(&b->frame_dev[k], b->frame_bytes), "allocating frame constants");
    }
    B_TRY(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking), "creating a stream");
    B_TRY(hipEventCreateWithFlags(&b->ev_gate, hipEventDisableTiming), "creating events");
    B_TRY(hipEventCreateWithFlags(&b->ev_primary, hipEventDisableTiming), "creating events");
    B_TRY(hipEventCreateWithFlags(&b->ev_tail, hipEventDisableTiming), "creating events");
    for (int k = 0; k < kFrameSlots; ++k) {
        B_TRY(hipHostMalloc((void **)&b->frame_host[k], b->frame_bytes, hipHostMallocDefault),
              "allocating pinned staging");
        B_TRY(hipEventCreateWithFlags(&b->frame_ev[k], hipEventDisableTiming), "creating events");
    }
    b->tuning.primary_chunk = 256;
    b->tuning.primary_blocks = batch_max_blocks(dev, false);
    b->tuning.hits_chunk = 64;
    b->tuning.hits_blocks = batch_max_blocks(dev, true);
    b->tuning.refill = 40;
    b->tuning.blend_probes = 16;
    b->tuning.blend_chunk = 64;
    B_TRY(hipStreamSynchronize(b->stream), "waiting for the uploads");
    B_TRY(batch_capture(b), "capturing the frame graphs");
#undef B_TRY
    *out = b;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_batch_update_frame(sdfddgi_batch *b, const sdfddgi_light *lights,
                                          uint64_t rotation_seed) {
    g_learned_error.clear();
    if (!b) return lfail(SDFDDGI_EINVAL, "batch is NULL");
    (void)hipGetLastError();
    hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return lhip_fail(e, "hipSetDevice");
    const int k = b->cur;
    const bool serial = b->serialize_next;
    b->serialize_next = true;  // until this frame has gone in completely
    // the front of frame f uses lane f mod 2, last used by frame f-2, whose back ran
    // on the caller's stream before frame f-1's gate
    if (serial) {
        if ((e = hipEventRecord(b->ev_tail, b->stream)) != hipSuccess ||
            (e = hipStreamWaitEvent(b->side, b->ev_tail, 0)) != hipSuccess)
            return lhip_fail(e, "ordering the frame");
    } else if ((e = hipStreamWaitEvent(b->side, b->ev_gate, 0)) != hipSuccess) {
        return lhip_fail(e, "ordering the frame");
    }
    sdfddgi_status st = batch_stage_frame(b, lights, rotation_seed, k, b->side);
    if (st != SDFDDGI_OK) return st;
    if ((e = hipGraphLaunch(b->front_exec[k], b->side)) != hipSuccess)
        return lhip_fail(e, "launching the frame graph");
    if ((e = hipEventRecord(b->ev_primary, b->side)) != hipSuccess ||
        (e = hipStreamWaitEvent(b->stream, b->ev_primary, 0)) != hipSuccess ||
        (e = hipEventRecord(b->ev_gate, b->stream)) != hipSuccess)
        return lhip_fail(e, "ordering the frame");
    if ((e = hipGraphLaunch(b->back_exec[k], b->stream)) != hipSuccess)
        return lhip_fail(e, "launching the frame graph");
    b->last_lane = k;
    b->cur = 1 - k;
    b->have_frame = true;
    b->serialize_next = false;
    return SDFDDGI_OK;
}

// The blend tile's ray chunk must divide every scene's ray count (the weight rows
// are read a whole chunk at a time).
static bool blend_chunk_fits(const sdfddgi_batch *b, int chunk) {
    for (const BatchScene &s : b->host_scenes)
        if (s.R % chunk != 0) return false;
    return true;
}

static bool tuning_valid(const sdfddgi_batch *b, const sdfddgi_batch_tuning *t) {
    return t && batch_chunk_supported(t->primary_chunk, false) &&
           batch_chunk_supported(t->hits_chunk, true) && t->primary_blocks >= 1 &&
           t->primary_blocks <= batch_max_blocks(b->device, false) && t->hits_blocks >= 1 &&
           t->hits_blocks <= batch_max_blocks(b->device, true) && t->refill >= 1 &&
           t->refill <= 64 && batch_blend_tile_supported(t->blend_probes, t->blend_chunk) &&
           blend_chunk_fits(b, t->blend_chunk);
}

sdfddgi_status sdfddgi_batch_set_tuning(sdfddgi_batch *b, const sdfddgi_batch_tuning *t) {
    g_learned_error.clear();
    if (!b) return lfail(SDFDDGI_EINVAL, "batch is NULL");
    (void)hipGetLastError();
    if (!tuning_valid(b, t)) return lfail(SDFDDGI_EINVAL, "tuning out of range");
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return lhip_fail(e, "waiting for the stream");
    if ((e = hipStreamSynchronize(b->side)) != hipSuccess)
        return lhip_fail(e, "waiting for the stream");
    b->serialize_next = true;
    b->tuning = BatchTuning{t->primary_chunk, t->primary_blocks, t->hits_chunk, t->hits_blocks,
                            t->refill, t->blend_probes, t->blend_chunk};
    if ((e = batch_capture(b)) != hipSuccess) return lhip_fail(e, "capturing the frame graphs");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_batch_autotune(sdfddgi_batch *b, const sdfddgi_light *lights,
                                      uint64_t rotation_seed, int32_t frames,
                                      sdfddgi_batch_tuning *chosen, int32_t *tried) {
    g_learned_error.clear();
    if (!b) return lfail(SDFDDGI_EINVAL, "batch is NULL");
    if (frames < 1 || frames > 64) return lfail(SDFDDGI_EINVAL, "frames_per_candidate in 1..64");
    (void)hipGetLastError();
    hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return lhip_fail(e, "hipSetDevice");
    // candidates run whole frames on the caller's stream, after everything so far
    b->serialize_next = true;
    if ((e = hipEventRecord(b->ev_tail, b->side)) != hipSuccess ||
        (e = hipStreamWaitEvent(b->stream, b->ev_tail, 0)) != hipSuccess)
        return lhip_fail(e, "ordering the autotuner");
    sdfddgi_status st = batch_stage_frame(b, lights, rotation_seed, b->cur, b->stream);
    if (st != SDFDDGI_OK) return st;
    // candidate frames read the current maps and write the other pair (the state
    // does not advance); the history flags, which a blend clears, are restored
    uint8_t *saved = nullptr;
    if ((e = dev_alloc(&saved, (size_t)b->GP)) != hipSuccess) return lhip_fail(e, "allocating");
    e = hipMemcpyAsync(saved, b->reject, (size_t)b->GP, hipMemcpyDeviceToDevice, b->stream);
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k < 4 && e == hipSuccess; ++k) e = hipEventCreate(&ev[k]);
    const int pmax = batch_max_blocks(b->device, false), hmax = batch_max_blocks(b->device, true);
    int count = 0;
    // time one configuration: mean primary, hit shading and blend kernel times over
    // `frames`
    float blend = 0.0f;
    auto measure = [&](const BatchTuning &t, float &prim, float &hits) -> hipError_t {
        prim = hits = blend = 0.0f;
        for (int f = 0; f < frames; ++f) {
            hipError_t x = batch_enqueue(b, b->cur, t, ev);
            if (x != hipSuccess) return x;
            if ((x = hipEventSynchronize(ev[3])) != hipSuccess) return x;
            float a = 0.0f, c = 0.0f, d = 0.0f;
            if ((x = hipEventElapsedTime(&a, ev[0], ev[1])) != hipSuccess) return x;
            if ((x = hipEventElapsedTime(&c, ev[1], ev[2])) != hipSuccess) return x;
            if ((x = hipEventElapsedTime(&d, ev[2], ev[3])) != hipSuccess) return x;
            prim += a / frames;
            hits += c / frames;
            blend += d / frames;
        }
        ++count;
        return hipSuccess;
    };
    BatchTuning best = b->tuning;
    float best_p = 1e30f, best_h = 1e30f, p = 0, h = 0;
    // the primary trace: chunk x refill x grid; then the hit shading: chunk x grid
    const int pchunks[4] = {64, 128, 256, 512}, refills[4] = {24, 32, 40, 48};
    const int pgrids[2] = {pmax, std::max(1, pmax / 2)};
    for (int ci = 0; ci < 4 && e == hipSuccess; ++ci)
        for (int ri = 0; ri < 4 && e == hipSuccess; ++ri)
            for (int gi = 0; gi < 2 && e == hipSuccess; ++gi) {
                BatchTuning t = best;
                t.primary_chunk = pchunks[ci];
                t.refill = refills[ri];
                t.primary_blocks = pgrids[gi];
                if ((e = measure(t, p, h)) == hipSuccess && p < best_p) {
                    best_p = p;
                    best.primary_chunk = t.primary_chunk;
                    best.refill = t.refill;
                    best.primary_blocks = t.primary_blocks;
                }
            }
    const int hchunks[4] = {16, 32, 64, 128};
    const int hgrids[2] = {hmax, std::max(1, hmax / 2)};
    for (int ci = 0; ci < 4 && e == hipSuccess; ++ci)
        for (int gi = 0; gi < 2 && e == hipSuccess; ++gi) {
            BatchTuning t = best;
            t.hits_chunk = hchunks[ci];
            t.hits_blocks = hgrids[gi];
            if ((e = measure(t, p, h)) == hipSuccess && h < best_h) {
                best_h = h;
                best.hits_chunk = t.hits_chunk;
                best.hits_blocks = t.hits_blocks;
            }
        }
    // the blend tile: probes per workgroup x rays per LDS stage (those that divide
    // every scene's ray count)
    const int bprobes[2] = {16, 8}, bchunks[3] = {32, 64, 128};
    float best_b = 1e30f;
    for (int pi = 0; pi < 2 && e == hipSuccess; ++pi)
        for (int ci = 0; ci < 3 && e == hipSuccess; ++ci) {
            if (!blend_chunk_fits(b, bchunks[ci])) continue;
            BatchTuning t = best;
            t.blend_probes = bprobes[pi];
            t.blend_chunk = bchunks[ci];
            if ((e = measure(t, p, h)) == hipSuccess && blend < best_b) {
                best_b = blend;
                best.blend_probes = t.blend_probes;
                best.blend_chunk = t.blend_chunk;
            }
        }
    // then the grids of both parts as consecutive frames run them, the front of one
    // beside the back of the previous (the times above are each kernel alone): whole
    // overlapped frames, lanes alternating, all reading the current maps
    auto measure_overlapped = [&](const BatchTuning &t, float &ms) -> hipError_t {
        const int n = 2 * frames + 2;
        hipError_t x = hipEventRecord(ev[0], b->stream);
        if (x == hipSuccess) x = hipStreamWaitEvent(b->side, ev[0], 0);
        for (int f = 0; f < n && x == hipSuccess; ++f) {
            const int lane = f & 1;
            if (f > 0) x = hipStreamWaitEvent(b->side, b->ev_gate, 0);
            if (x == hipSuccess) x = batch_enqueue_front(b, lane, t, b->side, nullptr);
            if (x == hipSuccess) x = hipEventRecord(b->ev_primary, b->side);
            if (x == hipSuccess) x = hipStreamWaitEvent(b->stream, b->ev_primary, 0);
            if (x == hipSuccess) x = hipEventRecord(b->ev_gate, b->stream);
            if (x == hipSuccess) x = batch_enqueue_back(b, b->cur, lane, t, b->stream, nullptr);
        }
        if (x == hipSuccess) x = hipEventRecord(ev[2], b->stream);
        if (x == hipSuccess) x = hipEventSynchronize(ev[2]);
        if (x == hipSuccess) x = hipEventElapsedTime(&ms, ev[0], ev[2]);
        ms /= n;
        ++count;
        return x;
    };
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->frame_dev[1 - b->cur], b->frame_dev[b->cur], b->frame_bytes,
                           hipMemcpyDeviceToDevice, b->stream);
    const int opgrids[3] = {pmax, std::max(1, pmax * 3 / 4), std::max(1, pmax / 2)};
    const int ohgrids[3] = {hmax, std::max(1, hmax / 2), std::max(1, hmax / 4)};
    const BatchTuning alone = best;
    float best_o = 1e30f, o = 0;
    for (int pi = 0; pi < 3 && e == hipSuccess; ++pi)
        for (int hi = 0; hi < 3 && e == hipSuccess; ++hi) {
            BatchTuning t = alone;
            t.primary_blocks = opgrids[pi];
            t.hits_blocks = ohgrids[hi];
            if ((e = measure_overlapped(t, o)) == hipSuccess && o < best_o) {
                best_o = o;
                best.primary_blocks = t.primary_blocks;
                best.hits_blocks = t.hits_blocks;
            }
        }
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->reject, saved, (size_t)b->GP, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    for (int k = 0; k < 4; ++k)
        if (ev[k]) (void)hipEventDestroy(ev[k]);
    dev_free(saved);
    if (e != hipSuccess) return lhip_fail(e, "autotuning");
    b->tuning = best;
    if ((e = batch_capture(b)) != hipSuccess) return lhip_fail(e, "capturing the frame graphs");
    if (chosen)
        *chosen = sdfddgi_batch_tuning{best.primary_chunk, best.primary_blocks, best.hits_chunk,
                                       best.hits_blocks, best.refill, best.blend_probes,
                                       best.blend_chunk};
    if (tried) *tried = count;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_batch_get_maps(sdfddgi_batch *b, int32_t scene, float *irr, float *depth) {
    g_learned_error.clear();
    if (!b) return lfail(SDFDDGI_EINVAL, "batch is NULL");
    if (scene < 0 || scene >= b->S) return lfail(SDFDDGI_EINVAL, "scene %d out of range", scene);
    (void)hipGetLastError();
    b->serialize_next = true;
    const BatchScene &d = b->host_scenes[scene];
    const size_t ti = 10 * 10 * 3, td = 18 * 18 * 2;
    hipError_t e = hipSuccess;
    if (irr)
        e = hipMemcpyAsync(irr, b->irr[b->cur] + (size_t)d.probe_base * ti,
                           (size_t)d.P * ti * sizeof(float), hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess && depth)
        e = hipMemcpyAsync(depth, b->depth[b->cur] + (size_t)d.probe_base * td,
                           (size_t)d.P * td * sizeof(float), hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return lhip_fail(e, "copying maps");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_batch_scene_latency(sdfddgi_batch *b, float *ms, float *frame_ms) {
    g_learned_error.clear();
    if (!b || !ms) return lfail(SDFDDGI_EINVAL, "null argument");
    if (!b->have_frame) return lfail(SDFDDGI_ESTATE, "no frame yet");
    (void)hipGetLastError();
    b->serialize_next = true;
    std::vector<unsigned long long> st(1 + (size_t)b->S);
    int rate_khz = 0;
    hipError_t e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, b->device);
    if (e == hipSuccess)
        e = hipMemcpyAsync(st.data(), b->stamps[b->last_lane],
                           st.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return lhip_fail(e, "reading the stamps");
    if (rate_khz <= 0) return lfail(SDFDDGI_EDEVICE, "no device clock rate");
    float worst = 0.0f;
    for (int s = 0; s < b->S; ++s) {
        ms[s] = (float)((double)(st[1 + s] - st[0]) / (double)rate_khz);
        worst = std::max(worst, ms[s]);
    }
    if (frame_ms) *frame_ms = worst;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_batch_sizes(const sdfddgi_batch *b, int64_t *probes, int64_t *rays) {
    if (!b) return SDFDDGI_EINVAL;
    if (probes) *probes = b->GP;
    if (rays) *rays = b->total_rays;
    return SDFDDGI_OK;
}

}  // extern "C"

// ------------------------------------------------------------ analytic SDF --

struct sdfddgi_analytic {
    int device = 0;
    hipStream_t stream = nullptr;
    int nprims = 0, nclusters = 0;
    int *kind = nullptr, *first = nullptr;
    float *center = nullptr, *half = nullptr, *lo = nullptr, *hi = nullptr;
    unsigned long long *evals = nullptr;
};

extern "C" {

sdfddgi_status sdfddgi_analytic_destroy(sdfddgi_analytic *an) {
    if (!an) return SDFDDGI_OK;
    (void)hipSetDevice(an->device);
    (void)hipStreamSynchronize(an->stream);
    dev_free(an->kind); dev_free(an->first); dev_free(an->center); dev_free(an->half);
    dev_free(an->lo); dev_free(an->hi); dev_free(an->evals);
    delete an;
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_analytic_create(int32_t nprims, const int32_t *kind, const double *center,
                                       const double *half, int32_t cluster_size,
                                       void *hip_stream, sdfddgi_analytic **out) {
    g_learned_error.clear();
    if (!out) return lfail(SDFDDGI_EINVAL, "out is NULL");
    *out = nullptr;
    HostClusters hc;
    const std::string why = build_clusters(nprims, kind, center, half, nullptr, cluster_size, hc);
    if (!why.empty()) return lfail(SDFDDGI_EINVAL, "%s", why.c_str());
    (void)hipGetLastError();
    const int nclusters = hc.nclusters;
    const std::vector<int> &h_kind = hc.kind, &h_first = hc.first;
    const std::vector<float> &h_cen = hc.cen, &h_half = hc.half, &h_lo = hc.lo, &h_hi = hc.hi;
    sdfddgi_analytic *an = new (std::nothrow) sdfddgi_analytic();
    if (!an) return lfail(SDFDDGI_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&an->device);
    an->stream = (hipStream_t)hip_stream;
    an->nprims = nprims;
    an->nclusters = nclusters;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(dev_alloc(&an->kind, nprims));
    chk(dev_alloc(&an->first, nclusters + 1));
    chk(dev_alloc(&an->center, 3 * (size_t)nprims));
    chk(dev_alloc(&an->half, 3 * (size_t)nprims));
    chk(dev_alloc(&an->lo, 3 * (size_t)nclusters));
    chk(dev_alloc(&an->hi, 3 * (size_t)nclusters));
    chk(dev_alloc(&an->evals, 1));
    if (e == hipSuccess) {
        chk(hipMemcpy(an->kind, h_kind.data(), nprims * sizeof(int), hipMemcpyHostToDevice));
        chk(hipMemcpy(an->first, h_first.data(), (nclusters + 1) * sizeof(int), hipMemcpyHostToDevice));
        chk(hipMemcpy(an->center, h_cen.data(), h_cen.size() * sizeof(float), hipMemcpyHostToDevice));
        chk(hipMemcpy(an->half, h_half.data(), h_half.size() * sizeof(float), hipMemcpyHostToDevice));
        chk(hipMemcpy(an->lo, h_lo.data(), h_lo.size() * sizeof(float), hipMemcpyHostToDevice));
        chk(hipMemcpy(an->hi, h_hi.data(), h_hi.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    if (e != hipSuccess) {
        sdfddgi_analytic_destroy(an);
        return lhip_fail(e, "creating the analytic scene");
    }
    *out = an;
    return SDFDDGI_OK;
}

static AnalyticArgs analytic_args(const sdfddgi_analytic *an) {
    AnalyticArgs a{};
    a.nprims = an->nprims;
    a.nclusters = an->nclusters;
    a.kind = an->kind;
    a.center = an->center;
    a.half = an->half;
    a.lo = an->lo;
    a.hi = an->hi;
    a.first = an->first;
    return a;
}

static hipError_t read_evals(sdfddgi_analytic *an, int64_t *evals) {
    unsigned long long v = 0;
    hipError_t e = hipMemcpyAsync(&v, an->evals, sizeof v, hipMemcpyDeviceToHost, an->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(an->stream);
    *evals = (int64_t)v;
    return e;
}

sdfddgi_status sdfddgi_analytic_query(sdfddgi_analytic *an, const float *points, int32_t n,
                                      int32_t mode, float *out, int64_t *evals) {
    g_learned_error.clear();
    if (!an || n < 0 || mode < 0 || mode > 1 || (n > 0 && (!points || !out)))
        return lfail(SDFDDGI_EINVAL, "bad argument (query modes are 0 and 1)");
    (void)hipGetLastError();
    hipError_t e = hipSetDevice(an->device);
    // two binary32 zeros clear the 64-bit evaluation counter
    if (e == hipSuccess && evals) e = launch_zero_f32(reinterpret_cast<float *>(an->evals), 2, an->stream);
    if (e == hipSuccess)
        e = launch_cluster_query(analytic_args(an), points, n, mode, out, evals ? an->evals : nullptr,
                                 an->stream);
    if (e == hipSuccess && evals) e = read_evals(an, evals);
    if (e != hipSuccess) return lhip_fail(e, "analytic query");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_analytic_trace(sdfddgi_analytic *an, const float *origins,
                                      const float *dirs, int32_t n, float t_max, float eps,
                                      float relax, int32_t max_steps, int32_t mode, float *t,
                                      int32_t *steps, int32_t *kind, int64_t *evals) {
    g_learned_error.clear();
    if (!an || n < 0 || mode < 0 || mode > 2 || (n > 0 && (!origins || !dirs || !t || !steps || !kind)))
        return lfail(SDFDDGI_EINVAL, "bad argument");
    const float v[3] = {t_max, eps, relax};
    if (!finite_all(v, 3) || !(t_max > 0) || !(eps > 0) || !(relax > 0 && relax <= 2) ||
        max_steps < 1 || max_steps > 4096)
        return lfail(SDFDDGI_EINVAL, "trace parameters out of range");
    (void)hipGetLastError();
    hipError_t e = hipSetDevice(an->device);
    if (e == hipSuccess && evals) e = launch_zero_f32(reinterpret_cast<float *>(an->evals), 2, an->stream);
    AnalyticTrace r{};
    r.n = n;
    r.o = origins;
    r.w = dirs;
    r.t_max = t_max;
    r.eps = eps;
    r.relax = relax;
    r.max_steps = max_steps;
    r.mode = mode;
    r.t_out = t;
    r.steps_out = steps;
    r.kind_out = kind;
    r.evals = evals ? an->evals : nullptr;
    if (e == hipSuccess) e = launch_cluster_trace(analytic_args(an), r, an->stream);
    if (e == hipSuccess && evals) e = read_evals(an, evals);
    if (e != hipSuccess) return lhip_fail(e, "analytic trace");
    return SDFDDGI_OK;
}

sdfddgi_status sdfddgi_analytic_clusters(const sdfddgi_analytic *an, int32_t *count) {
    if (!an || !count) return SDFDDGI_EINVAL;
    *count = an->nclusters;
    return SDFDDGI_OK;
}

}  // extern "C"
