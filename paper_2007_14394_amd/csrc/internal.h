// Internal interface between the host runtime (runtime.hip) and the gfx950
// kernels (kernels.hip). Plain structs passed by value as kernel arguments.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdfddgi {

constexpr int kMaxLevels = 4;
constexpr int kMaxRays = 1024;
constexpr int kMaxRes = 32;
constexpr int kXcds = 8;  // accelerator complex dies of the chip, one L2 each
constexpr int kPartStride = 32;  // ints between per-XCD work counters: one 128-B line each

// One cascade level as the kernels see it. org/inv/half are the binary32
// roundings of origin, 1/spacing and spacing/2 (computed once in binary64).
struct DevLevel {
    const void *quad;   // [n2-1][n1-1][n0] corner quads (see trilinear in kernels.hip):
                        // float4, or 4 x binary16 in the precision form
    const float *alb;   // [n2][n1][n0][3] or nullptr
    int n0, n1, n2;
    float org0, org1, org2;
    float inv;
    float half;
    // Exact binary32 bounds on x of the level's box test: for every float x,
    // lo <= (x - org) * inv  <=>  x >= xlo, and (x - org) * inv <= hi  <=>  x <= xhi,
    // with [lo, hi] = [1, n-2] (inner levels) or [0, n-1] (coarsest level).
    float xlo0, xlo1, xlo2, xhi0, xhi1, xhi2;
};

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

struct ProbeGridDev {
    int n0, n1, n2;
    float org0, org1, org2;     // (float)origin
    float inv0, inv1, inv2;     // (float)(1/spacing)
};

constexpr int kMaxAnalyticPrims = 1024;
constexpr int kMaxClusters = 256;

struct AnalyticArgs {
    int nprims, nclusters;
    const int *kind;                 // [nprims], primitives ordered by cluster
    const int *orig;                 // [nprims] each one's index in the caller's order
                                     //     (null: the cluster order is the caller's)
    const float *center, *half;      // [nprims][3] binary32
    const float *lo, *hi;            // [nclusters][3] widened bounding boxes
    const int *first;                // [nclusters + 1] first primitive of each cluster
};

struct TraceArgs {
    DevLevel lv[kMaxLevels];
    int nl;
    int half_sdf;               // 1: the quads hold binary16 values
    int P, R;
    int max_steps;
    int irr_res;
    ProbeGridDev pg;
    float eps, t_max, relax, bias, gain;
    float l0, l1, l2;           // unit direction toward the light (binary32)
    float rad0, rad1, rad2;
    float sky0, sky1, sky2;
    float alb0, alb1, alb2;
    const float *probe_pos;     // [P][3]
    const int *probe_order;     // [P] probes in Morton order of (x, y, z): the tracing order,
                                //     or the list of probes to trace
    const int *probe_count;     // null: trace all P probes; else the device-side length of
                                //     probe_order (the learned form's fallback list)
    const float *dirs;          // [R][3]
    const float *prev_irr;      // previous irradiance atlas
    float4 *payload;            // [P*R]
    int *records;               // [P*R*8] or nullptr
    int4 *hitq;                 // [P*R] queue of primary hits: (ray, bits of t, outcome|level<<4|steps<<8,
                                //     nearest primitive slot when analytic, else 0)
    int *counter;               // [3] (unused), queue entries claimed by hits_kernel, queue
                                //     length (all zeroed by tables_kernel)
    int *parts;                 // [kXcds * kPartStride] primary chunks claimed per XCD, one
                                //     counter per 128-B line (zeroed likewise)
    const int2 *probe_first;    // [P] each probe's first sample, which every one of its rays
                                //     takes at the probe position: (bits of the distance,
                                //     level or -1 outside every level; analytic: the nearest
                                //     primitive's slot); null: sample it
    int analytic;               // 1: distances from the primitives in `an`, not the grid
    AnalyticArgs an;
    const float *prim_alb;      // [nprims][3] albedo of each primitive, cluster order
    float4 *geo;                // null: hits_kernel shades each hit. Else hit shading is split:
                                //     hits_kernel stores, per hit-queue entry i, what does not
                                //     depend on the previous atlas -- geo[2i] = (normal, sun
                                //     term n.l or 0 in shadow), geo[2i+1] = (albedo, 0) -- and
                                //     shade_kernel adds the multi-bounce lookup later
};

struct TraceGrid {
    int primary_blocks = 0, hits_blocks = 0;
    int primary_blocks_overlapped = 0;  // primary trace beside the last frame's hit shading
    int hits_blocks_overlapped = 0;     // hit shading beside the next frame's primary trace
};

struct TableArgs {
    int R, Ti, Td;
    int Tpi, Tpd;               // row strides of the weight tables: T rounded up to 16
    double q[9];                // frame rotation, row-major
    const double *q_dev;        // null: q above; else the rotation read from device memory
                                //     (a captured graph replays with per-frame values)
    double sharp;               // depth cosine power
    const double *base;         // [R][3] unrotated spherical-Fibonacci set
    const double *texel_i;      // [Ti][3] irradiance texel directions
    const double *texel_d;      // [Td][3] depth texel directions
    float *dirs;                // [R][3]
    float *wt_i;                // [R][Tpi] w_ti, transposed; rows t >= Ti stay zero
    float *wt_d;                // [R][Tpd] w_ti^s, transposed; rows t >= Td stay zero
    float *norm_i;              // [Ti]  pi / sum_i w_ti   (-1: all weights vanish)
    float *norm_d;              // [Td]  1 / sum_i w_ti^s  (-1: all weights vanish)
    int *counter;               // [ncounter] counters reset here (may be null): the trace
    int ncounter;               //     kernels' and, in the learned form, the fallback pass's
    int Rpad;                   // row length of the 16-bit tables: R rounded up to 64
    _Float16 *w16_i;            // precision form: [Tpi][Rpad] FP16 w_ti (else null)
    __bf16 *w16_d;              // precision form: [Tpd][Rpad] BF16 w_ti^s (else null)
    int row0;                   // row of block 0 (set by the launch functions)
};

struct BlendArgs {
    int P, R, irr_res, depth_res;
    float hysteresis;
    const float4 *payload;
    const float *wt_i, *wt_d, *norm_i, *norm_d;
    int Rpad;
    const _Float16 *w16_i;      // precision form (see TableArgs); null: FP32 blend
    const __bf16 *w16_d;
    const float *prev_irr, *prev_depth;
    float *new_irr, *new_depth;
    uint8_t *reject;            // per-probe history flags (read, then cleared); null: none
    const int *probe_list;      // null: probes 0..P-1; else blend only these probes
    const int *probe_count;     //     (device-side count; P bounds it)
};

struct SampleArgs {
    int64_t n;
    int irr_res;
    ProbeGridDev pg;
    const float *atlas;
    const float *points, *normals;
    float *out;
};

// Launchers (kernels.hip). Each enqueues on `stream` and returns the launch status.
hipError_t launch_tables(const TableArgs &a, hipStream_t stream);
// The directions block alone (it also resets the counters), and the weight rows
// alone; together they do what launch_tables does.
hipError_t launch_tables_dirs(TableArgs a, hipStream_t stream);
hipError_t launch_tables_weights(TableArgs a, hipStream_t stream);
TraceGrid trace_grid(int device, int64_t rays, bool half, bool analytic = false);
hipError_t launch_primary(const TraceArgs &a, const TraceGrid &grid, hipStream_t stream);
hipError_t launch_hits(const TraceArgs &a, const TraceGrid &grid, hipStream_t stream);
// The atlas-dependent half of split hit shading (TraceArgs::geo): one thread per queue entry.
hipError_t launch_shade(const TraceArgs &a, hipStream_t stream);
hipError_t launch_blend(const BlendArgs &a, hipStream_t stream);
hipError_t launch_sample(const SampleArgs &a, hipStream_t stream);
hipError_t launch_pack_quads(const float *grid, int n0, int n1, int n2, bool half, void *quad,
                             hipStream_t stream);
hipError_t launch_fill_u8(uint8_t *dst, uint8_t value, int64_t n, hipStream_t stream);

}  // namespace sdfddgi

// ------------------------------------------------------------ learned form --
// A per-texel network (16 -> 64 -> 64 -> 64 -> 4, bfloat16 weights, FP32
// accumulation on MFMA) maps a low-ray Eq. 3 update to the many-ray one. Parameter
// vector (binary32 masters, row-major): W1[64][16] | W2[64][64] | b2[64] |
// W3[64][64] | b3[64] | W4[4][64] | b4[4].
namespace sdfddgi {

constexpr int kFeatures = 16, kHidden = 64, kOutputs = 4;
constexpr int kOffW1 = 0;
constexpr int kOffW2 = kOffW1 + kHidden * kFeatures;
constexpr int kOffB2 = kOffW2 + kHidden * kHidden;
constexpr int kOffW3 = kOffB2 + kHidden;
constexpr int kOffB3 = kOffW3 + kHidden * kHidden;
constexpr int kOffW4 = kOffB3 + kHidden;
constexpr int kOffB4 = kOffW4 + kOutputs * kHidden;
constexpr int kMlpParams = kOffB4 + kOutputs;
// Per-lane MFMA operand packs (16 bytes = 8 bfloat16 per lane and entry):
// forward A operands of the four layers, backward A operands (transposed W4, W3, W2)
constexpr int kFwdEntries = 22, kBwdEntries = 20;
constexpr int kBiasFloats = 2 * kHidden + 16;   // b2 | b3 | b4 padded to 16
constexpr int kMaxLearnedRes = 16;               // irradiance maps up to 16 x 16

struct MlpPack {
    const uint4 *fwd;     // [kFwdEntries][64]
    const uint4 *bwd;     // [kBwdEntries][64]
    const float *bias;    // [kBiasFloats]
};

// Inputs of the per-texel feature vector (see feature_group in learned.hip).
struct FeatureArgs {
    int irr_res, depth_res;
    float inv_s, inv_d;           // 1/S and 1/D in binary32
    const float *u_irr;           // low-ray Eq. 3 irradiance atlas (no hysteresis)
    const float *prev_irr, *prev_depth;
    const float *probe_sdf;       // [P] signed distance at each probe
    const float *texel_dir;       // [Ti][3] texel centre directions (binary32)
};

struct DenoiseArgs {
    FeatureArgs f;
    int P;
    float hysteresis, s, tau;
    const float *u_depth;         // low-ray depth moments atlas (no hysteresis)
    float *new_irr, *new_depth;
    MlpPack mlp;
    uint8_t *fb_flag;             // [P] in: the probe takes the plain update this frame
                                  //     (written nothing here); out: it will in the learned
                                  //     frame after next (mean predicted error above tau)
    float *mean_error;            // [P] mean predicted relative error (may be null)
};

struct ExampleArgs {
    FeatureArgs f;
    int P;
    const float *target_irr;      // target irradiance atlas (e.g. a many-ray run's maps)
    float rel_floor;              // added to |U*|_1 / S in the relative-error scale
    float *features;              // [P*Ti][16]
    float *targets;               // [P*Ti][4]: (U* - E_prev) / S, |U*|_1 / S + floor
};

struct InferArgs {
    int64_t n;
    const float *features;        // [n][16]
    float *out;                   // [n][4]
    MlpPack mlp;
};

struct TrainArgs {
    const float *features, *targets;
    int64_t count;                // samples available
    int batch;                    // samples of this step
    uint64_t seed;
    int sequential;               // 1: samples 0..batch-1 in order; 0: SplitMix64 draws
    MlpPack mlp;
    float inv_n, head_weight, min_error;
    float *grad;                  // [kMlpParams], accumulated (zero before the launch)
    float *loss;                  // [1], accumulated
};

struct AdamArgs {
    float *theta, *m, *v, *grad;  // grad is consumed and zeroed
    int n;
    float lr, beta1, beta2, eps, c1, c2;   // c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t)
};

hipError_t launch_probe_sdf(const TraceArgs &a, float *out, hipStream_t stream);
hipError_t launch_probe_first(const TraceArgs &a, int2 *out, hipStream_t stream);

// Alg. 1 (UpdateProbePos) for every probe: new positions from the grid positions,
// history rejected where a probe moved more than threshold2 since the last call.
struct RelocateArgs {
    const float *grid_pos;      // [P][3] the grid positions (binary32)
    float *pos;                 // [P][3] current positions: read as the last, then written
    uint8_t *reject;            // [P] set to 1 where the probe moved too far
    float t1, t2;               // threshold1 (distance), threshold2 (displacement)
    int iterations;
    float off0, off1, off2;     // (float)(max_offset * spacing) per axis
};
hipError_t launch_relocate(const TraceArgs &a, const RelocateArgs &r, hipStream_t stream);
hipError_t launch_pack_mlp(const float *theta, uint4 *fwd, uint4 *bwd, float *bias,
                           hipStream_t stream);
hipError_t launch_denoise(const DenoiseArgs &a, hipStream_t stream);
// Measurement: `threads` threads each gathering `reads` (a multiple of 8) random
// 32-byte records of a buffer of `records` (a power of two) records.
hipError_t launch_gather(const void *buf, int64_t records, int64_t threads, int reads,
                         uint32_t seed, float *sink, hipStream_t stream);
// The fallback list of a learned frame: every probe whose flag asks for the plain
// update or, when reject is given, whose history is rejected; the flag is set for
// both (the denoiser reads it, not the reject flags the fallback blend clears).
// count zeroed before.
hipError_t launch_select_fallback(const uint8_t *reject, uint8_t *fb_flag, int P, int *list,
                                  int *count, hipStream_t stream);
hipError_t launch_examples(const ExampleArgs &a, hipStream_t stream);
hipError_t launch_infer(const InferArgs &a, hipStream_t stream);
hipError_t launch_train(const TrainArgs &a, hipStream_t stream);
hipError_t launch_adam(const AdamArgs &a, hipStream_t stream);
hipError_t launch_zero_f32(float *dst, int64_t n, hipStream_t stream);

// Scene baking (scene.hip). Primitive arrays are device copies; kind 0 sphere
// (radius in half[0]), 1 axis-aligned box.
struct BakeArgs {
    int nprims;
    const int *kind;
    const double *center, *half, *albedo;   // [nprims][3]
    int n0, n1, n2;
    double org0, org1, org2, spacing;
    float empty_value;
    float *sdf;                             // [n2][n1][n0]
    float *alb;                             // [n2][n1][n0][3] or null
};

hipError_t launch_bake(const BakeArgs &a, hipStream_t stream);

// ------------------------------------------------------------ batched form --
// Many scenes of uneven size (one binary16 grid level each, 8x8 irradiance and
// 16x16 depth maps, their own probe grids and ray counts) updated by one set of
// launches per frame (batch.hip). Scenes are concatenated: scene s owns probes
// probe_base .. probe_base+P-1 of the batch's probe arrays and atlases, and rays
// ray_base .. ray_base+P*R-1 of its payload.
constexpr int kMaxBatchScenes = 64;
// batch counters: [0..2] primary rays claimed, hits claimed, hit-queue length; from
// [kPartStride] the primary trace's per-XCD counters
constexpr int kBatchCounters = kPartStride + kXcds * kPartStride;
constexpr int kBatchBlockRays = 65536;  // rays per block of the XCD interleave

struct BatchScene {
    LevelLds lv;                          // its grid level (binary16 quads)
    float xlo0, xlo1, xlo2, xhi0, xhi1, xhi2;   // exact x bounds of the grid box
    ProbeGridDev pg;
    int P, R, ray_base, probe_base, dir_base, max_steps;
    float eps, t_max, relax, bias, gain, hysteresis;
    float sky0, sky1, sky2, alb0, alb1, alb2;
    const _Float16 *w16_i;                // its ray set's tables
    const __bf16 *w16_d;
    const float *norm_i, *norm_d;
};

struct BatchArgs {
    int nscenes;
    const BatchScene *scenes;             // [nscenes]
    const float *lights;                  // [nscenes][6]: unit direction to the light, radiance
    int total_rays;
    const float *probe_pos;               // [GP][3]
    const int *probe_order;               // [GP]: each scene's probes in Morton order (local ids)
    const float *dirs;                    // ray sets' directions, concatenated [.][3]
    const float *prev_irr;                // [GP] irradiance tiles of the previous frame
    float4 *payload;                      // [total_rays]
    int4 *hitq;                           // [total_rays]: (ray, bits of t, info, scene)
    int *counter;                         // [3]
    int refill;                           // refill idle lanes below this many stepping lanes
};

struct BatchBlendArgs {
    int nscenes;
    const BatchScene *scenes;
    const int2 *blocks;                   // [nblocks16]: (scene, first probe) of each 16 probes
    const float4 *payload;
    const float *prev_irr, *prev_depth;
    float *new_irr, *new_depth;
    uint8_t *reject;                      // [GP]
    unsigned long long *done;             // [nscenes] device clock when the scene's last
                                          //     blend workgroup finished (atomic max)
};

struct BatchTuning {
    int primary_chunk, primary_blocks, hits_chunk, hits_blocks, refill;
    int blend_probes, blend_chunk;        // blend tile: probes per workgroup, rays per LDS stage
};

hipError_t launch_batch_begin(int *counter, unsigned long long *stamps, int nscenes,
                              hipStream_t stream);
hipError_t launch_batch_primary(const BatchArgs &a, const BatchTuning &t, hipStream_t stream);
hipError_t launch_batch_hits(const BatchArgs &a, const BatchTuning &t, hipStream_t stream);
// nblocks16 entries of the 16-probe block table, each split into 16 / blend_probes
// workgroups.
hipError_t launch_batch_blend(const BatchBlendArgs &a, int nblocks16, const BatchTuning &t,
                              hipStream_t stream);
bool batch_blend_tile_supported(int probes, int chunk);
int batch_max_blocks(int device, bool hits);

// -------------------------------------------------- analytic SDF (cluster.hip) --

struct AnalyticTrace {
    int n;
    const float *o, *w;              // [n][3] ray origins and unit directions
    float t_max, eps, relax;
    int max_steps, mode;             // mode 0 every primitive, 1 clusters, 2 clusters + bound
    float *t_out;
    int *steps_out, *kind_out;
    unsigned long long *evals;       // primitive distance evaluations (may be null)
};

hipError_t launch_cluster_query(const AnalyticArgs &a, const float *pts, int n, int mode,
                                float *out, unsigned long long *evals, hipStream_t stream);
hipError_t launch_cluster_trace(const AnalyticArgs &a, const AnalyticTrace &r,
                                hipStream_t stream);
bool batch_chunk_supported(int chunk, bool hits);

}  // namespace sdfddgi
