// gfx950 kernels of the learned form of the probe update (an extension beyond
// the paper): a small per-texel network maps the Eq. 3 update of a low ray count,
// with the probe's history, to the update of a many-ray set, and predicts its own
// relative error; probes whose mean predicted error is too high take the plain
// update instead.
//
//   pack_mlp_kernel   binary32 parameters -> per-lane bfloat16 MFMA operand packs
//   denoise_kernel    per probe: features, network, decision, hysteresis and
//                     border writes of accepted probes, fallback list of the rest
//   examples_kernel   training pairs: features and targets (a converged atlas) per texel
//   infer_kernel      the network on a feature array
//   train_kernel      loss gradient over a minibatch (forward, backward, weight
//                     gradients; all contractions on bfloat16 MFMA)
//   adam_kernel       Adam update of the binary32 masters
//
// MFMA layout (v_mfma_f32_16x16x32_bf16, wave64): lane l = n + 16 g holds the A
// operand A[n][8g .. 8g+7], the B operand B[8g .. 8g+7][n], and the result
// D[4g + r][n] in register r. A layer's outputs (rows = units, columns = 16
// texels) therefore sit as units 16 mt + 4 g + r of m-tile mt in lane (n, g). The
// next layer contracts over those units in an order of its own choosing: k-step
// ks, slot s of lane group g stands for unit 16 (2 ks + s/4) + 4 g + s%4, which
// is exactly what the lane holds -- activations never leave registers. The
// weight packs are written in that unit order.
#include "internal.h"
#include "octahedral.h"

#include <algorithm>

#pragma clang fp contract(off)

namespace sdfddgi {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// Unit of layer input slot s of k-step ks in lane group g (see above).
__host__ __device__ __forceinline__ int unit_of(int ks, int g, int s) {
    return 16 * (2 * ks + (s >> 2)) + 4 * g + (s & 3);
}

__device__ __forceinline__ bf16x8_t as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8_t, u); }

__device__ __forceinline__ floatx4 mfma(bf16x8_t a, bf16x8_t b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ReLU, round to bfloat16 and regroup a layer's four m-tiles into the two B
// operands (k-steps) of the next layer.
__device__ __forceinline__ void relu_pack(const floatx4 d[4], bf16x8_t h[2]) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int s = 0; s < 8; ++s) h[ks][s] = (__bf16)fmaxf(d[2 * ks + (s >> 2)][s & 3], 0.0f);
}

__device__ __forceinline__ floatx4 bias4(const float *s_bias, int off) {
    return floatx4{s_bias[off], s_bias[off + 1], s_bias[off + 2], s_bias[off + 3]};
}

// Forward pass of 16 texels (one per n); lanes g < 2 supply the input slots in xb.
// d1..d3 keep the pre-activations, h1..h3 the bfloat16 activations as B operands.
// Returns D of the output layer: lanes with g == 0 hold o[0..3] of texel n.
__device__ __forceinline__ floatx4 mlp_forward(const bf16x8_t *wf, const float *s_bias, int g,
                                               bf16x8_t xb, floatx4 d1[4], floatx4 d2[4],
                                               floatx4 d3[4], bf16x8_t h1[2], bf16x8_t h2[2],
                                               bf16x8_t h3[2]) {
    const floatx4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) d1[mt] = mfma(wf[mt], xb, zero);
    relu_pack(d1, h1);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        floatx4 acc = bias4(s_bias, 16 * mt + 4 * g);
        acc = mfma(wf[4 + 2 * mt], h1[0], acc);
        d2[mt] = mfma(wf[5 + 2 * mt], h1[1], acc);
    }
    relu_pack(d2, h2);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        floatx4 acc = bias4(s_bias, kHidden + 16 * mt + 4 * g);
        acc = mfma(wf[12 + 2 * mt], h2[0], acc);
        d3[mt] = mfma(wf[13 + 2 * mt], h2[1], acc);
    }
    relu_pack(d3, h3);
    floatx4 o = bias4(s_bias, 2 * kHidden + 4 * g);
    o = mfma(wf[20], h3[0], o);
    return mfma(wf[21], h3[1], o);
}

__device__ __forceinline__ void load_pack(const MlpPack &m, bf16x8_t *wf, float *s_bias) {
    const int lane = (int)__lane_id();
#pragma unroll
    for (int e = 0; e < kFwdEntries; ++e) wf[e] = as_bf16x8(m.fwd[e * 64 + lane]);
    for (int e = threadIdx.x; e < kBiasFloats; e += blockDim.x) s_bias[e] = m.bias[e];
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ------------------------------------------------------------------ packing --

// One thread per (entry, lane) of the forward and backward packs, plus the biases.
__global__ __launch_bounds__(256) void pack_mlp_kernel(const float *__restrict__ th,
                                                       uint4 *__restrict__ fwd,
                                                       uint4 *__restrict__ bwd,
                                                       float *__restrict__ bias) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    const int total = (kFwdEntries + kBwdEntries) * 64;
    if (id < kBiasFloats) {
        float b = 0.0f;
        if (id < kHidden) b = th[kOffB2 + id];
        else if (id < 2 * kHidden) b = th[kOffB3 + id - kHidden];
        else if (id - 2 * kHidden < kOutputs) b = th[kOffB4 + id - 2 * kHidden];
        bias[id] = b;
    }
    if (id >= total) return;
    const bool is_fwd = id < kFwdEntries * 64;
    const int e = is_fwd ? id >> 6 : (id >> 6) - kFwdEntries;
    const int lane = id & 63, m = lane & 15, g = lane >> 4;
    bf16x8_t v;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        float w = 0.0f;
        if (is_fwd) {
            if (e < 4) {                       // layer 1, m-tile e: natural feature order
                const int k = 8 * g + s;
                if (k < kFeatures) w = th[kOffW1 + (16 * e + m) * kFeatures + k];
            } else if (e < 20) {               // layers 2, 3: (m-tile, k-step)
                const int q = e < 12 ? e - 4 : e - 12, mt = q >> 1, ks = q & 1;
                const int off = e < 12 ? kOffW2 : kOffW3;
                w = th[off + (16 * mt + m) * kHidden + unit_of(ks, g, s)];
            } else {                           // layer 4, k-step e - 20, rows >= 4 are zero
                if (m < kOutputs) w = th[kOffW4 + m * kHidden + unit_of(e - 20, g, s)];
            }
        } else {
            if (e < 4) {                       // W4^T: rows = hidden units, k = outputs
                const int k = 8 * g + s;
                if (k < kOutputs) w = th[kOffW4 + k * kHidden + 16 * e + m];
            } else {                           // W3^T (e < 12), W2^T: (m-tile, k-step)
                const int q = e < 12 ? e - 4 : e - 12, mt = q >> 1, ks = q & 1;
                const int off = e < 12 ? kOffW3 : kOffW2;
                w = th[off + unit_of(ks, g, s) * kHidden + 16 * mt + m];
            }
        }
        v[s] = (__bf16)w;
    }
    const uint4 u = __builtin_bit_cast(uint4, v);
    if (is_fwd) fwd[id] = u;
    else bwd[id - kFwdEntries * 64] = u;
}

// ----------------------------------------------------------------- features --

// Slots 8g .. 8g+7 of the feature vector of interior irradiance texel t of probe p:
//   g = 0:  U_low / S (3), E_prev / S (3), mean E[t] / D, sqrt(mean E[t^2]) / D over
//           the k x k depth texels covering the texel (k = depth_res / irr_res)
//   g = 1:  texel direction (3), clamp(probe distance / D, -4, 4), 1, 0, 0, 0
__device__ __forceinline__ void feature_group(const FeatureArgs &f, int p, int t, int g,
                                              float v[8]) {
    const int ri = f.irr_res, rd = f.depth_res;
    const int i = t % ri, j = t / ri;
    if (g == 0) {
        const int si = ri + 2, sd = rd + 2;
        const size_t ti = (size_t)p * si * si * 3 + ((size_t)(j + 1) * si + (i + 1)) * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[c] = f.u_irr[ti + c] * f.inv_s;
            v[3 + c] = f.prev_irr[ti + c] * f.inv_s;
        }
        const int k = rd / ri;
        const float *dt = f.prev_depth + (size_t)p * sd * sd * 2;
        float m1 = 0.0f, m2 = 0.0f;
        for (int b = 0; b < k; ++b)
            for (int a = 0; a < k; ++a) {
                const float *d = dt + ((size_t)(k * j + b + 1) * sd + (k * i + a + 1)) * 2;
                m1 += d[0];
                m2 += d[1];
            }
        const float inv_kk = 1.0f / (float)(k * k);
        v[6] = m1 * inv_kk * f.inv_d;
        v[7] = sqrtf(fmaxf(m2 * inv_kk, 0.0f)) * f.inv_d;
    } else {
        v[0] = f.texel_dir[3 * t];
        v[1] = f.texel_dir[3 * t + 1];
        v[2] = f.texel_dir[3 * t + 2];
        v[3] = fminf(fmaxf(f.probe_sdf[p] * f.inv_d, -4.0f), 4.0f);
        v[4] = 1.0f;
        v[5] = v[6] = v[7] = 0.0f;
    }
}

__device__ __forceinline__ bf16x8_t to_bf16x8(const float v[8]) {
    bf16x8_t b;
#pragma unroll
    for (int s = 0; s < 8; ++s) b[s] = (__bf16)v[s];
    return b;
}

// ------------------------------------------------------------------ denoise --

constexpr int kWaves = 4;
constexpr int kDenoiseTiles = 4;   // 16-texel tiles a wave pushes through the network at once
constexpr int kDenoiseBlocksPerCu = 4;

// ReLU of one m-tile's D (units 16 mt + 4 g + r), rounded to bfloat16 into its slots
// of the next layer's B operands: k-step mt / 2, slots 4 (mt % 2) + r.
__device__ __forceinline__ void relu_into(floatx4 d, int mt, bf16x8_t h[2]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) h[mt >> 1][4 * (mt & 1) + r] = (__bf16)fmaxf(d[r], 0.0f);
}

// Forward pass of kDenoiseTiles 16-texel tiles with the weight packs in LDS: each
// A operand is read once and applied to every tile, and each layer is produced one
// m-tile at a time straight into the next layer's operands (no pre-activations are
// kept), so that the kernel fits four waves per SIMD. The same products and
// roundings as mlp_forward. out[q]: lanes g == 0 hold o[0..3] of texel n of tile q.
template <int kT = kDenoiseTiles>
__device__ __forceinline__ void mlp_forward_lds(const uint4 *s_w, const float *s_bias, int g,
                                                int lane, const bf16x8_t xb[kT], floatx4 out[kT]) {
    const floatx4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8_t h[kT][2], hn[kT][2];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const bf16x8_t w = as_bf16x8(s_w[mt * 64 + lane]);
#pragma unroll
        for (int q = 0; q < kT; ++q) relu_into(mfma(w, xb[q], zero), mt, h[q]);
    }
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const int e0 = layer ? 12 : 4, b0 = layer ? kHidden : 0;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8_t w0 = as_bf16x8(s_w[(e0 + 2 * mt) * 64 + lane]);
            const bf16x8_t w1 = as_bf16x8(s_w[(e0 + 2 * mt + 1) * 64 + lane]);
            const floatx4 b = bias4(s_bias, b0 + 16 * mt + 4 * g);
#pragma unroll
            for (int q = 0; q < kT; ++q)
                relu_into(mfma(w1, h[q][1], mfma(w0, h[q][0], b)), mt, hn[q]);
        }
#pragma unroll
        for (int q = 0; q < kT; ++q) {
            h[q][0] = hn[q][0];
            h[q][1] = hn[q][1];
        }
    }
    const bf16x8_t w0 = as_bf16x8(s_w[20 * 64 + lane]), w1 = as_bf16x8(s_w[21 * 64 + lane]);
    const floatx4 b = bias4(s_bias, 2 * kHidden + 4 * g);
#pragma unroll
    for (int q = 0; q < kT; ++q) out[q] = mfma(w1, h[q][1], mfma(w0, h[q][0], b));
}

// One wave per probe (persistent waves stride over probes). Per group of 16-texel
// tiles: features, the network, U_hat = max(0, E_prev + S o[0..2]) staged in LDS,
// and exp(o[3]) summed. A probe whose flag says it takes the plain update this frame
// (its fallback pass writes its maps) only records its prediction; every other probe
// mixes U_hat into its irradiance in place of the plain update (hysteresis, interior
// and borders), and the low-ray depth moments into its depth map. The flag is then
// replaced by the probe's decision for the learned frame after next: mean predicted
// error above tau.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void denoise_kernel(DenoiseArgs a) {
    __shared__ uint4 s_w[kFwdEntries * 64];
    __shared__ float s_bias[kBiasFloats];
    __shared__ float s_u[kWaves][kMaxLearnedRes * kMaxLearnedRes * 3];
    for (int e = threadIdx.x; e < kFwdEntries * 64; e += blockDim.x) s_w[e] = a.mlp.fwd[e];
    for (int e = threadIdx.x; e < kBiasFloats; e += blockDim.x) s_bias[e] = a.mlp.bias[e];
    __syncthreads();
    const int lane = (int)__lane_id(), n = lane & 15, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int ri = a.f.irr_res, Ti = ri * ri, tiles = (Ti + 15) >> 4;
    const int si = ri + 2, sd = a.f.depth_res + 2;
    const size_t tile_i = (size_t)si * si * 3, tile_d = (size_t)sd * sd * 2;
    float *su = s_u[wave];
    for (int p = blockIdx.x * kWaves + wave; p < a.P; p += gridDim.x * kWaves) {
        float esum = 0.0f;
        for (int tb = 0; tb < tiles; tb += kDenoiseTiles) {
            // keep the weight packs in LDS: without this the compiler hoists their
            // (loop-invariant) reads out of the probe loop into 88 registers
            asm volatile("" ::: "memory");
            bf16x8_t xb[kDenoiseTiles];
#pragma unroll
            for (int q = 0; q < kDenoiseTiles; ++q) {
                const int t = (tb + q) * 16 + n;
                float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                if (g < 2 && t < Ti) feature_group(a.f, p, t, g, v);
                xb[q] = to_bf16x8(v);
            }
            floatx4 o[kDenoiseTiles];
            mlp_forward_lds(s_w, s_bias, g, lane, xb, o);
#pragma unroll
            for (int q = 0; q < kDenoiseTiles; ++q) {
                const int t = (tb + q) * 16 + n;
                if (g == 0 && t < Ti) {
                    const float *prev = a.f.prev_irr + (size_t)p * tile_i +
                                        ((size_t)(t / ri + 1) * si + (t % ri + 1)) * 3;
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        su[3 * t + c] = fmaxf(0.0f, fmaf(a.s, o[q][c], prev[c]));
                    esum += expf(o[q][3]);
                }
            }
        }
        const float mean = wave_sum(esum) / (float)Ti;
        const int plain = __builtin_amdgcn_readfirstlane((int)a.fb_flag[p]);
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            if (a.mean_error) a.mean_error[p] = mean;
            a.fb_flag[p] = mean > a.tau ? 1 : 0;
        }
        if (plain) continue;
        __builtin_amdgcn_wave_barrier();
        const float h = a.hysteresis;
        float *new_i = a.new_irr + (size_t)p * tile_i;
        const float *old_i = a.f.prev_irr + (size_t)p * tile_i;
        // kBatch elements per lane at a time, every load issued before the stores (one
        // batch covers an 8x8 irradiance map and an 18x18 depth tile)
        constexpr int kBatch = 3;
        for (int e0 = 0; e0 < Ti * 3; e0 += 64 * kBatch) {
            float old[kBatch];
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int e = e0 + 64 * k + lane;
                const int t = e / 3, c = e - 3 * t;
                old[k] = e < Ti * 3 ? old_i[((t / ri + 1) * si + (t % ri + 1)) * 3 + c] : 0.0f;
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int e = e0 + 64 * k + lane;
                if (e >= Ti * 3) break;
                const int t = e / 3, c = e - 3 * t;
                const float u = su[e];
                store_with_border(new_i, ri, 3, t % ri, t / ri, c, fmaf(h, old[k] - u, u));
            }
        }
        // depth tiles are whole float4s: (res+2)^2 * 2 floats with res even
        const float4 *old_d = reinterpret_cast<const float4 *>(a.f.prev_depth + (size_t)p * tile_d);
        const float4 *ud = reinterpret_cast<const float4 *>(a.u_depth + (size_t)p * tile_d);
        float4 *new_d = reinterpret_cast<float4 *>(a.new_depth + (size_t)p * tile_d);
        const int nd4 = (int)(tile_d / 4);
        for (int e0 = 0; e0 < nd4; e0 += 64 * kBatch) {
            float4 u[kBatch], o[kBatch];
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int e = e0 + 64 * k + lane;
                if (e < nd4) {
                    u[k] = ud[e];
                    o[k] = old_d[e];
                }
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int e = e0 + 64 * k + lane;
                if (e >= nd4) break;
                new_d[e] = make_float4(fmaf(h, o[k].x - u[k].x, u[k].x),
                                       fmaf(h, o[k].y - u[k].y, u[k].y),
                                       fmaf(h, o[k].z - u[k].z, u[k].z),
                                       fmaf(h, o[k].w - u[k].w, u[k].w));
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// denoise_kernel for kRi x kRi irradiance and kRd x kRd depth maps small enough to
// stage a probe's tiles in LDS (8 x 8 and 16 x 16), with one memory round trip per
// probe instead of three: every load of the probe (its previous and low-ray depth
// tiles as float4s, the texels' features) is issued at once; the new depth tile is
// written as soon as they arrive, the previous one is kept in LDS for the depth
// features, and the new irradiance tile is assembled in LDS and written whole,
// borders included, with consecutive lanes on consecutive floats. The same values,
// rounded in the same order, as denoise_kernel.
template <int kRi, int kRd>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void denoise_tile_kernel(DenoiseArgs a) {
    constexpr int kTi = kRi * kRi, kSi = kRi + 2, kSd = kRd + 2, kK = kRd / kRi;
    constexpr int kTileI = kSi * kSi * 3, kD4 = kSd * kSd * 2 / 4, kD4Lane = (kD4 + 63) / 64;
    static_assert(kTi == 16 * kDenoiseTiles, "one group of 16-texel tiles per probe");
    static_assert(kRd % kRi == 0 && (kSd * kSd * 2) % 4 == 0, "depth tile of whole float4s");
    __shared__ uint4 s_w[kFwdEntries * 64];
    __shared__ float s_bias[kBiasFloats];
    __shared__ float4 s_dep[kWaves][kD4];
    __shared__ float s_irr[kWaves][kTi * 3];
    for (int e = threadIdx.x; e < kFwdEntries * 64; e += blockDim.x) s_w[e] = a.mlp.fwd[e];
    for (int e = threadIdx.x; e < kBiasFloats; e += blockDim.x) s_bias[e] = a.mlp.bias[e];
    __syncthreads();
    const int lane = (int)__lane_id(), n0 = lane & 15, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const float *sdep = reinterpret_cast<const float *>(s_dep[wave]);
    float *sirr = s_irr[wave];
    const float h = a.hysteresis, inv_s = a.f.inv_s, inv_d = a.f.inv_d;
    for (int p = blockIdx.x * kWaves + wave; p < a.P; p += gridDim.x * kWaves) {
        asm volatile("" ::: "memory");   // the packs stay in LDS (see denoise_kernel)
        // fresh copies each probe: addresses derived from the lane are recomputed
        // rather than hoisted out of the loop into registers the network needs
        int n = n0, ln = lane;
        asm volatile("" : "+v"(n), "+v"(ln));
        const int plain = __builtin_amdgcn_readfirstlane((int)a.fb_flag[p]);
        const size_t di = (size_t)p * kD4, ii = (size_t)p * kTileI;
        const float4 *old_d = reinterpret_cast<const float4 *>(a.f.prev_depth) + di;
        const float4 *low_d = reinterpret_cast<const float4 *>(a.u_depth) + di;
        float4 od[kD4Lane], ud[kD4Lane];
#pragma unroll
        for (int k = 0; k < kD4Lane; ++k) {
            const int e = 64 * k + ln;
            if (e < kD4) {
                od[k] = old_d[e];
                if (!plain) ud[k] = low_d[e];
            }
        }
        // g == 0: low-ray and previous irradiance of the texel; g == 1: its direction
        float fv[kDenoiseTiles][6];
#pragma unroll
        for (int q = 0; q < kDenoiseTiles; ++q) {
            const int t = q * 16 + n;
            if (g == 0) {
                const size_t at = ii + ((size_t)(t / kRi + 1) * kSi + (t % kRi + 1)) * 3;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    fv[q][c] = a.f.u_irr[at + c];
                    fv[q][3 + c] = a.f.prev_irr[at + c];
                }
            } else if (g == 1) {
#pragma unroll
                for (int c = 0; c < 3; ++c) fv[q][c] = a.f.texel_dir[3 * t + c];
            }
        }
        const float sdf = g == 1 ? a.f.probe_sdf[p] : 0.0f;
        float4 *new_d = reinterpret_cast<float4 *>(a.new_depth) + di;
#pragma unroll
        for (int k = 0; k < kD4Lane; ++k) {
            const int e = 64 * k + ln;
            if (e < kD4) {
                if (!plain)
                    new_d[e] = make_float4(fmaf(h, od[k].x - ud[k].x, ud[k].x),
                                           fmaf(h, od[k].y - ud[k].y, ud[k].y),
                                           fmaf(h, od[k].z - ud[k].z, ud[k].z),
                                           fmaf(h, od[k].w - ud[k].w, ud[k].w));
                s_dep[wave][e] = od[k];
            }
        }
        __builtin_amdgcn_wave_barrier();
        // features (feature_group's slots and order), the previous irradiance to LDS
        bf16x8_t xb[kDenoiseTiles];
#pragma unroll
        for (int q = 0; q < kDenoiseTiles; ++q) {
            const int t = q * 16 + n, i = t % kRi, j = t / kRi;
            float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (g == 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    v[c] = fv[q][c] * inv_s;
                    v[3 + c] = fv[q][3 + c] * inv_s;
                    sirr[3 * t + c] = fv[q][3 + c];
                }
                float m1 = 0.0f, m2 = 0.0f;
#pragma unroll
                for (int b = 0; b < kK; ++b)
#pragma unroll
                    for (int c = 0; c < kK; ++c) {
                        const float *d = sdep + ((kK * j + b + 1) * kSd + (kK * i + c + 1)) * 2;
                        m1 += d[0];
                        m2 += d[1];
                    }
                const float inv_kk = 1.0f / (float)(kK * kK);
                v[6] = m1 * inv_kk * inv_d;
                v[7] = sqrtf(fmaxf(m2 * inv_kk, 0.0f)) * inv_d;
            } else if (g == 1) {
                v[0] = fv[q][0];
                v[1] = fv[q][1];
                v[2] = fv[q][2];
                v[3] = fminf(fmaxf(sdf * inv_d, -4.0f), 4.0f);
                v[4] = 1.0f;
            }
            xb[q] = to_bf16x8(v);
        }
        // two tiles at a time: the activations of four do not fit beside the rest
        floatx4 o[kDenoiseTiles];
        mlp_forward_lds<2>(s_w, s_bias, g, lane, xb, o);
        __builtin_amdgcn_sched_barrier(0);
        mlp_forward_lds<2>(s_w, s_bias, g, lane, xb + 2, o + 2);
        // U_hat, the hysteresis mix in place of the previous value, the error sum
        float esum = 0.0f;
#pragma unroll
        for (int q = 0; q < kDenoiseTiles; ++q) {
            const int t = q * 16 + n;
            if (g == 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float prev = sirr[3 * t + c];
                    const float u = fmaxf(0.0f, fmaf(a.s, o[q][c], prev));
                    sirr[3 * t + c] = fmaf(h, prev - u, u);
                }
                esum += expf(o[q][3]);
            }
        }
        const float mean = wave_sum(esum) / (float)kTi;
        if (lane == 0) {
            if (a.mean_error) a.mean_error[p] = mean;
            a.fb_flag[p] = mean > a.tau ? 1 : 0;
        }
        if (plain) continue;
        __builtin_amdgcn_wave_barrier();
        float *new_i = a.new_irr + ii;
        for (int e = ln; e < kTileI; e += 64) {
            const int pos = e / 3, c = e - 3 * pos;
            int i, j;
            padded_source(kRi, pos % kSi, pos / kSi, i, j);
            new_i[e] = sirr[3 * (j * kRi + i) + c];
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// One thread per probe: the frame's fallback list, from the flags and (when given)
// the reject flags, which are folded into the flags.
__global__ __launch_bounds__(256) void select_fallback_kernel(const uint8_t *__restrict__ reject,
                                                              uint8_t *__restrict__ fb_flag,
                                                              int P, int *__restrict__ list,
                                                              int *__restrict__ count) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    if ((reject && reject[p]) || fb_flag[p]) {
        fb_flag[p] = 1;
        list[atomicAdd(count, 1)] = p;
    }
}

// ---------------------------------------------------------------- examples ---

// One thread per (probe, texel): the 16 features and the target pair.
__global__ __launch_bounds__(256) void examples_kernel(ExampleArgs a) {
    const int Ti = a.f.irr_res * a.f.irr_res;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)a.P * Ti) return;
    const int p = (int)(id / Ti), t = (int)(id - (int64_t)p * Ti);
    float v[8];
    float *x = a.features + id * kFeatures;
    feature_group(a.f, p, t, 0, v);
#pragma unroll
    for (int s = 0; s < 8; ++s) x[s] = v[s];
    feature_group(a.f, p, t, 1, v);
#pragma unroll
    for (int s = 0; s < 8; ++s) x[8 + s] = v[s];
    const int ri = a.f.irr_res, si = ri + 2;
    const size_t at = (size_t)p * si * si * 3 + ((size_t)(t / ri + 1) * si + (t % ri + 1)) * 3;
    float *z = a.targets + id * 4;
    float l1 = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float u = a.target_irr[at + c];
        z[c] = (u - a.f.prev_irr[at + c]) * a.f.inv_s;
        l1 += fabsf(u);
    }
    z[3] = l1 * a.f.inv_s + a.rel_floor;
}

// ------------------------------------------------------------------- infer ---

__global__ __launch_bounds__(256) void infer_kernel(InferArgs a) {
    __shared__ float s_bias[kBiasFloats];
    bf16x8_t wf[kFwdEntries];
    load_pack(a.mlp, wf, s_bias);
    __syncthreads();
    const int lane = (int)__lane_id(), n = lane & 15, g = lane >> 4;
    const int64_t tiles = (a.n + 15) >> 4;
    for (int64_t tile = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); tile < tiles;
         tile += (int64_t)gridDim.x * kWaves) {
        const int64_t q = tile * 16 + n;
        float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (g < 2 && q < a.n) {
            const float *x = a.features + q * kFeatures + 8 * g;
#pragma unroll
            for (int s = 0; s < 8; ++s) v[s] = x[s];
        }
        floatx4 d1[4], d2[4], d3[4];
        bf16x8_t h1[2], h2[2], h3[2];
        const floatx4 o = mlp_forward(wf, s_bias, g, to_bf16x8(v), d1, d2, d3, h1, h2, h3);
        if (g == 0 && q < a.n) {
            float *out = a.out + q * kOutputs;
            out[0] = o[0]; out[1] = o[1]; out[2] = o[2]; out[3] = o[3];
        }
    }
}

// ------------------------------------------------------------------- train ---

constexpr int kTrainBlock = 128;             // samples per workgroup iteration
constexpr int kRowPitch = kTrainBlock + 8;   // bfloat16 per LDS row (+8 spreads banks)
// LDS rows: inputs, activations of the three hidden layers, output gradients
// (rows >= 4 stay zero), hidden gradients after their ReLU masks
constexpr int kRowX = 0, kRowH1 = 16, kRowH2 = 80, kRowH3 = 144, kRowDO = 208;
constexpr int kRowG1 = 224, kRowG2 = 288, kRowG3 = 352, kRows = 416;

__device__ __forceinline__ uint64_t splitmix_first(uint64_t state) {
    uint64_t z = state + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Store a layer's D-layout values (unit 16 mt + 4 g + r of sample column) as
// bfloat16 rows of the LDS matrix starting at `row0`.
__device__ __forceinline__ void store_units(__bf16 *lds, int row0, int g, int col,
                                            const floatx4 d[4], bool relu) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float v = relu ? fmaxf(d[mt][r], 0.0f) : d[mt][r];
            lds[(row0 + 16 * mt + 4 * g + r) * kRowPitch + col] = (__bf16)v;
        }
}

// Hidden gradient of one layer from the next layer's gradient B operands:
// D = W^T g_next (per m-tile, two k-steps), masked where the pre-activation is <= 0.
__device__ __forceinline__ void back_layer(const bf16x8_t *wb, const bf16x8_t gn[2],
                                           const floatx4 pre[4], floatx4 out[4]) {
    const floatx4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        floatx4 acc = mfma(wb[2 * mt], gn[0], zero);
        acc = mfma(wb[2 * mt + 1], gn[1], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) out[mt][r] = pre[mt][r] > 0.0f ? acc[r] : 0.0f;
    }
}

// Gradient of the mean loss over the step's samples (see the checker's loss). Each
// workgroup iteration takes 128 samples: every wave runs 2 x 16 of them forward and
// backward in registers and writes inputs, activations and gradients as bfloat16
// rows to LDS; then the 40 weight-gradient tiles (dW1 4, dW2 16, dW3 16, dW4 4) are
// contracted over the samples on MFMA, 10 per wave, accumulating in registers across
// iterations, and the bias gradients are summed from the same rows. One atomic add
// per gradient element and workgroup at the end.
__global__ __launch_bounds__(256) void train_kernel(TrainArgs a) {
    __shared__ float s_bias[kBiasFloats];
    __shared__ __attribute__((aligned(16))) __bf16 s_m[kRows * kRowPitch];
    __shared__ float s_loss[kWaves];
    bf16x8_t wf[kFwdEntries], wb[kBwdEntries];
    load_pack(a.mlp, wf, s_bias);
    const int lane = (int)__lane_id(), n = lane & 15, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
#pragma unroll
    for (int e = 0; e < kBwdEntries; ++e) wb[e] = as_bf16x8(a.mlp.bwd[e * 64 + lane]);
    for (int e = threadIdx.x; e < 16 * kRowPitch; e += blockDim.x)
        s_m[kRowDO * kRowPitch + e] = (__bf16)0.0f;
    __syncthreads();

    floatx4 acc[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;     // bias gradient of row threadIdx.x (< 132)
    float lsum = 0.0f;
    const floatx4 zero = {0.0f, 0.0f, 0.0f, 0.0f};

    const int blocks = (a.batch + kTrainBlock - 1) / kTrainBlock;
    for (int blk = blockIdx.x; blk < blocks; blk += gridDim.x) {
        // ---- forward and backward, 2 x 16 samples per wave
        for (int half = 0; half < 2; ++half) {
            const int col = wave * 32 + half * 16 + n;       // sample column in LDS
            const int pos = blk * kTrainBlock + col;         // position in the batch
            const bool valid = pos < a.batch;
            int64_t idx = 0;
            if (valid) idx = a.sequential ? pos : (int64_t)(splitmix_first(a.seed + (uint64_t)pos) %
                                                            (uint64_t)a.count);
            float v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (g < 2 && valid) {
                const float *x = a.features + idx * kFeatures + 8 * g;
#pragma unroll
                for (int s = 0; s < 8; ++s) v[s] = x[s];
            }
            const bf16x8_t xb = to_bf16x8(v);
            floatx4 d1[4], d2[4], d3[4];
            bf16x8_t h1[2], h2[2], h3[2];
            const floatx4 o = mlp_forward(wf, s_bias, g, xb, d1, d2, d3, h1, h2, h3);
            // output gradient (lanes g == 0 own the sample's four outputs)
            float go[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (g == 0 && valid) {
                const float *z = a.targets + idx * 4;
                float err = 0.0f, sq = 0.0f;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float dlt = o[c] - z[c];
                    sq += dlt * dlt;
                    err += fabsf(dlt);
                    go[c] = 2.0f * a.inv_n * dlt;
                }
                const float r = err / z[3];
                const float dh = o[3] - logf(fmaxf(r, a.min_error));
                go[3] = 2.0f * a.head_weight * a.inv_n * dh;
                lsum += (sq + a.head_weight * dh * dh) * a.inv_n;
            }
            bf16x8_t gb[2];
            gb[0] = bf16x8_t{(__bf16)go[0], (__bf16)go[1], (__bf16)go[2], (__bf16)go[3],
                             (__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f, (__bf16)0.0f};
            // hidden gradients: W4^T (k = outputs, one k-step), then W3^T, W2^T
            floatx4 g3[4], g2[4], g1[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const floatx4 t = mfma(wb[mt], gb[0], zero);
#pragma unroll
                for (int r = 0; r < 4; ++r) g3[mt][r] = d3[mt][r] > 0.0f ? t[r] : 0.0f;
            }
            bf16x8_t g3b[2], g2b[2];
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                for (int s = 0; s < 8; ++s) g3b[ks][s] = (__bf16)g3[2 * ks + (s >> 2)][s & 3];
            back_layer(wb + 4, g3b, d2, g2);
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                for (int s = 0; s < 8; ++s) g2b[ks][s] = (__bf16)g2[2 * ks + (s >> 2)][s & 3];
            back_layer(wb + 12, g2b, d1, g1);
            // rows for the weight-gradient contractions
            if (g < 2)
#pragma unroll
                for (int s = 0; s < 8; ++s) s_m[(kRowX + 8 * g + s) * kRowPitch + col] = xb[s];
            store_units(s_m, kRowH1, g, col, d1, true);
            store_units(s_m, kRowH2, g, col, d2, true);
            store_units(s_m, kRowH3, g, col, d3, true);
            store_units(s_m, kRowG1, g, col, g1, false);
            store_units(s_m, kRowG2, g, col, g2, false);
            store_units(s_m, kRowG3, g, col, g3, false);
            if (g == 0)
#pragma unroll
                for (int c = 0; c < 4; ++c) s_m[(kRowDO + c) * kRowPitch + col] = gb[0][c];
        }
        __syncthreads();
        // ---- weight gradients: tile k of this wave is tile id wave + 4 k
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            const int id = wave + 4 * k;
            int arow, brow;
            if (id < 4) { arow = kRowG1 + 16 * id; brow = kRowX; }
            else if (id < 20) { arow = kRowG2 + 16 * ((id - 4) >> 2); brow = kRowH1 + 16 * ((id - 4) & 3); }
            else if (id < 36) { arow = kRowG3 + 16 * ((id - 20) >> 2); brow = kRowH2 + 16 * ((id - 20) & 3); }
            else { arow = kRowDO; brow = kRowH3 + 16 * (id - 36); }
#pragma unroll
            for (int k0 = 0; k0 < kTrainBlock; k0 += 32) {
                const bf16x8_t av = *reinterpret_cast<const bf16x8_t *>(
                    &s_m[(arow + n) * kRowPitch + k0 + 8 * g]);
                const bf16x8_t bv = *reinterpret_cast<const bf16x8_t *>(
                    &s_m[(brow + n) * kRowPitch + k0 + 8 * g]);
                acc[k] = mfma(av, bv, acc[k]);
            }
        }
        // bias gradients: rows G2 (b2), G3 (b3), DO 0..3 (b4)
        if (threadIdx.x < 2 * kHidden + kOutputs) {
            const int row = threadIdx.x < kHidden ? kRowG2 + threadIdx.x
                          : threadIdx.x < 2 * kHidden ? kRowG3 + threadIdx.x - kHidden
                                                      : kRowDO + threadIdx.x - 2 * kHidden;
            float sum = 0.0f;
            for (int c = 0; c < kTrainBlock; ++c) sum += (float)s_m[row * kRowPitch + c];
            bsum += sum;
        }
        __syncthreads();
    }
    // ---- accumulate into the global gradient: D[4g + r][n] of tile (out mt, in nt)
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        const int id = wave + 4 * k;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 4 * g + r;
            int dst;
            if (id < 4) dst = kOffW1 + (16 * id + row) * kFeatures + n;
            else if (id < 20) dst = kOffW2 + (16 * ((id - 4) >> 2) + row) * kHidden + 16 * ((id - 4) & 3) + n;
            else if (id < 36) dst = kOffW3 + (16 * ((id - 20) >> 2) + row) * kHidden + 16 * ((id - 20) & 3) + n;
            else dst = row < kOutputs ? kOffW4 + row * kHidden + 16 * (id - 36) + n : -1;
            if (dst >= 0) atomicAdd(a.grad + dst, acc[k][r]);
        }
    }
    if (threadIdx.x < 2 * kHidden + kOutputs) {
        const int dst = threadIdx.x < kHidden ? kOffB2 + threadIdx.x
                      : threadIdx.x < 2 * kHidden ? kOffB3 + threadIdx.x - kHidden
                                                  : kOffB4 + threadIdx.x - 2 * kHidden;
        atomicAdd(a.grad + dst, bsum);
    }
    const float wl = wave_sum(lsum);
    if (lane == 0) s_loss[wave] = wl;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(a.loss, s_loss[0] + s_loss[1] + s_loss[2] + s_loss[3]);
}

__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const float g = a.grad[k];
    const float m = a.beta1 * a.m[k] + (1.0f - a.beta1) * g;
    const float v = a.beta2 * a.v[k] + (1.0f - a.beta2) * g * g;
    a.m[k] = m;
    a.v[k] = v;
    a.theta[k] -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
    a.grad[k] = 0.0f;
}

__global__ __launch_bounds__(256) void zero_f32_kernel(float *dst, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = 0.0f;
}

// ---------------------------------------------------------------- launchers --

static unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

static int device_cus() {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus > 0 ? cus : 256;
}

hipError_t launch_pack_mlp(const float *theta, uint4 *fwd, uint4 *bwd, float *bias,
                           hipStream_t s) {
    const int total = (kFwdEntries + kBwdEntries) * 64;
    hipLaunchKernelGGL(pack_mlp_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, theta, fwd,
                       bwd, bias);
    return hipGetLastError();
}

hipError_t launch_denoise(const DenoiseArgs &a, hipStream_t s) {
    // persistent: as many workgroups as are resident at once (each loads the weight
    // packs into its LDS once)
    const int blocks =
        (int)std::min<int64_t>(grid_for(a.P, kWaves), kDenoiseBlocksPerCu * device_cus());
    if (a.f.irr_res == 8 && a.f.depth_res == 16)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(denoise_tile_kernel<8, 16>), dim3(blocks), dim3(256), 0,
                           s, a);
    else
        hipLaunchKernelGGL(denoise_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_select_fallback(const uint8_t *reject, uint8_t *fb_flag, int P, int *list,
                                  int *count, hipStream_t s) {
    hipLaunchKernelGGL(select_fallback_kernel, dim3(grid_for(P, 256)), dim3(256), 0, s, reject,
                       fb_flag, P, list, count);
    return hipGetLastError();
}

hipError_t launch_examples(const ExampleArgs &a, hipStream_t s) {
    const int64_t n = (int64_t)a.P * a.f.irr_res * a.f.irr_res;
    hipLaunchKernelGGL(examples_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_infer(const InferArgs &a, hipStream_t s) {
    const int64_t tiles = (a.n + 15) / 16;
    const int blocks = (int)std::min<int64_t>(grid_for(tiles, kWaves), 8 * device_cus());
    hipLaunchKernelGGL(infer_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_train(const TrainArgs &a, hipStream_t s) {
    const int blocks = (int)std::min<int64_t>(grid_for(a.batch, kTrainBlock), device_cus());
    hipLaunchKernelGGL(train_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_zero_f32(float *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_f32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, n);
    return hipGetLastError();
}

}  // namespace sdfddgi
