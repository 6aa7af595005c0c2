// The Eq. 3 blend of one workgroup's probes, shared by the single-scene kernels
// (kernels.hip) and the batched ones (batch.hip).
#pragma once

#include "internal.h"
#include "octahedral.h"

namespace sdfddgi {

constexpr int kBlendProbes = 16;  // probes per workgroup: the N extent of a tile row
typedef float floatx4 __attribute__((ext_vector_type(4)));

// The probes of one blend workgroup of kP (slots pb .. pb+np-1 of the probe list, or
// of 0..P-1) and their hysteresis: none where the history is rejected. The first
// __syncthreads of the caller's ray loop publishes them.
template <int kP = kBlendProbes>
__device__ __forceinline__ void load_blend_probes(const BlendArgs &a, int pb, int np, int *s_pid,
                                                  float *s_h) {
    const int tid = threadIdx.x;
    if (tid < kP) {
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
// kClamp (precision form): the depth map's second moment is raised to the square of
// its first where rounding left it below (the moments of any set of depths satisfy
// E[t^2] >= E[t]^2); the two moments of a probe sit in neighbouring lanes.
template <bool kClamp = false>
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
        float v = nrm < 0.0f ? old : fmaf(h, old - u, u);
        if (kClamp && !irr) {
            const float first = __shfl_xor(v, 1);  // lane pairs (row, row ^ 1) hold (E[t], E[t^2])
            if (c == 1) v = fmaxf(v, first * first);
        }
        store_with_border(new_tile, res, comps, i, j, c, v);
    }
}

// Floats of the LDS buffer the standard-layout epilogue needs: 16 probes x 256
// depth texels x 2 moments (the irradiance map, 16 x 64 x 3, fits in it too).
constexpr int kEpilogueFloats = kBlendProbes * 256 * 2;

// One map of the standard-layout epilogue (n x n interior, comps components per
// texel) through LDS: the waves have left the normalised update u of each interior
// texel in buf as [probe][texel][component]; the workgroup mixes it with the
// previous interior (hysteresis, or none where the history is rejected; the previous
// value where all weights vanish), then writes every probe's whole padded tile,
// interior and border, in order -- coalesced reads and stores instead of one
// scattered store per texel and border copy. kFast: the previous interior read
// kBatch elements per thread at a time (every read issued before the first use),
// and each padded position's source taken from a table built once per workgroup
// instead of being derived per element; the same values, the same order.
template <int kN, int kComps, bool kClamp = false, bool kFast = false>
__device__ __forceinline__ void epilogue_map_lds(const float *prev, float *next, const float *norm,
                                                 const float *s_h, const int *s_pid, int np,
                                                 float *buf) {
    constexpr int T = kN * kN, kSide = kN + 2, kTile = kSide * kSide * kComps;
    const int tid = threadIdx.x, total = np * T * kComps;
    __shared__ short s_src[kFast ? kTile : 1];
    if (kFast)
        for (int r = tid; r < kTile; r += 256) {
            const int pos = r / kComps, c = r - pos * kComps;
            int i, j;
            padded_source(kN, pos % kSide, pos / kSide, i, j);
            s_src[r] = (short)((j * kN + i) * kComps + c);
        }
    __syncthreads();  // the waves' updates are in buf
    if (kFast) {
        constexpr int kBatch = 8;   // past the end a thread reads the last element, unused
        for (int e0 = 0; e0 < total; e0 += 256 * kBatch) {
            float old[kBatch], nrm[kBatch];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const int e = min(e0 + 256 * b + tid, total - 1);
                const int q = e / (T * kComps), rem = e - q * (T * kComps);
                const int t = rem / kComps, c = rem - t * kComps;
                const int i = t % kN, j = t / kN;
                old[b] = prev[(size_t)s_pid[q] * kTile + ((j + 1) * kSide + (i + 1)) * kComps + c];
                nrm[b] = norm[t];
            }
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const int e = e0 + 256 * b + tid;
                if (e < total) {
                    const float u = buf[e];
                    buf[e] = nrm[b] < 0.0f ? old[b] : fmaf(s_h[e / (T * kComps)], old[b] - u, u);
                }
            }
        }
    } else {
        for (int e = tid; e < total; e += blockDim.x) {
            const int q = e / (T * kComps), rem = e - q * (T * kComps);
            const int t = rem / kComps, c = rem - t * kComps;
            const int i = t % kN, j = t / kN;
            const float old = prev[(size_t)s_pid[q] * kTile + ((j + 1) * kSide + (i + 1)) * kComps + c];
            const float nrm = norm[t];
            const float u = buf[e];
            buf[e] = nrm < 0.0f ? old : fmaf(s_h[q], old - u, u);
        }
    }
    if (kClamp) {  // moments (kComps == 2): E[t^2] no smaller than E[t]^2
        __syncthreads();
        for (int e = tid; e < np * T; e += blockDim.x)
            buf[2 * e + 1] = fmaxf(buf[2 * e + 1], buf[2 * e] * buf[2 * e]);
    }
    __syncthreads();
    for (int e = tid; e < np * kTile; e += blockDim.x) {
        const int q = e / kTile, rem = e - q * kTile;
        if (kFast) {
            next[(size_t)s_pid[q] * kTile + rem] = buf[q * T * kComps + s_src[rem]];
        } else {
            const int pos = rem / kComps, c = rem - pos * kComps;
            int i, j;
            padded_source(kN, pos % kSide, pos / kSide, i, j);
            next[(size_t)s_pid[q] * kTile + rem] = buf[(q * T + j * kN + i) * kComps + c];
        }
    }
    __syncthreads();  // buf is free again
}

// Epilogue of the standard layout (8x8 irradiance in slot 0 of every wave, 16x16
// depth in slots 1..4) for one workgroup's probes; buf: kEpilogueFloats of LDS that
// the caller no longer needs. kClamp: as for blend_epilogue. kNi / kNd: the 16-column
// N-tiles of the irradiance (3 per probe) and depth (2 per probe) products. kFast: as
// for epilogue_map_lds.
template <bool kClamp = false, int kNi = 3, int kNd = 2, bool kFast = false>
__device__ __forceinline__ void blend_epilogue_std(const BlendArgs &a, const float *s_h,
                                                   const int *s_pid, int np, int wave, int row,
                                                   int krow, const floatx4 (&acc)[kMSlots][kNi],
                                                   float *buf) {
    __syncthreads();  // every wave is done with what buf held before
#pragma unroll
    for (int n = 0; n < kNi; ++n) {
        const int col = n * 16 + row, q = col / 3, c = col - 3 * q;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int t = wave * 16 + 4 * krow + r;
            if (q < np) buf[(q * 64 + t) * 3 + c] = acc[0][n][r] * a.norm_i[t];
        }
    }
    epilogue_map_lds<8, 3, false, kFast>(a.prev_irr, a.new_irr, a.norm_i, s_h, s_pid, np, buf);
#pragma unroll
    for (int s = 1; s < kMSlots; ++s) {
        const int tile = (s - 1) * 4 + wave;
#pragma unroll
        for (int n = 0; n < kNd; ++n) {
            const int col = n * 16 + row, q = col >> 1, m = col & 1;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = tile * 16 + 4 * krow + r;
                if (q < np) buf[(q * 256 + t) * 2 + m] = acc[s][n][r] * a.norm_d[t];
            }
        }
    }
    epilogue_map_lds<16, 2, kClamp, kFast>(a.prev_depth, a.new_depth, a.norm_d, s_h, s_pid, np,
                                           buf);
}

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// Precision form of the blend: the same tiling as blend_kernel, with the weights as
// FP16 (irradiance) / BF16 (depth) rows [T][Rpad] and the payload staged in LDS as
// FP16 radiance and BF16 (t, t^2) columns, contracted 32 rays at a time on
// v_mfma_f32_16x16x32_{f16,bf16} with FP32 accumulation.
// One workgroup's share (probe slots pb .. pb+kP-1) of the precision-form blend; also
// the body of the batched blend, which passes each scene's arguments. The tile: kP
// probes per workgroup (16: 3 irradiance and 2 depth N-tiles of 16 columns; 8: 2 and
// 1, the last irradiance tile a third empty) and kChunk rays staged in LDS at a time
// (a multiple of 32 that divides Rpad).
template <bool kStd, int kP = kBlendProbes, int kChunk = kBlendChunk>
__device__ __forceinline__ void blend16_block(const BlendArgs &a, int pb) {
    constexpr int kPitch = kChunk + 8;  // halves per LDS column (+8 spreads the banks)
    constexpr int kNi = (3 * kP + 15) / 16, kNd = (2 * kP + 15) / 16;
    // payload staging (FP16 radiance, BF16 moments); the standard layout's epilogue
    // reuses the buffer
    constexpr int kSi = (kP * 3 + 1) * kPitch, kSd = (kP * 2 + 1) * kPitch;
    static_assert(kP <= kBlendProbes && kChunk % 32 == 0, "tile within the buffers");
    static_assert((kSi + kSd) * 2 <= kEpilogueFloats * 4, "staging fits the epilogue buffer");
    static_assert(kSi % 8 == 0, "16-byte aligned depth staging");
    __shared__ __attribute__((aligned(16))) float sbuf[kEpilogueFloats];
    _Float16 *si = reinterpret_cast<_Float16 *>(sbuf);
    __bf16 *sd = reinterpret_cast<__bf16 *>(si + kSi);
    __shared__ float s_h[kP];
    __shared__ int s_pid[kP];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row = lane & 15, kgrp = lane >> 4;
    const int count = a.probe_list ? min(*a.probe_count, a.P) : a.P;
    if (pb >= count) return;
    const int np = min(kP, count - pb);
    const int Ti = a.irr_res * a.irr_res, Td = a.depth_res * a.depth_res;
    const int mti = (Ti + 15) >> 4, mtd = (Td + 15) >> 4;
    const int mtiles = mti + mtd;
    load_blend_probes<kP>(a, pb, np, s_pid, s_h);
    for (int e = tid; e < kPitch; e += 256) {
        si[kP * 3 * kPitch + e] = (_Float16)0.0f;
        sd[kP * 2 * kPitch + e] = (__bf16)0.0f;
    }
    int bi_off[kNi], bd_off[kNd];
#pragma unroll
    for (int n = 0; n < kNi; ++n) {
        const int col = n * 16 + row;
        bi_off[n] = (col / 3 < np ? col : kP * 3) * kPitch;
    }
#pragma unroll
    for (int n = 0; n < kNd; ++n) {
        const int col = n * 16 + row;
        bd_off[n] = ((col >> 1) < np ? col : kP * 2) * kPitch;
    }
    const int passes = kStd ? 1 : (mtiles + 4 * kMSlots - 1) / (4 * kMSlots);
    for (int pass = 0; pass < passes; ++pass) {
        floatx4 acc[kMSlots][kNi];
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
            for (int n = 0; n < kNi; ++n) acc[s][n] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        }
        for (int k0 = 0; k0 < a.Rpad; k0 += kChunk) {
            __syncthreads();
            const int kc = min(kChunk, a.R - k0);  // rays present in this chunk
            for (int e = tid; e < kP * kChunk; e += 256) {
                const int q = e / kChunk, kk = e - q * kChunk;
                float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (q < np && kk < kc) v = a.payload[(size_t)s_pid[q] * a.R + k0 + kk];
                si[(q * 3 + 0) * kPitch + kk] = (_Float16)v.x;
                si[(q * 3 + 1) * kPitch + kk] = (_Float16)v.y;
                si[(q * 3 + 2) * kPitch + kk] = (_Float16)v.z;
                sd[(q * 2 + 0) * kPitch + kk] = (__bf16)v.w;
                sd[(q * 2 + 1) * kPitch + kk] = (__bf16)(v.w * v.w);
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < kChunk; kk += 32) {
                const int kl = kk + 8 * kgrp;  // this lane's 8 rays within the chunk
                half8_t bi[kNi];
                bf16x8_t bd[kNd];
#pragma unroll
                for (int n = 0; n < kNi; ++n)
                    bi[n] = *reinterpret_cast<const half8_t *>(&si[bi_off[n] + kl]);
#pragma unroll
                for (int n = 0; n < kNd; ++n)
                    bd[n] = *reinterpret_cast<const bf16x8_t *>(&sd[bd_off[n] + kl]);
#pragma unroll
                for (int s = 0; s < kMSlots; ++s) {
                    if (kStd ? s == 0 : mt[s] < mti) {
                        const half8_t av = *reinterpret_cast<const half8_t *>(wi[s] + k0 + kl);
#pragma unroll
                        for (int n = 0; n < kNi; ++n)
                            acc[s][n] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bi[n], acc[s][n], 0, 0, 0);
                    } else if (kStd || mt[s] < mtiles) {
                        const bf16x8_t av = *reinterpret_cast<const bf16x8_t *>(wd[s] + k0 + kl);
#pragma unroll
                        for (int n = 0; n < kNd; ++n)
                            acc[s][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bd[n], acc[s][n], 0, 0, 0);
                    }
                }
            }
        }
        if (kStd) {
            blend_epilogue_std<true, kNi, kNd, true>(a, s_h, s_pid, np, wave, row, kgrp, acc, sbuf);
            continue;
        }
#pragma unroll
        for (int s = 0; s < kMSlots; ++s) {
            if (!kStd && mt[s] >= mtiles) continue;
            const bool irr = kStd ? s == 0 : mt[s] < mti;
#pragma unroll
            for (int n = 0; n < kNi; ++n) {
                if (!irr && n >= kNd) break;
                blend_epilogue<true>(a, s_h, s_pid, np, irr, irr ? mt[s] : mt[s] - mti, n, row,
                                     kgrp, acc[s][n]);
            }
        }
    }
    __syncthreads();
    if (tid < np && a.reject) a.reject[s_pid[tid]] = 0;
}

}  // namespace sdfddgi
