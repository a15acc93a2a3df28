// bf16 MFMA GEMM with fused epilogues for the MLP demapper.
//
// C[M x N] = sum_k A(m, k) B(k, n), A and B in bf16 addressed by element
// strides (so row-major, transposed and batched-transposed operands share
// one kernel), FP32 accumulation on v_mfma_f32_32x32x16_bf16. A block of 4
// waves owns a 64 x 64 output tile and walks K through LDS (64 k per stage,
// two stages' loads in flight, where both operands are k-contiguous with
// 16-byte rows; else 32 k per step); each wave owns a 32 x 32 quarter. Tiles are stored k-contiguous in LDS,
// so every lane's MFMA operand (8 consecutive k of one row / column) is one
// 16-byte read. Operands whose k is contiguous in memory are fetched 8 at a
// time; others are fetched along m / n and transposed on the way into LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>

namespace mdgmi {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kTile = 64;
constexpr int kKStep = 32;
constexpr int kLdsPitch = kKStep + 8;  // bf16 elements per LDS row (16-byte aligned rows)

// GELU, tanh form (Hendrycks & Gimpel 2016): x * sigmoid(2 sqrt(2/pi) (x + 0.044715 x^3)),
// evaluated with the base-2 exponential and the hardware reciprocal.
__device__ __forceinline__ float gelu_f(float x) {
    const float k = -2.0f * 0.7978845608028654f * 1.4426950408889634f;  // -2 sqrt(2/pi) log2(e)
    const float u = x * fmaf(0.044715f * k, x * x, k);
    return x * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(u));
}

__device__ __forceinline__ float gelu_grad_f(float x) {
    const float c = 0.7978845608028654f;
    const float k = -2.0f * c * 1.4426950408889634f;
    const float u = x * fmaf(0.044715f * k, x * x, k);
    const float sg = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(u));  // sigmoid(2 t), t = c (x + a x^3)
    // d/dx [x sigmoid(2t)] = sigmoid(2t) + x * 2 sigmoid(2t)(1 - sigmoid(2t)) dt/dx
    const float dt = c * fmaf(3.0f * 0.044715f, x * x, 1.0f);
    return fmaf(x * 2.0f * sg * (1.0f - sg), dt, sg);
}

enum Epi : int {
    kEpiF32 = 0,        // C (FP32) = bias[n] (if bias) + acc
    kEpiGeluBf16 = 1,   // Z (FP32) = bias[n] + acc; H (bf16) = gelu(Z)
    kEpiGeluGrad = 2,   // D (bf16) = acc * gelu'(Z[m][n])
    kEpiPartial = 3     // C + split * M * N (FP32) = acc  (split-K partials)
};

struct GemmArgs {
    const __bf16* A;
    int64_t a_sm, a_sk;          // element strides of A(m, k)
    const __bf16* B;
    int64_t b_sk, b_sn;          // element strides of B(k, n)
    int M, N;
    int64_t K;
    int64_t k_per_split;         // K range per grid.z slice (multiple of kKStep)
    const float* bias;           // [N] or null
    float* C;                    // FP32 output, row-major [M][ldc]
    int64_t ldc;
    __bf16* H;                   // bf16 output, row-major [M][ldh]
    int64_t ldh;
    const float* Z;              // pre-activation for kEpiGeluGrad, row-major [M][ldz]
    int64_t ldz;
    __bf16* Ht;                  // optional transposed copy of H, [N][ldht] (kEpiGeluBf16, kEpiGeluGrad)
    int64_t ldht;
};

template <bool A_K_CONTIG>
__device__ __forceinline__ void load_tile_a(const GemmArgs& g, int64_t m0, int64_t k0, int64_t k1, __bf16* As) {
    const int t = threadIdx.x;  // 256 threads
    if (A_K_CONTIG) {
        const int mm = t >> 2, kk = (t & 3) * 8;
        const int64_t m = m0 + mm;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int64_t k = k0 + kk + i;
            As[mm * kLdsPitch + kk + i] = (m < g.M && k < k1) ? g.A[m * g.a_sm + k * g.a_sk] : (__bf16)0.0f;
        }
    } else {
        // consecutive threads walk m (contiguous in memory), transposed store
        const int mm = t & 63, kk = (t >> 6) * 8;
        const int64_t m = m0 + mm;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int64_t k = k0 + kk + i;
            As[mm * kLdsPitch + kk + i] = (m < g.M && k < k1) ? g.A[m * g.a_sm + k * g.a_sk] : (__bf16)0.0f;
        }
    }
}

template <bool B_K_CONTIG>
__device__ __forceinline__ void load_tile_b(const GemmArgs& g, int64_t n0, int64_t k0, int64_t k1, __bf16* Bs) {
    const int t = threadIdx.x;
    if (B_K_CONTIG) {
        const int nn = t >> 2, kk = (t & 3) * 8;
        const int64_t n = n0 + nn;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int64_t k = k0 + kk + i;
            Bs[nn * kLdsPitch + kk + i] = (n < g.N && k < k1) ? g.B[k * g.b_sk + n * g.b_sn] : (__bf16)0.0f;
        }
    } else {
        const int nn = t & 63, kk = (t >> 6) * 8;
        const int64_t n = n0 + nn;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int64_t k = k0 + kk + i;
            Bs[nn * kLdsPitch + kk + i] = (n < g.N && k < k1) ? g.B[k * g.b_sk + n * g.b_sn] : (__bf16)0.0f;
        }
    }
}

template <bool A_K_CONTIG, bool B_K_CONTIG, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) __bf16 As[kTile * kLdsPitch];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[kTile * kLdsPitch];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;  // this wave's quarter
    const int64_t m0 = (int64_t)blockIdx.y * kTile, n0 = (int64_t)blockIdx.x * kTile;
    const int64_t kb = (int64_t)blockIdx.z * g.k_per_split;
    const int64_t ke = kb + g.k_per_split < g.K ? kb + g.k_per_split : g.K;
    f32x16 acc = {};
    // The epilogue's inputs are fetched before the K loop, so that their
    // latency is spent under it: the bias seeds the accumulators, and the
    // pre-activations that GELU' reads are held in registers.
    // lane holds rows 8 (r >> 2) + 4 (lane >> 5) + (r & 3) of column lane & 31
    const int64_t n = n0 + wn + (lane & 31);
    if constexpr (EPI == kEpiF32 || EPI == kEpiGeluBf16) {
        if (g.bias && n < g.N) {
            const float b = g.bias[n];
#pragma unroll
            for (int r = 0; r < 16; r++) acc[r] = b;
        }
    }
    float zp[16];
    if constexpr (EPI == kEpiGeluGrad) {
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int64_t m = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            zp[r] = (m < g.M && n < g.N) ? g.Z[m * g.ldz + n] : 0.0f;
        }
    }
    if constexpr (A_K_CONTIG && B_K_CONTIG) {
        // Both operands k-contiguous (every call of the training step): each
        // thread moves 8 consecutive k of one A row and one B column per
        // 32 k.
        const int t = threadIdx.x, rr = t >> 2, kk = (t & 3) * 8;
        const bool avec = g.a_sk == 1 && g.a_sm % 8 == 0 && ((uintptr_t)g.A & 15) == 0;
        const bool bvec = g.b_sk == 1 && g.b_sn % 8 == 0 && ((uintptr_t)g.B & 15) == 0;
        if (avec && bvec && (ke - kb) % 8 == 0 && ke - kb >= 8) {
            // 16-byte loads with no branch: rows past M / N and k past ke
            // read a clamped in-range address and are zeroed when stored to
            // LDS, so no load waits for another and each is first waited for
            // where its stage stores it.
            const bool arow = m0 + rr < g.M, brow = n0 + rr < g.N;
            const __bf16* pa = g.A + (arow ? m0 + rr : g.M - 1) * g.a_sm;
            const __bf16* pb = g.B + (brow ? n0 + rr : g.N - 1) * g.b_sn;
            auto ld = [&](const __bf16* p, int64_t k) { return *(const uint4*)(p + (k < ke - 8 ? k : ke - 8)); };
            // zeroing by masks on the values (a select of whole vectors is
            // made through the stack)
            auto masked = [](uint4 v, bool keep) {
                const uint32_t m = keep ? ~0u : 0u;
                return make_uint4(v.x & m, v.y & m, v.z & m, v.w & m);
            };
            // One stage of kStage k: the operands loaded two stages earlier
            // go to LDS, and the same registers take the loads for two stages
            // later, so two stages' loads are in flight under each stage's
            // MFMAs.
            constexpr int kStage = 64, kSub = kStage / 32, kStagePitch = kStage + 8;
            __shared__ __attribute__((aligned(16))) __bf16 Aw[kTile * kStagePitch];
            __shared__ __attribute__((aligned(16))) __bf16 Bw[kTile * kStagePitch];
            auto stage = [&](int64_t k0, uint4 (&ra)[kSub], uint4 (&rb)[kSub]) {
#pragma unroll
                for (int j = 0; j < kSub; j++) {
                    const bool kin = k0 + 32 * j + kk < ke;
                    *(uint4*)(Aw + rr * kStagePitch + 32 * j + kk) = masked(ra[j], arow && kin);
                    *(uint4*)(Bw + rr * kStagePitch + 32 * j + kk) = masked(rb[j], brow && kin);
                }
                __syncthreads();
                // unconditional (loads past ke read a clamped address and go
                // unused): a conditional load would be merged with the old
                // value, and that copy waits for the load
#pragma unroll
                for (int j = 0; j < kSub; j++) {
                    ra[j] = ld(pa, k0 + 2 * kStage + 32 * j + kk);
                    rb[j] = ld(pb, k0 + 2 * kStage + 32 * j + kk);
                }
#pragma unroll
                for (int ks = 0; ks < kStage; ks += 16) {
                    const int kofs = ks + 8 * (lane >> 5);
                    const bf16x8 a = *(const bf16x8*)(Aw + (wm + (lane & 31)) * kStagePitch + kofs);
                    const bf16x8 b = *(const bf16x8*)(Bw + (wn + (lane & 31)) * kStagePitch + kofs);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
                }
                __syncthreads();
            };
            uint4 ra0[kSub], rb0[kSub], ra1[kSub], rb1[kSub];
#pragma unroll
            for (int j = 0; j < kSub; j++) {
                ra0[j] = ld(pa, kb + 32 * j + kk);
                rb0[j] = ld(pb, kb + 32 * j + kk);
                ra1[j] = ld(pa, kb + kStage + 32 * j + kk);
                rb1[j] = ld(pb, kb + kStage + 32 * j + kk);
            }
            // stages in pairs; k past ke (in a stage or a whole stage) multiplies zeros
            for (int64_t k0 = kb; k0 < ke; k0 += 2 * kStage) {
                stage(k0, ra0, rb0);
                stage(k0 + kStage, ra1, rb1);
            }
        } else {
            // any pitch, pointer or K range: element loads, zero past the edges
            auto fetch = [&](const __bf16* base, int64_t row, int64_t rows, int64_t pitch, int64_t sk, int64_t k0) {
                const int64_t k = k0 + kk;
                union {
                    uint4 u;
                    __bf16 h[8];
                } p;
#pragma unroll
                for (int i = 0; i < 8; i++)
                    p.h[i] = (row < rows && k + i < ke) ? base[row * pitch + (k + i) * sk] : (__bf16)0.0f;
                return p.u;
            };
            for (int64_t k0 = kb; k0 < ke; k0 += kKStep) {
                *(uint4*)(As + rr * kLdsPitch + kk) = fetch(g.A, m0 + rr, g.M, g.a_sm, g.a_sk, k0);
                *(uint4*)(Bs + rr * kLdsPitch + kk) = fetch(g.B, n0 + rr, g.N, g.b_sn, g.b_sk, k0);
                __syncthreads();
#pragma unroll
                for (int ks = 0; ks < kKStep; ks += 16) {
                    const int kofs = ks + 8 * (lane >> 5);
                    const bf16x8 a = *(const bf16x8*)(As + (wm + (lane & 31)) * kLdsPitch + kofs);
                    const bf16x8 b = *(const bf16x8*)(Bs + (wn + (lane & 31)) * kLdsPitch + kofs);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
                }
                __syncthreads();
            }
        }
    } else {
        for (int64_t k0 = kb; k0 < ke; k0 += kKStep) {
            load_tile_a<A_K_CONTIG>(g, m0, k0, ke, As);
            load_tile_b<B_K_CONTIG>(g, n0, k0, ke, Bs);
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < kKStep; ks += 16) {
                const int kofs = ks + 8 * (lane >> 5);
                const bf16x8 a = *(const bf16x8*)(As + (wm + (lane & 31)) * kLdsPitch + kofs);
                const bf16x8 b = *(const bf16x8*)(Bs + (wn + (lane & 31)) * kLdsPitch + kofs);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
            }
            __syncthreads();
        }
    }
    __bf16 hv[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const int64_t m = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (m >= g.M || n >= g.N) continue;
        const float v = acc[r];
        if (EPI == kEpiF32) {
            g.C[m * g.ldc + n] = v;
        } else if (EPI == kEpiGeluBf16) {
            ((float*)g.C)[m * g.ldc + n] = v;  // pre-activation kept for the backward pass
            hv[r] = (__bf16)gelu_f(v);
            g.H[m * g.ldh + n] = hv[r];
        } else if (EPI == kEpiGeluGrad) {
            hv[r] = (__bf16)(v * gelu_grad_f(zp[r]));
            g.H[m * g.ldh + n] = hv[r];
        } else {
            g.C[(int64_t)blockIdx.z * g.M * g.N + m * g.N + n] = v;
        }
    }
    if constexpr (EPI == kEpiGeluBf16 || EPI == kEpiGeluGrad) {
        // H^T [n][m]: each run of four rows is four consecutive m of column n,
        // one 8-byte store where the run is whole and the pitch allows
        if (g.Ht && n < g.N) {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int64_t mb = m0 + wm + 8 * q + 4 * (lane >> 5);
                __bf16* dst = g.Ht + n * g.ldht + mb;
                if (mb + 4 <= g.M && g.ldht % 4 == 0 && ((uintptr_t)g.Ht & 7) == 0) {
                    union {
                        uint2 u;
                        __bf16 h[4];
                    } p;
#pragma unroll
                    for (int j = 0; j < 4; j++) p.h[j] = hv[4 * q + j];
                    *(uint2*)dst = p.u;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        if (mb + j < g.M) dst[j] = hv[4 * q + j];
                }
            }
        }
    }
}

}  // namespace mlp
}  // namespace mdgmi
