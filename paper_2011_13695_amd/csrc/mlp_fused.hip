// Fused inference of the MLP demapper: its logits (LLRs) or the GMI cost of
// those logits.
//
// Shape served: [in <= 16, 256, 256, 256, out <= 32]. Every layer is computed
// transposed, H_l^T = W_l H_(l-1)^T, on v_mfma_f32_32x32x16_bf16 with the
// weights as the A operand (rows = output features) and the activations as
// the B operand (columns = 32 samples of one wave). The MFMA output leaves
// each lane with 16 features of its sample; converted to bf16 they are
// directly the B operand of the next layer's K-blocks, provided the
// weights' input columns are permuted to match (layout built by
// k_fused_weights): for a K-block of 16 inputs, lane half h holds inputs
// {4h..4h+3, 8+4h..8+4h+3}. Activations never leave registers.
//
// GELU: the hidden layers' accumulators hold s = x / 4 (the weights of the
// first layer and the hidden biases are scaled by 1/4, the output layer's
// weights by 4, all exact powers of two), and they become GELU(4 s) / 4 in
// packed fp16 arithmetic without transcendentals (gelu_quarter8 below). In
// the hidden layers each output tile's GELUs run interleaved with the next
// tile's MFMA chain.
//
// LDS: W_1 (8 KiB), W_4 (16 KiB) and all biases stay resident; W_2 and W_3
// (128 KiB each) are staged in turn into one buffer, once per block of
// 32 samples per wave (8 waves by default, two per SIMD). In GMI mode the logits are turned into
// the per-sample GMI cost in the kernel and only FP64 block partials are
// written; in LLR mode the logits are stored, [n][out] FP32.
#include <algorithm>
#include <cmath>

#include "device_common.h"
#include "mlp_gemm.h"
#include "mlp_layout.h"

namespace mdgmi {
namespace fused {

using mlp::bf16x8;
using mlp::f32x16;

constexpr int kH = 256;                 // hidden width
constexpr int kTiles = kH / 32;         // output tiles of a hidden layer
constexpr int kKB = kH / 16;            // K-blocks of a hidden layer input
// LDS layout in 16-byte units
constexpr int kW1U = kTiles * 1 * 64;           // 512
constexpr int kW4U = 1 * kKB * 64;              // 1024
constexpr int kWHU = kTiles * kKB * 64;         // 8192 (128 KiB)
constexpr int kBiasF = 3 * kH + 32;             // floats

union P8 {
    bf16x8 v;
    uint4 u;
    __bf16 h[8];
};


// Accumulator seeded with the bias of output tile ot: register r of lane
// half h is row 8 (r >> 2) + 4 h + (r & 3), four runs of four consecutive
// rows, i.e. four 16-byte LDS reads straight into the accumulator.
__device__ __forceinline__ f32x16 bias_acc(const float* __restrict__ bias, int ot, int h) {
    f32x16 a;
#pragma unroll
    for (int g = 0; g < 4; g++) {
        const float4 v = *(const float4*)(bias + 32 * ot + 8 * g + 4 * h);
        a[4 * g + 0] = v.x;
        a[4 * g + 1] = v.y;
        a[4 * g + 2] = v.z;
        a[4 * g + 3] = v.w;
    }
    return a;
}

typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef _Float16 half8v __attribute__((ext_vector_type(8)));

__device__ __forceinline__ half8v splat8(float c) {
    const _Float16 h = (_Float16)c;
    return (half8v){h, h, h, h, h, h, h, h};
}

__device__ __forceinline__ half8v clamp01(half8v v) {
    return __builtin_elementwise_min(__builtin_elementwise_max(v, splat8(0.0f)), splat8(1.0f));
}

// The gate of the tanh-form GELU, Phi(x) = sigmoid(2 sqrt(2/pi) (x + 0.044715 x^3)),
// at x = 4 s is taken as clamp(1/2 + s P(v), 0, 1) with v = max(1 - s^2, 0)
// and P(v) = sum_k kGateP[k] v^k. P(0) = 1/2 makes the gate exactly 1 for
// x >= 4 and 0 for x <= -4 (the tanh form is within 2e-5 of those there).
// The coefficients are a minimax fit of the gate on [0, 4] (odd symmetry
// gives the rest), rounded to fp16 and then adjusted by a few fp16 ulps to
// minimise the error of the fp16 evaluation below; that error is at most
// 8e-4 on the gate and 2.1e-3 on GELU(x) - GELU_tanh(x) over all inputs.
constexpr float kGateP[7] = {0.5f, 0.241455078125f, 0.3515625f, -0.87451171875f,
                             2.96875f, -3.5546875f, 1.9609375f};

// GELU(4 s) / 4 = s Phi(4 s) of eight accumulators, rounded to bf16: s to
// fp16 (toward zero, v_cvt_pkrtz, two values per instruction), v, P and the
// gate in packed fp16 FMAs (with the [0, 1] clamp of the instruction), the
// product with the FP32 s in one v_fma_mix_f32 per value. 12 issue slots per
// pair against 19 for the exp2 + reciprocal form. Eight values at a time
// give four independent Horner chains: a chain of dependent packed FMAs
// would need a wait state between its steps.
__device__ __forceinline__ void gelu_quarter8(const float* z, bf16x8& out) {
    half8v s;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const half2v t = __builtin_bit_cast(half2v, __builtin_amdgcn_cvt_pkrtz(z[2 * i], z[2 * i + 1]));
        s[2 * i] = t.x;
        s[2 * i + 1] = t.y;
    }
    const half8v v = clamp01(__builtin_elementwise_fma(-s, s, splat8(1.0f)));
    half8v p = splat8(kGateP[6]);
#pragma unroll
    for (int k = 5; k >= 0; k--) p = __builtin_elementwise_fma(p, v, splat8(kGateP[k]));
    const half8v phi = clamp01(__builtin_elementwise_fma(s, p, splat8(0.5f)));
#pragma unroll
    for (int i = 0; i < 8; i++)  // fma with +0, not a product, keeps the fp16 conversion inside v_fma_mix_f32
        out[i] = (__bf16)__builtin_fmaf(z[i], (float)phi[i], 0.0f);
}

// Keeps a value's computation where it is written: without it the compiler
// may sink a tile's GELUs towards their use in the next layer, out of the
// MFMA chain they are meant to overlap.
__device__ __forceinline__ void pin(bf16x8& v) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 u = __builtin_bit_cast(u32x4, v);
    asm volatile("" : "+v"(u));
    v = __builtin_bit_cast(bf16x8, u);
}

// Sixteen accumulators of one output tile -> two bf16x8 activations.
__device__ __forceinline__ void gelu_tile(const f32x16& z, bf16x8& lo, bf16x8& hi) {
    float a[16];
#pragma unroll
    for (int r = 0; r < 16; r++) a[r] = z[r];
    gelu_quarter8(a, lo);
    gelu_quarter8(a + 8, hi);
}

// Fused-layout weights of the four layers: [out tile][K-block][lane][8]
// bf16, times a power-of-two scale (layer 0: 1/4, so that the first
// accumulators hold x / 4; the output layer: 4, as it reads GELU / 4).
// Layer 0 takes its inputs in natural order; later layers in the order the
// previous MFMA output lands in registers. One launch, blockIdx.y = layer.
struct FusedWArgs {
    const float* W[4];
    __bf16* dst[4];
    int out[4], in[4];
};

__global__ void k_fused_weights(FusedWArgs a) {
    const int l = blockIdx.y;
    const int out = a.out[l], in = a.in[l], n_tiles = (out + 31) / 32, n_kb = (in + 15) / 16;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one per (tile, kb, lane)
    if (g >= (int64_t)n_tiles * n_kb * 64) return;
    const float scale = layer_scale(l);
    const float* __restrict__ W = a.W[l];
    const int lane = (int)(g % 64), kb = (int)((g / 64) % n_kb), t = (int)(g / (64 * n_kb));
    const int row = 32 * t + (lane & 31), h = lane >> 5;
    P8 p;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int k = 16 * kb + (l > 0 ? perm_in(h, i) : 8 * h + i);
        p.h[i] = (row < out && k < in) ? (__bf16)(W[(int64_t)row * in + k] * scale) : (__bf16)0.0f;
    }
    ((uint4*)a.dst[l])[g] = p.u;
}

// One hidden layer: in activations act_in [kTiles][2] (bf16x8 per lane),
// weights in LDS (fused layout), out activations gelu(W h + b) into act_out.
// Software-pipelined over the output tiles: the MFMA chain of tile t (16
// K-blocks, weights read from LDS) is interleaved with the GELUs of tile
// t - 1, so that within each wave the vector ALU works while the matrix
// core runs (each MFMA of the chain is followed by about six of the GELUs'
// vector instructions: 96 per tile against 16 MFMAs).
__device__ __forceinline__ void hidden_layer(const uint4* __restrict__ Wl, const float* __restrict__ bias,
                                             const bf16x8 (&act_in)[kTiles][2], bf16x8 (&act_out)[kTiles][2],
                                             int lane) {
    const int h = lane >> 5;
    f32x16 prev;
#pragma unroll
    for (int t = 0; t < kTiles; t++) {
        f32x16 acc = bias_acc(bias, t, h);
#pragma unroll
        for (int kb = 0; kb < kKB; kb++) {
            P8 a;
            a.u = Wl[(t * kKB + kb) * 64 + lane];
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v, act_in[kb >> 1][kb & 1], acc, 0, 0, 0);
        }
        if (t > 0) {
            gelu_tile(prev, act_out[t - 1][0], act_out[t - 1][1]);
#pragma unroll
            for (int kb = 0; kb < kKB; kb++) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
                __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);  // six vector ALU instructions
            }
            pin(act_out[t - 1][0]);
            pin(act_out[t - 1][1]);
        }
        __builtin_amdgcn_sched_barrier(0);
        prev = acc;
    }
    gelu_tile(prev, act_out[kTiles - 1][0], act_out[kTiles - 1][1]);
}

// LLR: store the logits (llr [n][out_dim]); else the GMI cost into part.
// The SNR feature of sample i is (snr_db[i] - 9.5) / 4.5 when snr_db is
// given, else snr_feat.
template <int kWaves, bool LLR>
__global__ __launch_bounds__(kWaves * 64) void k_mlp_fused(
    const uint4* __restrict__ w1f, const uint4* __restrict__ w2f, const uint4* __restrict__ w3f,
    const uint4* __restrict__ w4f, const float* __restrict__ b1, const float* __restrict__ b2,
    const float* __restrict__ b3, const float* __restrict__ b4, int in_dim, int out_dim, const float* __restrict__ y,
    int dim, const uint32_t* __restrict__ tx, const uint32_t* __restrict__ labels, int M, int64_t n,
    const float* __restrict__ snr_db, float snr_feat, float* __restrict__ llr, double* __restrict__ part) {
    constexpr int kThreads = kWaves * 64;
    extern __shared__ uint4 lds[];
    uint4* sW1 = lds;
    uint4* sW4 = sW1 + kW1U;
    float* sB = (float*)(sW4 + kW4U);
    uint4* sWH = (uint4*)(sB + kBiasF);  // kBiasF * 4 bytes is a multiple of 16
    for (int k = threadIdx.x; k < kW1U; k += kThreads) sW1[k] = w1f[k];
    for (int k = threadIdx.x; k < kW4U; k += kThreads) sW4[k] = w4f[k];
    for (int k = threadIdx.x; k < kBiasF; k += kThreads) {
        float v;  // hidden biases / 4: their accumulators hold x / 4
        if (k < kH)
            v = 0.25f * b1[k];
        else if (k < 2 * kH)
            v = 0.25f * b2[k - kH];
        else if (k < 3 * kH)
            v = 0.25f * b3[k - 2 * kH];
        else
            v = (k - 3 * kH) < out_dim ? b4[k - 3 * kH] : 0.0f;
        sB[k] = v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, col = lane & 31;
    CostAcc acc;
    const int64_t nblk = (n + kWaves * 32 - 1) / (kWaves * 32);
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t i = blk * (kWaves * 32) + wave * 32 + col;
        const bool valid = i < n;
        // ---- layer 1: B operand = features in natural order, lane half h holds 8h..8h+7
        bf16x8 xin;
        {
            const float feat = snr_db != nullptr && valid ? (float)(((double)snr_db[i] - 9.5) / 4.5) : snr_feat;
            P8 p;
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int f = 8 * h + q;
                float v = 0.0f;
                if (valid) {
                    if (f < dim)
                        v = y[i * dim + f];
                    else if (f == dim)
                        v = feat;
                }
                p.h[q] = (__bf16)v;
            }
            xin = p.v;
        }
        __syncthreads();  // sW1 / sB staged (first pass) or previous block done with sWH
        bf16x8 actA[kTiles][2], actB[kTiles][2];
#pragma unroll
        for (int ot = 0; ot < kTiles; ot++) {
            P8 a;
            a.u = sW1[ot * 64 + lane];
            const f32x16 z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v, xin, bias_acc(sB, ot, h), 0, 0, 0);
            gelu_tile(z, actA[ot][0], actA[ot][1]);
            __builtin_amdgcn_sched_barrier(0);
        }
        // ---- layer 2
#pragma unroll 4
        for (int k = threadIdx.x; k < kWHU; k += kThreads) sWH[k] = w2f[k];
        __syncthreads();
        hidden_layer(sWH, sB + kH, actA, actB, lane);
        __syncthreads();
        // ---- layer 3
#pragma unroll 4
        for (int k = threadIdx.x; k < kWHU; k += kThreads) sWH[k] = w3f[k];
        __syncthreads();
        hidden_layer(sWH, sB + 2 * kH, actB, actA, lane);
        // ---- layer 4: logits, one output tile of 32 rows
        f32x16 zo = bias_acc(sB + 3 * kH, 0, h);
#pragma unroll
        for (int kb = 0; kb < kKB; kb++) {
            P8 a;
            a.u = sW4[kb * 64 + lane];
            zo = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v, actA[kb >> 1][kb & 1], zo, 0, 0, 0);
        }
        if constexpr (LLR) {
            // registers 4g..4g+3 of lane half h are the consecutive logit
            // rows 8g + 4h .. 8g + 4h + 3: one 16-byte store per group that
            // lies wholly below out_dim (4-byte aligned, as global stores
            // allow), and one store of the 1-3 rows of the group that out_dim
            // cuts, by the lane half that holds it. (Row-by-row conditional
            // stores here led the compiler to a schedule of the hidden layers
            // without the GELU/MFMA interleaving.)
            if (valid) {
                float* dst = llr + i * out_dim;
                typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));
                typedef float f32x3u __attribute__((ext_vector_type(3), aligned(4)));
                typedef float f32x2u __attribute__((ext_vector_type(2), aligned(4)));
#pragma unroll
                for (int g = 0; g < 4; g++) {
                    const int r0 = 8 * g + 4 * h;
                    if (r0 + 4 <= out_dim)
                        *(f32x4u*)(dst + r0) = (f32x4u){zo[4 * g], zo[4 * g + 1], zo[4 * g + 2], zo[4 * g + 3]};
                }
                const int tail = out_dim & 3, rt = out_dim & ~3, gt = rt >> 3;
                if (tail != 0 && ((rt >> 2) & 1) == h) {
                    float t0 = zo[0], t1 = zo[1], t2 = zo[2];
#pragma unroll
                    for (int g = 1; g < 4; g++)
                        if (g == gt) {
                            t0 = zo[4 * g];
                            t1 = zo[4 * g + 1];
                            t2 = zo[4 * g + 2];
                        }
                    if (tail == 3)
                        *(f32x3u*)(dst + rt) = (f32x3u){t0, t1, t2};
                    else if (tail == 2)
                        *(f32x2u*)(dst + rt) = (f32x2u){t0, t1};
                    else
                        dst[rt] = t0;
                }
            }
            continue;
        }
        // ---- per-sample GMI cost of the logits (bits), both lane halves:
        // the sum over rows of max(x, 0) + log2(1 + 2^-|x|), the second part
        // as one logarithm of the product of its factors (each in (1, 2]).
        // In GMI mode out_dim is the format's bit count (<= 12), so rows
        // 0..15, registers 0..7, hold every logit; rows out_dim..15 have zero
        // weights and bias: their logit is exactly 0, their factor exactly 2
        // and their cost exactly one bit, taken off at the end.
        const uint32_t row = valid ? tx[i] : 0u;
        const bool row_ok = row < (uint32_t)M;
        const uint32_t labh = labels[row_ok ? row : 0u] >> (4 * h);
        float mx = 0.0f, prod = 1.0f;
#pragma unroll
        for (int r = 0; r < 8; r++) {
            const float z = zo[r] * 1.4426950408889634f;
            const float xx = ((labh >> (8 * (r >> 2) + (r & 3))) & 1) ? -z : z;
            mx += fmaxf(xx, 0.0f);
            prod *= 1.0f + ex2(-fabsf(xx));
        }
        double c = (double)mx + (double)lg2(prod);
        c += __shfl_xor(c, 32, 64);
        c -= (double)(16 - out_dim);
        if (h == 0 && valid) acc.add(row_ok ? c : NAN, 0.0);
    }
    if constexpr (!LLR) block_reduce_store(acc, part + (size_t)blockIdx.x * kNPart);
}

constexpr size_t kLdsBytes = (size_t)(kW1U + kW4U) * 16 + (size_t)kBiasF * 4 + (size_t)kWHU * 16;

}  // namespace fused

bool fused_shape_ok(const int* sizes, int L) {
    return L == 4 && sizes[0] >= 1 && sizes[0] <= 16 && sizes[1] == fused::kH && sizes[2] == fused::kH &&
           sizes[3] == fused::kH && sizes[4] >= 1 && sizes[4] <= 32;
}

size_t fused_weight_bytes(int layer) {
    using namespace fused;
    return 16 * (size_t)(layer == 0 ? kW1U : layer == 3 ? kW4U : kWHU);
}

hipError_t build_fused_weights(const float* const* W, const int* out, const int* in, __bf16* const* dst,
                               hipStream_t st) {
    using namespace fused;
    FusedWArgs a;
    int64_t most = 0;
    for (int l = 0; l < 4; l++) {
        a.W[l] = W[l];
        a.dst[l] = dst[l];
        a.out[l] = out[l];
        a.in[l] = in[l];
        most = std::max<int64_t>(most, (int64_t)((out[l] + 31) / 32) * ((in[l] + 15) / 16) * 64);
    }
    hipLaunchKernelGGL(k_fused_weights, dim3((unsigned)((most + 255) / 256), 4), dim3(256), 0, st, a);
    return hipGetLastError();
}

int fused_grid() { return device_cu_count(); }

int g_fused_waves = 8;  // 8: two waves per SIMD (256 VGPRs each); 4: one, whole register file

template <int W, bool LLR>
hipError_t launch_fused_w(__bf16* const* wf, const float* const* bias, int in_dim, int out_dim, const float* y, int dim,
                          const uint32_t* tx, const uint32_t* labels, int M, int64_t n, const float* snr_db,
                          float snr_feat, float* llr, double* part, int grid, hipStream_t st) {
    using namespace fused;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_mlp_fused<W, LLR>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_mlp_fused<W, LLR>), dim3(grid), dim3(W * 64), kLdsBytes, st, (const uint4*)wf[0],
                       (const uint4*)wf[1], (const uint4*)wf[2], (const uint4*)wf[3], bias[0], bias[1], bias[2],
                       bias[3], in_dim, out_dim, y, dim, tx, labels, M, n, snr_db, snr_feat, llr, part);
    return hipGetLastError();
}

hipError_t launch_mlp_gmi_fused(__bf16* const* wf, const float* const* bias, int in_dim, int out_dim, const float* y,
                                int dim, const uint32_t* tx, const uint32_t* labels, int M, int64_t n, float snr_feat,
                                double* part, int grid, hipStream_t st) {
    if (out_dim < 1 || out_dim > 16) return hipErrorInvalidValue;  // the GMI cost reads rows 0..15
    if (g_fused_waves == 8)
        return launch_fused_w<8, false>(wf, bias, in_dim, out_dim, y, dim, tx, labels, M, n, nullptr, snr_feat,
                                        nullptr, part, grid, st);
    return launch_fused_w<4, false>(wf, bias, in_dim, out_dim, y, dim, tx, labels, M, n, nullptr, snr_feat, nullptr,
                                    part, grid, st);
}

hipError_t launch_mlp_llr_fused(__bf16* const* wf, const float* const* bias, int in_dim, int out_dim, const float* y,
                                int dim, int64_t n, const float* snr_db, float snr_feat, float* llr, int grid,
                                hipStream_t st) {
    if (g_fused_waves == 4)
        return launch_fused_w<4, true>(wf, bias, in_dim, out_dim, y, dim, nullptr, nullptr, 0, n, snr_db, snr_feat,
                                       llr, nullptr, grid, st);
    return launch_fused_w<8, true>(wf, bias, in_dim, out_dim, y, dim, nullptr, nullptr, 0, n, snr_db, snr_feat, llr,
                                   nullptr, grid, st);
}

}  // namespace mdgmi

extern "C" int mdgmi_mlp_set_fused(int waves) {
    if (waves != 0 && waves != 4 && waves != 8) return MDGMI_E_ARG;
    mdgmi::g_fused_waves = waves;
    return MDGMI_OK;
}
