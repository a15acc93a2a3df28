// Device core of the per-sample 4x4-block MFMA demapper for small
// constellations, shared by the per-SNR kernels (exact_mfma4.hip) and the
// ragged persistent batch (batch.hip).
#pragma once

// The FP32 exact demapper for small constellations (4 <= M <= 512; 8-D up to
// M = 256) with the distance term on the matrix cores and one sample per lane.
//
// v_mfma_f32_4x4x4_16b_f16 evaluates 16 independent 4 x 4 blocks with K = 4:
// lane 4b + i supplies row i of block b's A operand (four halves), lane
// 4b + j column j of its B operand, and lane 4b + j receives column j of the
// block's output, row r in register r. With A = four points (the same four
// in every block, see the broadcast below) and B = the lane's own sample,
// every lane receives u of those four points for its own sample. The class sums of a sample therefore stay inside one lane, as on
// the vector-ALU path, while the matrix cores produce the distance term; the
// 32 x 32 shape (mfma_core.h) spreads a sample over two lanes, whose shared
// per-sample work outweighs the pairs of a small constellation.
//
// The factors are split into an fp16 high part and remainder as in the
// 32 x 32 shape; the k slots of one point (A) and one sample (B) are
//   A [x'h 0..D-1 | x'l 0..D-1 | x'h 0..D-1 | -nh -nl | 0 ...]
//   B [yh  0..D-1 | yh  0..D-1 | yl  0..D-1 |  1   1  | 0 ...]
// in NK = ceil((3D + 2) / 4) MFMAs of K = 4 (2, 2, 4 and 7 for D = 1, 2, 4,
// 8), with the accumulator started at K = kBias - s ||y||^2 in FP32, so the
// output is u_j(y) = kBias - s ||y - x_j||^2 in log2 units (x' = 2 s x,
// n = s ||x||^2).
//
// The A operands of a group reach every block through the MFMA's broadcast
// (CBSZ = 4: block ABID's A rows feed all 16 blocks), so one register holds
// 16 groups: lane 4b + i keeps point 64 t + 4b + i of register set t, and
// group g is the MFMA with ABID = g mod 16 on set g / 16. The whole image is
// ceil(M / 64) sets of NK half4 registers, loaded once per wave.
//
// Class sums: point p of group g sits in register r = p & 3; points come in
// chunks of CH labels (8, or 16 from M = 256), whose low label bits index a running
// bank (one add per pair) and whose totals (one add per pair) carry the
// bits above. Everything is unrolled for the format size, so no per-bit
// work depends on run-time values.
#include <utility>

#include "mfma_core.h"

namespace mdgmi {
namespace small {

using mfma::kSplitF16;
using mfma::split16;
using mfma::split16f;

typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

union H4 {
    half4 v;
    uint2 u;
    _Float16 h[4];
};

constexpr int kSmallThreads = 256;

template <int DIM>
struct Nk4 {
    static constexpr int value = (3 * DIM + 2 + 3) / 4;
};

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Pairwise sum of N values v[OFF], v[OFF + ST], ... (a fixed tree).
template <int N, int ST, int OFF>
__device__ __forceinline__ float tsum(const float* v) {
    if constexpr (N == 1)
        return v[OFF];
    else
        return tsum<N / 2, 2 * ST, OFF>(v) + tsum<N / 2, 2 * ST, OFF + ST>(v);
}

// Class sums of the log2(N) index bits of N values: s0[k] / s1[k] = sum over
// the indices whose bit k is 0 / 1. v is consumed (pair sums replace it).
template <int N>
__device__ __forceinline__ void half_sums(float* v, float* s0, float* s1) {
    if constexpr (N >= 2) {
        s0[0] = tsum<N / 2, 2, 0>(v);
        s1[0] = tsum<N / 2, 2, 1>(v);
#pragma unroll
        for (int r = 0; r < N / 2; r++) v[r] = v[2 * r] + v[2 * r + 1];
        half_sums<N / 2>(v, s0 + 1, s1 + 1);
    }
}

// The same with maxima (exact, order-free).
template <int N>
__device__ __forceinline__ void half_maxes(float* v, float* s0, float* s1) {
    if constexpr (N >= 2) {
        float a = v[0], b = v[1];
#pragma unroll
        for (int r = 2; r < N; r += 2) {
            a = fmaxf(a, v[r]);
            b = fmaxf(b, v[r + 1]);
        }
        s0[0] = a;
        s1[0] = b;
#pragma unroll
        for (int r = 0; r < N / 2; r++) v[r] = fmaxf(v[2 * r], v[2 * r + 1]);
        half_maxes<N / 2>(v, s0 + 1, s1 + 1);
    }
}

// u of the lane's sample against the four points of group ABID of the
// register set a (broadcast from block ABID to every block); the
// accumulator starts at c0 = {K, K, K, K}.
template <int NK, int ABID>
__device__ __forceinline__ f32x4 chain_group(const half4* a, const half4* b, const f32x4& c0) {
    f32x4 c = __builtin_amdgcn_mfma_f32_4x4x4f16(a[0], b[0], c0, 4, ABID, 0);
#pragma unroll
    for (int k = 1; k < NK; k++) c = __builtin_amdgcn_mfma_f32_4x4x4f16(a[k], b[k], c, 4, ABID, 0);
    return c;
}

// u of the lane's sample against the point whose A operands the lane itself
// supplies (no broadcast): register l & 3 of the result.
template <int NK>
__device__ __forceinline__ f32x4 chain_own(const half4* a, const half4* b, const f32x4& c0) {
    f32x4 c = __builtin_amdgcn_mfma_f32_4x4x4f16(a[0], b[0], c0, 0, 0, 0);
#pragma unroll
    for (int k = 1; k < NK; k++) c = __builtin_amdgcn_mfma_f32_4x4x4f16(a[k], b[k], c, 0, 0, 0);
    return c;
}

// f(std::integral_constant<int, 0>) ... f(std::integral_constant<int, N - 1>)
// in order: the group walk is unrolled by construction, so every group
// index (ABID, register set, bank slot) is a compile-time constant however
// large the format.
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <int NG>
struct Sets {
    static constexpr int value = (NG + 15) / 16;
};

// A operands of point slot j (label order) at scale s: NK half4 at dst.
template <int DIM>
__device__ inline void image_slot(const double* __restrict__ X64, double s, int j, uint2* __restrict__ dst) {
    constexpr int NK = Nk4<DIM>::value;
    _Float16 p[4 * NK];
#pragma unroll
    for (int k = 0; k < 4 * NK; k++) p[k] = (_Float16)0.0f;
    double n2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; d++) {
        const double x = X64[(size_t)j * DIM + d];
        n2 += x * x;
        _Float16 xh, xl;
        split16(2.0 * s * x, xh, xl);
        p[d] = xh;
        p[DIM + d] = xl;
        p[2 * DIM + d] = xh;
    }
    _Float16 nh, nl;
    split16(s * n2, nh, nl);
    p[3 * DIM] = -nh;
    p[3 * DIM + 1] = -nl;
#pragma unroll
    for (int k = 0; k < NK; k++) {
        H4 v;
#pragma unroll
        for (int i = 0; i < 4; i++) v.h[i] = p[4 * k + i];
        dst[k] = v.u;
    }
}

// The wave's A operand registers: lane l holds point 64 t + l of set t
// (zero past M).
template <int DIM, int NG>
__device__ __forceinline__ void load_image(const uint2* __restrict__ gimg, int M,
                                           half4 (&a)[(NG + 15) / 16][Nk4<DIM>::value]) {
    constexpr int NK = Nk4<DIM>::value;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int t = 0; t < (NG + 15) / 16; t++) {
        const int p = 64 * t + lane;  // lane 4b + i: point 4 (16 t + b) + i
#pragma unroll
        for (int k = 0; k < NK; k++) {
            H4 v;
            v.u = p < M ? gimg[(size_t)p * NK + k] : make_uint2(0u, 0u);
            a[t][k] = v.v;
        }
    }
}

// One sample per lane (all 64 lanes call it: the MFMAs need every lane;
// lanes past n run on y = 0 and store nothing).
template <int DIM, int NG, int MODE>
__device__ __forceinline__ void small_sample(const half4 (&a)[Sets<NG>::value][Nk4<DIM>::value],
                                             const uint2* __restrict__ gimg,
                                             const float* __restrict__ ys, const uint32_t* __restrict__ txs,
                                             int64_t i, int64_t n, float s, const float* __restrict__ X32,
                                             const uint32_t* __restrict__ labels, float* __restrict__ llr,
                                             CostAcc& acc, HdAcc& hd, float guard = 0.0f) {
    constexpr int NK = Nk4<DIM>::value;
    constexpr int M = 4 * NG, m = ilog2(M);
    // chunk size near sqrt(M): the bank adds, the chunk totals and the two
    // final class-sum folds cost least (140 adds per sample at M = 64
    // against 148 with chunks of 16)
    constexpr int CH = M <= 128 ? (M < 8 ? M : 8) : 16, CHB = ilog2(CH), NC = M / CH, GPC = CH / 4;
    constexpr bool ML = mode_is_ml(MODE), HD = MODE == kModeHd;
    const int lane = threadIdx.x & 63;
    const bool valid = i < n;
    // lanes past n read the last sample (no branch around the loads) and
    // then work on y = 0
    const int64_t ic = valid ? i : n - 1;
    float yv[DIM], ys2 = 0.0f;
#pragma unroll
    for (int d = 0; d < DIM; d++) {
        const float v = ys[ic * DIM + d];
        yv[d] = valid ? v : 0.0f;
        ys2 = fmaf(yv[d], yv[d], ys2);
    }
    // y beyond the fp16 range of its split (or not finite) takes the FP32
    // per-class path below
    const bool ybad = !(ys2 < 1.0e9f);
    const float K = fmaf(-s, ys2, kBias);
    half4 bo[NK];
    {
        _Float16 yh[DIM], yl[DIM];
#pragma unroll
        for (int d = 0; d < DIM; d++) split16f(yv[d], yh[d], yl[d]);
        _Float16 b[4 * NK];
#pragma unroll
        for (int k = 0; k < 4 * NK; k++) b[k] = (_Float16)0.0f;
#pragma unroll
        for (int d = 0; d < DIM; d++) {
            b[d] = yh[d];
            b[DIM + d] = yh[d];
            b[2 * DIM + d] = yl[d];
        }
        b[3 * DIM] = (_Float16)1.0f;
        b[3 * DIM + 1] = (_Float16)1.0f;
#pragma unroll
        for (int k = 0; k < NK; k++) bo[k] = (half4){b[4 * k], b[4 * k + 1], b[4 * k + 2], b[4 * k + 3]};
    }
    float bank[CH], T[NC];
    float umax = -INFINITY;
    // the sent point's row and label are fetched before the walk, its A
    // operands halfway through it, so that their latency hides behind the
    // exponentials
    constexpr bool SENT = !mode_is_llr(MODE) && !ML;
    uint32_t row = 0u, slot = 0u;
    bool twin = false;  // hard decisions: a lower label shares the sent point
    if (SENT) {
        const uint32_t r = txs[ic];
        row = valid ? r : 0u;
        const uint32_t lw = labels[row < (uint32_t)M ? row : 0u];
        slot = lw & kLabelMask;
        twin = HD && (lw & kTwinBit) != 0u;
    }
    half4 ad[NK];
    // Kc = {K, K, K, K}, passed through an empty asm after each group so that
    // the MFMAs of group g + 2 cannot be hoisted above the exponentials of
    // group g: one group of lookahead, not every group's u held in registers
    // at once. The same four registers seed every chain.
    f32x4 Kc = {K, K, K, K};
    f32x4 nxt = chain_group<NK, 0>(a[0], bo, Kc);
    static_for<NG>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        const f32x4 u = nxt;
        if constexpr (g + 1 < NG) nxt = chain_group<NK, (g + 1) % 16>(a[(g + 1) / 16], bo, Kc);
        if constexpr (SENT && g == NG / 2) {
#pragma unroll
            for (int k = 0; k < NK; k++) {
                H4 v;
                v.u = gimg[(size_t)slot * NK + k];
                ad[k] = v.v;
            }
        }
        constexpr int c = g / GPC, r0 = 4 * (g % GPC);
        constexpr bool first = g % GPC == 0;
        if constexpr (ML) {
#pragma unroll
            for (int r = 0; r < 4; r++) bank[r0 + r] = c == 0 ? u[r] : fmaxf(bank[r0 + r], u[r]);
            if constexpr (NC > 1) {
                const float gm = fmaxf(fmaxf(u[0], u[1]), fmaxf(u[2], u[3]));
                T[c] = first ? gm : fmaxf(T[c], gm);
            }
        } else {
            if constexpr (HD) umax = fmaxf(fmaxf(umax, fmaxf(u[0], u[1])), fmaxf(u[2], u[3]));
            float e[4];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                e[r] = ex2(u[r]);
                bank[r0 + r] = c == 0 ? e[r] : bank[r0 + r] + e[r];
            }
            if constexpr (NC > 1) {
                const float gs = (e[0] + e[1]) + (e[2] + e[3]);
                T[c] = first ? gs : T[c] + gs;
            }
        }
        // every value this group produced goes into the barrier, so that
        // none of its exponentials (and with them its u) is sunk to the end
        asm volatile("" : "+v"(Kc) : "v"(bank[r0]), "v"(bank[r0 + 1]), "v"(bank[r0 + 2]), "v"(bank[r0 + 3]),
                     "v"(NC > 1 ? T[c] : 0.0f), "v"(umax));
        __builtin_amdgcn_sched_barrier(0);
    });
    // per-bit class sums (or maxima): bits below CHB from the bank, the
    // rest from the chunk totals
    float S0[m], S1[m];
    if constexpr (ML) {
        half_maxes<CH>(bank, S0, S1);
        if constexpr (NC > 1) half_maxes<NC>(T, S0 + CHB, S1 + CHB);
    } else {
        half_sums<CH>(bank, S0, S1);
        if constexpr (NC > 1) half_sums<NC>(T, S0 + CHB, S1 + CHB);
    }
    if constexpr (ML) {
        const float best = fmaxf(S0[0], S1[0]);
        bool finite = true;
#pragma unroll
        for (int d = 0; d < DIM; d++) finite = finite && __builtin_isfinite(yv[d]);
        float u0[MDGMI_MAX_BITS], u1[MDGMI_MAX_BITS];
#pragma unroll
        for (int k = 0; k < m; k++) {
            u0[k] = S0[k];
            u1[k] = S1[k];
        }
        bool redo = !(best >= kFarLog2) || ybad;
        if (MODE == kModeMlLlr) {
#pragma unroll
            for (int k = 0; k < m; k++) redo = redo || fabsf(u1[k] - u0[k]) < guard;
        }
        if (redo) class_max_u_f32<DIM>(yv, X32, M, m, s, u0, u1);
        if (!valid) return;
        if (MODE == kModeMlLlr) {
#pragma unroll
            for (int k = 0; k < m; k++) llr[i * m + k] = finite ? (u1[k] - u0[k]) * (float)kLn2 : NAN;
        } else {
            const uint32_t row = txs[i];
            const bool row_ok = row < (uint32_t)M;
            const uint32_t slot = labels[row_ok ? row : 0u];
            float cg = 0.0f;
#pragma unroll
            for (int k = 0; k < m; k++) {
                const bool bk = (slot >> k) & 1;
                cg += bit_cost2(bk ? u0[k] - u1[k] : u1[k] - u0[k]);
            }
            acc.add(row_ok && finite ? cg : NAN, 0.0f);
        }
        return;
    }
    if constexpr (MODE == kModeLlr) {
        float smin = INFINITY;
        float out[m];
#pragma unroll
        for (int k = 0; k < m; k++) {
            smin = fminf(smin, fminf(S0[k], S1[k]));
            out[k] = log2_ratio_fast(S1[k], S0[k]);
        }
        // a class too far for the common offset, y out of range, or (guard)
        // an LLR near zero at a large s
        bool redo = !(smin >= ex2(kFarLog2)) || ybad;
#pragma unroll
        for (int k = 0; k < m; k++) redo = redo || fabsf(out[k]) < guard;
        if (redo) {
            float ls0[MDGMI_MAX_BITS], ls1[MDGMI_MAX_BITS], ltot, ti;
            exact_classes_f32<DIM>(yv, X32, M, m, s, -1, ls0, ls1, ltot, ti);
#pragma unroll
            for (int k = 0; k < m; k++) out[k] = ls1[k] - ls0[k];
        }
        if (valid) {
#pragma unroll
            for (int k = 0; k < m; k++) llr[i * m + k] = out[k] * (float)kLn2;
        }
        return;
    }
    const float tot = S0[0] + S1[0];
    // a sent row outside [0, M) gives a NaN cost instead of a stray read
    const bool row_ok = row < (uint32_t)M;
    // u of the sent point from the same MFMA arithmetic: the lane supplies
    // its own sent point as A row l & 3 of its block, so register l & 3 of
    // the output is u_i(y), bit-identical to the value inside the class sums
    // (a broadcast MFMA and a plain one form element (i, j) alike)
    const f32x4 ud = chain_own<NK>(ad, bo, Kc);
    const bool q1 = lane & 1, q2 = lane & 2;
    const float ui = q2 ? (q1 ? ud[3] : ud[2]) : (q1 ? ud[1] : ud[0]);
    // GMI cost sum_k log2(T / S_sent,k) as one logarithm of the product of
    // S_sent,k / T (cost_from_product); bit by bit where a sample of the
    // wave has a cost beyond 120 bits or a non-finite sum
    float cg = 0.0f, cm, be = 0.0f, sym, prod = 1.0f;
    const float rT = __builtin_amdgcn_rcpf(tot);
#pragma unroll
    for (int k = 0; k < m; k++) {
        const bool bk = (slot >> k) & 1;
        prod *= (bk ? S1[k] : S0[k]) * rT;
        if (HD) be += (S1[k] > S0[k]) != bk ? 1.0f : 0.0f;  // bitwise MAP decision
    }
    if (__ballot(!(prod >= 0x1p-120f)) == 0ull) {
        cost_from_product(prod, cg);
    } else {
        asm volatile("" ::: "memory");  // keeps the rare path a real branch
#pragma unroll
        for (int k = 0; k < m; k++) cg += bit_cost_sum2(S0[k] + S1[k], ((slot >> k) & 1) ? S1[k] : S0[k]);
    }
    // another point strictly nearer, or the sent point's coordinates shared
    // with a lower label (ties go to the lowest label)
    sym = umax > ui || twin ? 1.0f : 0.0f;
    if (ui >= kFarLog2 && !ybad) {
        cm = mi_cost2(tot, ui);
    } else {
        // the sent point itself is far from y (or y is out of range)
        float ls0[MDGMI_MAX_BITS], ls1[MDGMI_MAX_BITS], ltot, ti = 0.0f, tmin = 0.0f;
        exact_classes_f32<DIM>(yv, X32, M, m, s, (int)slot, ls0, ls1, ltot, ti, HD ? &tmin : nullptr);
        cg = 0.0f;
        be = 0.0f;
        if (HD) sym = tmin < ti || twin ? 1.0f : 0.0f;
#pragma unroll
        for (int k = 0; k < m; k++) {
            const bool bk = (slot >> k) & 1;
            cg += bit_cost2(bk ? ls0[k] - ls1[k] : ls1[k] - ls0[k]);
            if (HD) be += (ls1[k] > ls0[k]) != bk ? 1.0f : 0.0f;
        }
        cm = ltot + ti;
    }
    if (!valid) return;
    if (!row_ok) cg = cm = NAN;
    acc.add(cg, cm);
    if (HD) {
        const bool finite = cg == cg && cm == cm && ui == ui;
        hd.be += finite ? (double)be : (double)m;
        hd.se += finite ? (double)sym : 1.0;
    }
}

}  // namespace small
}  // namespace mdgmi
