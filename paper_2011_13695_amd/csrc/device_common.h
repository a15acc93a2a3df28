// Device helpers shared by the demapper kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace mdgmi {

// v_exp_f32 / v_log_f32: base-2 transcendentals of the vector ALU.
__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float lg2(float x) { return __builtin_amdgcn_logf(x); }

// log2(1 + 2^x) for every x (base-2 softplus).
__device__ __forceinline__ float softplus2(float x) {
    return fmaxf(x, 0.0f) + lg2(1.0f + ex2(-fabsf(x)));
}

// log2(Sa / Sb) of two class sums, given also lsa = log2 Sa, lsb = log2 Sb.
// Both logarithms are near the common offset (~kBias), so their difference
// loses ~1e-5 to cancellation; the ratio form keeps full FP32 accuracy and is
// used whenever the ratio stays well inside the float range. Sb = 0 gives
// +inf, Sa = 0 gives -inf, NaN propagates.
__device__ __forceinline__ float log2_ratio(float Sa, float Sb, float lsa, float lsb) {
    const float d = lsa - lsb;
    if (fabsf(d) < 60.0f) return lg2(Sa * __builtin_amdgcn_rcpf(Sb));
    return d;
}

// log2(Sa / Sb) from the ratio alone while it stays within 2^+-60 (the
// usual case: one reciprocal and one logarithm), else as a difference of
// logarithms. Sb = 0 gives +inf, Sa = 0 gives -inf, NaN propagates.
// The rare branch is entered only when one of the wave's active lanes needs
// it (a wave vote), so the common case issues one reciprocal and one
// logarithm.
__device__ __forceinline__ float log2_ratio_fast(float Sa, float Sb) {
    const float r = Sa * __builtin_amdgcn_rcpf(Sb);
    const bool ok = r > 0x1p-60f && r < 0x1p60f;
    float v = lg2(r);
    if (__ballot(!ok) != 0ull) {
        asm volatile("" ::: "memory");  // keeps the rare path a real branch
        if (!ok) v = lg2(Sa) - lg2(Sb);
    }
    return v;
}

// Base-2 GMI cost of one bit from the class sums: log2(1 + S_other / S_sent)
// = log2(tot / S_sent) with tot = S_sent + S_other >= S_sent; the ratio form
// keeps full FP32 accuracy near zero cost, the difference of logarithms
// takes over for costs beyond 60 bits (and propagates NaN).
__device__ __forceinline__ float bit_cost_sum2(float tot, float Ssent) {
    const float r = tot * __builtin_amdgcn_rcpf(Ssent);
    const bool ok = r < 0x1p60f;
    float v = fmaxf(lg2(r), 0.0f);
    if (__ballot(!ok) != 0ull) {
        asm volatile("" ::: "memory");  // keeps the rare path a real branch
        if (!ok) v = lg2(tot) - lg2(Ssent);
    }
    return v;
}

// MI cost log2(sum_j 2^(u_j - u_i)) = log2(tot * 2^-u_i) without the
// cancellation of log2(tot) - u_i: the integer part of u_i is removed exactly
// with ldexp first. tot >= 2^u_i always (the sent point is in the sum).
__device__ __forceinline__ float mi_cost2(float tot, float ui) {
    const float d = lg2(tot) - ui;
    if (d < 60.0f) {
        const float fl = floorf(ui);
        return lg2(ldexpf(tot, -(int)fl)) - (ui - fl);
    }
    return d;
}

// Base-2 GMI cost of one bit, log2(1 + S_nb / S_b), from x = log2(S_nb / S_b).
// S_nb = 0 gives x = -inf and cost 0; NaN propagates.
__device__ __forceinline__ float bit_cost2(float x) { return softplus2(x); }

// Class sums of the label bits above a group of G = 1, 2, 4 or 8 consecutive
// blocks of points (a block is a chunk of consecutive labels; the block
// index supplies these bits). Inside a group the lowest log2(G) block-index
// bits are known at compile time; the bits above come from the group index
// and are applied without branches: each group total is added to the class
// of each such bit through an FMA with a 0/1 factor formed in scalar
// registers. Unused high bits accumulate values that are never read.
template <int G, int MAXHI>
struct HiAcc {
    static constexpr int GB = G == 8 ? 3 : (G == 4 ? 2 : (G == 2 ? 1 : 0));
    float R0[MAXHI > 0 ? MAXHI : 1], R1[MAXHI > 0 ? MAXHI : 1];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int l = 0; l < (MAXHI > 0 ? MAXHI : 1); l++) R0[l] = R1[l] = 0.0f;
    }
    // T[i]: total of block G*grp + i.
    __device__ __forceinline__ void add_group(int grp, const float* T) {
        if (G == 1 || MAXHI == 0) return;
        float GT;
        if (G == 2) {
            R0[0] += T[0];
            R1[0] += T[1];
            GT = T[0] + T[1];
        } else if (G == 4) {
            R0[0] += T[0] + T[2];
            R1[0] += T[1] + T[3];
            const float a = T[0] + T[1], b = T[2] + T[3];
            R0[1] += a;
            R1[1] += b;
            GT = a + b;
        } else {
            R0[0] += (T[0] + T[2]) + (T[4] + T[6]);
            R1[0] += (T[1] + T[3]) + (T[5] + T[7]);
            const float a0 = T[0] + T[1], a1 = T[2] + T[3], a2 = T[4] + T[5], a3 = T[6] + T[7];
            R0[1] += a0 + a2;
            R1[1] += a1 + a3;
            const float q0 = a0 + a1, q1 = a2 + a3;
            R0[2] += q0;
            R1[2] += q1;
            GT = q0 + q1;
        }
#pragma unroll
        for (int l = GB; l < MAXHI; l++) {
            const uint32_t bit = ((uint32_t)grp >> (l - GB)) & 1u;
            const float one_if = __uint_as_float(bit * 0x3f800000u);
            const float one_ifn = __uint_as_float((bit ^ 1u) * 0x3f800000u);
            R1[l] = fmaf(GT, one_if, R1[l]);
            R0[l] = fmaf(GT, one_ifn, R0[l]);
        }
    }
};

// The max counterpart of HiAcc for max-log metrics: per tile-index bit l,
// R0[l] / R1[l] = largest u over the tiles whose bit l is 0 / 1, from the
// tile maxima T of G consecutive tiles at a time. Max is exact, so the
// grouping does not change any value.
template <int G, int MAXHI>
struct HiMax {
    static constexpr int GB = G == 8 ? 3 : (G == 4 ? 2 : (G == 2 ? 1 : 0));
    float R0[MAXHI > 0 ? MAXHI : 1], R1[MAXHI > 0 ? MAXHI : 1];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int l = 0; l < (MAXHI > 0 ? MAXHI : 1); l++) R0[l] = R1[l] = -INFINITY;
    }
    __device__ __forceinline__ void add_group(int grp, const float* T) {
        if (G == 1 || MAXHI == 0) return;
        float GT;
        if (G == 2) {
            R0[0] = fmaxf(R0[0], T[0]);
            R1[0] = fmaxf(R1[0], T[1]);
            GT = fmaxf(T[0], T[1]);
        } else if (G == 4) {
            R0[0] = fmaxf(R0[0], fmaxf(T[0], T[2]));
            R1[0] = fmaxf(R1[0], fmaxf(T[1], T[3]));
            const float a = fmaxf(T[0], T[1]), b = fmaxf(T[2], T[3]);
            R0[1] = fmaxf(R0[1], a);
            R1[1] = fmaxf(R1[1], b);
            GT = fmaxf(a, b);
        } else {
            R0[0] = fmaxf(R0[0], fmaxf(fmaxf(T[0], T[2]), fmaxf(T[4], T[6])));
            R1[0] = fmaxf(R1[0], fmaxf(fmaxf(T[1], T[3]), fmaxf(T[5], T[7])));
            const float a0 = fmaxf(T[0], T[1]), a1 = fmaxf(T[2], T[3]);
            const float a2 = fmaxf(T[4], T[5]), a3 = fmaxf(T[6], T[7]);
            R0[1] = fmaxf(R0[1], fmaxf(a0, a2));
            R1[1] = fmaxf(R1[1], fmaxf(a1, a3));
            const float q0 = fmaxf(a0, a1), q1 = fmaxf(a2, a3);
            R0[2] = fmaxf(R0[2], q0);
            R1[2] = fmaxf(R1[2], q1);
            GT = fmaxf(q0, q1);
        }
#pragma unroll
        for (int l = GB; l < MAXHI; l++) {
            // grp is uniform over the wave: a scalar branch
            if (((uint32_t)grp >> (l - GB)) & 1u)
                R1[l] = fmaxf(R1[l], GT);
            else
                R0[l] = fmaxf(R0[l], GT);
        }
    }
};

// Per-lane FP64 accumulators of the Monte-Carlo sums.
struct CostAcc {
    double sg = 0.0, sg2 = 0.0, sm = 0.0, sm2 = 0.0, bad = 0.0;
    __device__ __forceinline__ void add(double cg, double cm) {
        sg += cg;
        sg2 += cg * cg;
        sm += cm;
        sm2 += cm * cm;
        // a class test, not x - x == 0: contraction may turn x - x into
        // fma(a, b, -x) when x = a * b, which is the product's rounding error
        const bool fin = __builtin_isfinite(cg) && __builtin_isfinite(cm);
        bad += fin ? 0.0 : 1.0;
    }
};

// Sum over the bits of log2(T / S_k), the GMI cost of a sample (T the total
// of all its terms, S_k the class sum of sent bit k), as -log2(prod_k S_k / T):
// one reciprocal of T, one product per bit, one logarithm. Each factor is in
// (0, 1] up to rounding; while the product stays at least 2^-120 (a cost
// below 120 bits) it is a normal FP32 number and the result is exact to
// rounding. Returns false (cost untouched) when it is not, or not finite:
// the caller then takes the per-bit form.
__device__ __forceinline__ bool cost_from_product(float prod, float& cost) {
    const bool ok = prod >= 0x1p-120f;
    if (ok) cost = fmaxf(-__builtin_amdgcn_logf(prod), 0.0f);
    return ok;
}

// Per-lane hard-decision error counts (bits, symbols), kept as doubles.
struct HdAcc {
    double be = 0.0, se = 0.0;
};

// Fixed-order reduction of NP partials over a block; thread 0 writes them to
// dst[0..NP-1]. The shuffle tree and the per-wave order are fixed, so the
// result does not depend on scheduling.
template <int NP>
__device__ inline void block_reduce_vals(double (&v)[NP], double* dst) {
    __shared__ double red[16][NP];
#pragma unroll
    for (int q = 0; q < NP; q++) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[q] += __shfl_down(v[q], off, 64);
    }
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NP; q++) red[wave][q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int nw = (blockDim.x + 63) >> 6;
        for (int q = 0; q < NP; q++) {
            double s = 0.0;
            for (int w = 0; w < nw; w++) s += red[w][q];
            dst[q] = s;
        }
    }
}

__device__ inline void block_reduce_store(CostAcc a, double* dst) {
    double v[kNPart] = {a.sg, a.sg2, a.sm, a.sm2, a.bad};
    block_reduce_vals<kNPart>(v, dst);
}

__device__ inline void block_reduce_store_hd(CostAcc a, HdAcc h, double* dst) {
    double v[kNPartHd] = {a.sg, a.sg2, a.sm, a.sm2, a.bad, h.be, h.se};
    block_reduce_vals<kNPartHd>(v, dst);
}

// Distance terms relative to a reference point, from the factored difference
//   ||y - x_j||^2 - ||y - x_r||^2 = (x_r - x_j) . (2y - x_r - x_j),
// whose error is relative to the difference itself: a difference of two
// squared distances of size ||y||^2 loses everything once ||y|| is large
// (|y| ~ 5e4: ||y||^2 ~ 1e10, FP32 spacing ~ 1e3), the factored form keeps
// about 1e-7 of each term. y2 = 2y.
template <int DIM>
__device__ inline float rel_dist(const float* y2, const float* __restrict__ xr, const float* __restrict__ xj) {
#pragma clang fp contract(off)
    float d = 0.0f;
#pragma unroll
    for (int q = 0; q < DIM; q++) d = fmaf(xr[q] - xj[q], (y2[q] - xr[q]) - xj[q], d);
    return d;
}

// Label slot of the point nearest to y (FP32; ties and near-ties within
// rounding go to either point).
template <int DIM>
__device__ inline int nearest_slot(const float* y2, const float* __restrict__ X32, int M) {
    int r = 0;
    float best = 0.0f;  // relative to slot 0
#pragma unroll 2
    for (int j = 1; j < M; j++) {
        const float d = rel_dist<DIM>(y2, X32, X32 + j * DIM);
        if (d < best) {
            best = d;
            r = j;
        }
    }
    return r;
}

// Exact per-class evaluation of one sample in FP32, used when a class sum
// taken relative to the common offset could have lost terms to underflow
// (a class more than about 2*kBias log2-units away from y) or when the sent
// point itself is that far. Each class gets its own reference: its nearest
// point. t_j = s (||y - x_j||^2 - ||y - x_r||^2) in log2 units relative to
// the point r nearest to y, from the factored difference (rel_dist), so an
// LLR (the difference of two class minima, one of them t_r = 0) keeps FP32
// relative accuracy at any distance of y. Every output is relative to t_r;
// callers use differences only.
// Outputs: lsb[k] = log2 sum_{j in class(k,b)} 2^-t_j  (k < m, b = 0, 1),
//          ltot = log2 sum_j 2^-t_j,  ti = t of slot `sent` (if sent >= 0),
//          tmin = min_j t_j.
// t_j must stay a rounded product: contracted into fma(-s, d, cmin),
// cmin - t_j of the nearest point would be the product's rounding error
// instead of 0. Contraction is therefore off in these per-class paths.
template <int DIM>
__device__ inline void exact_classes_f32(const float* yv, const float* __restrict__ X32, int M, int m,
                                         float s, int sent, float* ls0, float* ls1, float& ltot, float& ti,
                                         float* tmin_out = nullptr) {
#pragma clang fp contract(off)
    float y2[DIM];
#pragma unroll
    for (int q = 0; q < DIM; q++) y2[q] = 2.0f * yv[q];
    const float* xr = X32 + nearest_slot<DIM>(y2, X32, M) * DIM;
    float cmin0[MDGMI_MAX_BITS], cmin1[MDGMI_MAX_BITS];
    float tmin = INFINITY;
#pragma unroll
    for (int k = 0; k < MDGMI_MAX_BITS; k++) cmin0[k] = cmin1[k] = INFINITY;
#pragma unroll 2
    for (int j = 0; j < M; j++) {
        const float t = s * rel_dist<DIM>(y2, xr, X32 + j * DIM);
        tmin = fminf(tmin, t);
#pragma unroll
        for (int k = 0; k < MDGMI_MAX_BITS; k++) {
            if (k < m) {
                if ((j >> k) & 1)
                    cmin1[k] = fminf(cmin1[k], t);
                else
                    cmin0[k] = fminf(cmin0[k], t);
            }
        }
        if (j == sent) ti = t;
    }
    float S0[MDGMI_MAX_BITS], S1[MDGMI_MAX_BITS];
    float tot = 0.0f;
#pragma unroll
    for (int k = 0; k < MDGMI_MAX_BITS; k++) S0[k] = S1[k] = 0.0f;
#pragma unroll 2
    for (int j = 0; j < M; j++) {
        const float t = s * rel_dist<DIM>(y2, xr, X32 + j * DIM);
        tot += ex2(tmin - t);
#pragma unroll
        for (int k = 0; k < MDGMI_MAX_BITS; k++) {
            if (k < m) {
                if ((j >> k) & 1)
                    S1[k] += ex2(cmin1[k] - t);
                else
                    S0[k] += ex2(cmin0[k] - t);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < MDGMI_MAX_BITS; k++) {
        if (k < m) {
            ls0[k] = lg2(S0[k]) - cmin0[k];
            ls1[k] = lg2(S1[k]) - cmin1[k];
        }
    }
    ltot = lg2(tot) - tmin;
    if (tmin_out) *tmin_out = tmin;
}

// Max-log fallback in FP32 for one sample: per bit, the log2 metric of the
// nearest point of each class, u0[k] = -min_{j: bit k = 0} t_j and
// u1[k] = -min_{j: bit k = 1} t_j, with t_j relative to the point nearest
// to y from the factored difference (accurate at any distance; X32 in label
// order). Callers use differences only.
template <int DIM>
__device__ inline void class_max_u_f32(const float* yv, const float* __restrict__ X32, int M, int m, float s,
                                       float* u0, float* u1) {
#pragma clang fp contract(off)
    float y2[DIM];
#pragma unroll
    for (int q = 0; q < DIM; q++) y2[q] = 2.0f * yv[q];
    const float* xr = X32 + nearest_slot<DIM>(y2, X32, M) * DIM;
#pragma unroll
    for (int k = 0; k < MDGMI_MAX_BITS; k++) u0[k] = u1[k] = -INFINITY;
#pragma unroll 2
    for (int j = 0; j < M; j++) {
        const float u = -(s * rel_dist<DIM>(y2, xr, X32 + j * DIM));
#pragma unroll
        for (int k = 0; k < MDGMI_MAX_BITS; k++) {
            if (k < m) {
                if ((j >> k) & 1)
                    u1[k] = fmaxf(u1[k], u);
                else
                    u0[k] = fmaxf(u0[k], u);
            }
        }
    }
}

}  // namespace mdgmi
