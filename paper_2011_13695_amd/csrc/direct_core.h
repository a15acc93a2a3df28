// Device core of the FP32 direct exact demapper, shared by the per-SNR
// kernels (exact_direct.hip) and the ragged persistent batch (batch.hip).
#pragma once

// The distance term on the vector ALUs.
//
// One lane per sample; the constellation is walked in label order through
// uniform (scalar) loads of a per-SNR image {2 s x_j, s ||x_j||^2}, with
// s = log2(e) / (2 sigma2), so that
//     u_j = kBias - s ||y - x_j||^2 = K + <2 s x_j, y> - s ||x_j||^2,
//     K   = kBias - s ||y||^2,
// costs DIM fused multiply-adds plus one add per (sample, point), followed by
// one v_exp_f32: e_j = 2^u_j.
//
// Class sums without per-bit work: points come in chunks of CH = 2^CHB
// consecutive labels. Inside a chunk the low CHB label bits are the
// position r, so e_j is added to a running bank[r] (one add); the chunk total
// (CH - 1 adds) is added once per chunk to the class of every higher label
// bit. Class sums of the low bits are formed from the banks at the end.
#include "device_common.h"

namespace mdgmi {
namespace direct {

template <int DIM>
struct DirectRec {
    static constexpr int value = ((DIM + 1 + 3) / 4) * 4;  // floats per point record
};

// Record of point j in a direct image: {2 s x_j (dim floats), s ||x_j||^2, 0...}.
__device__ inline void direct_record(const double* __restrict__ X64, int dim, int rec, double s, int j,
                                     float* __restrict__ r) {
    double n2 = 0.0;
    for (int d = 0; d < dim; d++) {
        double x = X64[(size_t)j * dim + d];
        n2 += x * x;
        r[d] = (float)(2.0 * s * x);
    }
    r[dim] = (float)(s * n2);
    for (int d = dim + 1; d < rec; d++) r[d] = 0.0f;
}

// One sample (index i of one (format, SNR) instance) against all M points of
// the instance's direct image im (records {2 s x_j, s ||x_j||^2}).
// MODE: kModeGmi (costs into acc), kModeLlr (LLRs into llr) or kModeHd
// (costs and hard-decision error counts into hd).
template <int DIM, int CHB, int G, int MODE>
__device__ __forceinline__ void direct_sample(const float* __restrict__ im, const float* __restrict__ ys,
                                              const uint32_t* __restrict__ txs, int64_t i, int M, int m,
                                              float s, const float* __restrict__ X32,
                                              const uint32_t* __restrict__ labels, float* __restrict__ llr,
                                              CostAcc& acc, HdAcc* hd = nullptr, float guard = 0.0f) {
    constexpr bool LLR = MODE == kModeLlr;
    constexpr int CH = 1 << CHB;
    constexpr int REC = DirectRec<DIM>::value;
    constexpr int MAXHI = MDGMI_MAX_BITS - CHB;
    const int nchunk = M >> CHB;
    float yv[DIM];
    float ys2 = 0.0f;
#pragma unroll
    for (int q = 0; q < DIM; q++) {
        yv[q] = ys[i * DIM + q];
        ys2 = fmaf(yv[q], yv[q], ys2);
    }
    const float K = kBias - s * ys2;
    float bank[CH];
#pragma unroll
    for (int r = 0; r < CH; r++) bank[r] = 0.0f;
    HiAcc<G, MAXHI> hi;
    hi.zero();
    float umax = -INFINITY;  // nearest point (hard decisions only)
    for (int c0 = 0; c0 < nchunk; c0 += G) {
        float T[G];
#pragma unroll
        for (int i = 0; i < G; i++) {
            const float* __restrict__ rc = im + (size_t)(c0 + i) * CH * REC;
            float ev[CH];
#pragma unroll
            for (int r = 0; r < CH; r++) {
                float u = K - rc[r * REC + DIM];
#pragma unroll
                for (int q = 0; q < DIM; q++) u = fmaf(rc[r * REC + q], yv[q], u);
                if (MODE == kModeHd) umax = fmaxf(umax, u);
                ev[r] = ex2(u);
                bank[r] += ev[r];
            }
            if (G > 1) {
#pragma unroll
                for (int w = 1; w < CH; w <<= 1) {
#pragma unroll
                    for (int r = 0; r < CH; r += 2 * w) ev[r] += ev[r + w];
                }
                T[i] = ev[0];
            }
        }
        hi.add_group(c0 / G, T);
    }
    // log2 class sums (relative to the common offset kBias)
    float ls0[MDGMI_MAX_BITS], ls1[MDGMI_MAX_BITS], S0[MDGMI_MAX_BITS], S1[MDGMI_MAX_BITS];
    float tot = 0.0f;
#pragma unroll
    for (int r = 0; r < CH; r++) tot += bank[r];
    float smin = INFINITY;
#pragma unroll
    for (int k = 0; k < MDGMI_MAX_BITS; k++) {
        if (k < m) {
            float a0 = 0.0f, a1 = 0.0f;
            if (k < CHB) {
#pragma unroll
                for (int r = 0; r < CH; r++) {
                    if ((r >> k) & 1)
                        a1 += bank[r];
                    else
                        a0 += bank[r];
                }
            } else {
#pragma unroll
                for (int l = 0; l < (MAXHI > 0 ? MAXHI : 1); l++) {
                    if (l == k - CHB) {
                        a0 = hi.R0[l];
                        a1 = hi.R1[l];
                    }
                }
            }
            smin = fminf(smin, fminf(a0, a1));
            S0[k] = a0;
            S1[k] = a1;
            ls0[k] = lg2(a0);
            ls1[k] = lg2(a1);
        }
    }
    if (LLR) {
        float lam[MDGMI_MAX_BITS];
        bool ok = smin >= ex2(kFarLog2);
#pragma unroll
        for (int k = 0; k < MDGMI_MAX_BITS; k++) {
            lam[k] = 0.0f;
            if (k < m) {
                lam[k] = log2_ratio(S1[k], S0[k], ls1[k], ls0[k]);
                // an LLR near zero at a large s: recompute from differences
                ok = ok && !(fabsf(lam[k]) < guard);
            }
        }
        if (ok) {
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++)
                if (k < m) llr[i * m + k] = lam[k] * (float)kLn2;
        } else {
            // a class lies too far for the common offset (or y is not finite,
            // or the guard above fired)
            float ltot, ti;
            exact_classes_f32<DIM>(yv, X32, M, m, s, -1, ls0, ls1, ltot, ti);
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++)
                if (k < m) llr[i * m + k] = (ls1[k] - ls0[k]) * (float)kLn2;
        }
    } else {
        // a sent row outside [0, M) gives a NaN cost instead of a stray read
        const uint32_t row = txs[i];
        const bool row_ok = row < (uint32_t)M;
        const uint32_t lw = labels[row_ok ? row : 0u];
        const uint32_t slot = lw & kLabelMask;
        const float* ri = im + (size_t)slot * REC;
        float ui = K - ri[DIM];
#pragma unroll
        for (int q = 0; q < DIM; q++) ui = fmaf(ri[q], yv[q], ui);
        float cg = 0.0f, cm;
        if (ui >= kFarLog2) {
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++) {
                if (k < m) {
                    bool b = (slot >> k) & 1;
                    cg += bit_cost2(b ? log2_ratio(S0[k], S1[k], ls0[k], ls1[k])
                                      : log2_ratio(S1[k], S0[k], ls1[k], ls0[k]));
                }
            }
            cm = mi_cost2(tot, ui);
        } else {
            // the sent point itself is far from y (or y is not finite)
            float ltot, ti = 0.0f;
            exact_classes_f32<DIM>(yv, X32, M, m, s, (int)slot, ls0, ls1, ltot, ti);
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++) {
                if (k < m) {
                    bool b = (slot >> k) & 1;
                    cg += bit_cost2(b ? ls0[k] - ls1[k] : ls1[k] - ls0[k]);
                }
            }
            cm = ltot + ti;
            // decisions below from the exact per-class logarithms
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++) {
                S0[k] = ls0[k];
                S1[k] = ls1[k];
            }
        }
        if (!row_ok) cg = cm = NAN;
        acc.add(cg, cm);
        if (MODE == kModeHd) {
            // bitwise MAP decisions (S1 > S0 decides 1; log2 sums on the
            // exact path, same order) and the nearest point
            int be = 0;
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++)
                if (k < m) be += (S1[k] > S0[k] ? 1 : 0) != (int)((slot >> k) & 1u);
            const bool finite = cg == cg && cm == cm && ui == ui;
            hd->be += finite ? (double)be : (double)m;
            // another point strictly nearer, or the sent point's coordinates
            // shared with a lower label (ties go to the lowest label)
            const bool twin = (lw & kTwinBit) != 0u;
            hd->se += (finite && !(umax > ui) && !twin) ? 0.0 : 1.0;
        }
    }
}

// Max-log metrics of one sample (MODE kModeMlLlr: LLRs into llr; kModeMlGmi:
// the GMI cost of those LLRs into acc, no MI). The same walk as
// direct_sample with maxima instead of exponentials and sums: bank[r] keeps
// the largest u of chunk position r, HiMax the largest u per class of the
// chunk-index bits. A sample whose nearest point lies outside the exponent
// window (or whose y is not finite) takes the FP32 per-class path.
template <int DIM, int CHB, int G, int MODE>
__device__ __forceinline__ void direct_sample_ml(const float* __restrict__ im, const float* __restrict__ ys,
                                                 const uint32_t* __restrict__ txs, int64_t i, int M, int m,
                                                 float s, const float* __restrict__ X32,
                                                 const uint32_t* __restrict__ labels, float* __restrict__ llr,
                                                 CostAcc& acc, float guard = 0.0f) {
    constexpr int CH = 1 << CHB;
    constexpr int REC = DirectRec<DIM>::value;
    constexpr int MAXHI = MDGMI_MAX_BITS - CHB;
    const int nchunk = M >> CHB;
    float yv[DIM];
    float ys2 = 0.0f;
#pragma unroll
    for (int q = 0; q < DIM; q++) {
        yv[q] = ys[i * DIM + q];
        ys2 = fmaf(yv[q], yv[q], ys2);
    }
    const float K = kBias - s * ys2;
    float bank[CH];
#pragma unroll
    for (int r = 0; r < CH; r++) bank[r] = -INFINITY;
    HiMax<G, MAXHI> hi;
    hi.zero();
    for (int c0 = 0; c0 < nchunk; c0 += G) {
        float T[G];
#pragma unroll
        for (int g = 0; g < G; g++) {
            const float* __restrict__ rc = im + (size_t)(c0 + g) * CH * REC;
            float uv[CH];
#pragma unroll
            for (int r = 0; r < CH; r++) {
                float u = K - rc[r * REC + DIM];
#pragma unroll
                for (int q = 0; q < DIM; q++) u = fmaf(rc[r * REC + q], yv[q], u);
                uv[r] = u;
                bank[r] = fmaxf(bank[r], u);
            }
            if (G > 1) {
#pragma unroll
                for (int w = 1; w < CH; w <<= 1) {
#pragma unroll
                    for (int r = 0; r < CH; r += 2 * w) uv[r] = fmaxf(uv[r], uv[r + w]);
                }
                T[g] = uv[0];
            }
        }
        hi.add_group(c0 / G, T);
    }
    float u0[MDGMI_MAX_BITS], u1[MDGMI_MAX_BITS];
    float best = -INFINITY;
#pragma unroll
    for (int r = 0; r < CH; r++) best = fmaxf(best, bank[r]);
#pragma unroll
    for (int k = 0; k < MDGMI_MAX_BITS; k++) {
        u0[k] = u1[k] = 0.0f;
        if (k < m) {
            float a0 = -INFINITY, a1 = -INFINITY;
            if (k < CHB) {
#pragma unroll
                for (int r = 0; r < CH; r++) {
                    if ((r >> k) & 1)
                        a1 = fmaxf(a1, bank[r]);
                    else
                        a0 = fmaxf(a0, bank[r]);
                }
            } else {
#pragma unroll
                for (int l = 0; l < (MAXHI > 0 ? MAXHI : 1); l++) {
                    if (l == k - CHB) {
                        a0 = hi.R0[l];
                        a1 = hi.R1[l];
                    }
                }
            }
            u0[k] = a0;
            u1[k] = a1;
        }
    }
    // fmaxf drops NaN: a non-finite y shows as best = -inf or as y itself
    bool finite = true;
#pragma unroll
    for (int q = 0; q < DIM; q++) finite = finite && __builtin_isfinite(yv[q]);
    bool redo = !(best >= kFarLog2) || !finite;
    if (MODE == kModeMlLlr) {
#pragma unroll
        for (int k = 0; k < MDGMI_MAX_BITS; k++)
            if (k < m) redo = redo || fabsf(u1[k] - u0[k]) < guard;
    }
    if (redo) class_max_u_f32<DIM>(yv, X32, M, m, s, u0, u1);
    if (MODE == kModeMlLlr) {
#pragma unroll
        for (int k = 0; k < MDGMI_MAX_BITS; k++)
            if (k < m) llr[i * m + k] = finite ? (u1[k] - u0[k]) * (float)kLn2 : NAN;
    } else {
        const uint32_t row = txs[i];
        const bool row_ok = row < (uint32_t)M;
        const uint32_t slot = labels[row_ok ? row : 0u];
        float cg = 0.0f;
#pragma unroll
        for (int k = 0; k < MDGMI_MAX_BITS; k++) {
            if (k < m) {
                const bool b = (slot >> k) & 1;
                cg += bit_cost2(b ? u0[k] - u1[k] : u1[k] - u0[k]);
            }
        }
        if (!row_ok || !finite) cg = NAN;
        acc.add(cg, 0.0f);
    }
}

}  // namespace direct
}  // namespace mdgmi
