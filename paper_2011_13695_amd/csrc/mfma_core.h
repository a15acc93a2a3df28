// Device core of the MFMA-split exact demapper, shared by the per-SNR
// kernels (exact_mfma.hip) and the ragged persistent batch (batch.hip).
#pragma once

// The distance term on the matrix cores.
//
// A wave evaluates a 32-point x 32-sample tile with v_mfma_f32_32x32x16_f16:
// A = points (rows), B = samples (columns). The MFMA output is directly
//     u_j(y) = kBias - s ||y - x_j||^2     (log2 units, s = log2(e)/(2 sigma2))
// from the expansion  <2 s x_j, y> - s ||x_j||^2 + (kBias - s ||y||^2),
// each factor split into an fp16 high part and an fp16 remainder:
//     <x', y> ~ x'_hi y_hi + x'_hi y_lo + x'_lo y_hi
// (x'_lo y_lo, ~2^-22 relative, is dropped), products exact in the FP32
// accumulator. 8-D needs K = 28 (two K=16 MFMAs), 4-D and 2-D one MFMA.
//
// The k-slot layout of one point row (A) and one sample column (B); lanes
// 0-31 hold k = 0..7 and lanes 32-63 hold k = 8..15 of each MFMA:
//   8D blk0: A [x'h 0..7 | x'h 0..7]           B [yh 0..7 | yl 0..7]
//      blk1: A [x'l 0..7 | -nh -nl 1 1 0 0 0 0] B [yh 0..7 | 1 1 Kh Kl 0 0 0 0]
//   4D     : A [x'h 0..3 x'l 0..3 | x'h 0..3 -nh -nl 1 1]
//            B [yh 0..3 yh 0..3   | yl 0..3 1 1 Kh Kl]
//   2D     : A [x'h0 x'h1 x'l0 x'l1 x'h0 x'h1 0 0 | -nh -nl 1 1 0 0 0 0]
//            B [yh0 yh1 yh0 yh1 yl0 yl1 0 0        | 1 1 Kh Kl 0 0 0 0]
//   1D     : A [x'h0 x'l0 x'h0 0 0 0 0 0          | -nh -nl 1 1 0 0 0 0]
//            B [yh0 yh0 yl0 0 0 0 0 0             | 1 1 Kh Kl 0 0 0 0]
// with x' = 2 s x, n = s ||x||^2 and K = kBias - s ||y||^2.
//
// Output layout of the 32x32 MFMA: lane l, register r holds row
// p = 8 (r >> 2) + 4 (l >> 5) + (r & 3) of column l & 31. With points stored
// in label order, label bits 0, 1, 3, 4 of the point are bits of r, bit 2 is
// the lane half and bits 5.. are the tile index. Each lane keeps a running
// bank[r] of its 16 exponentials (one add per pair) and adds the tile total
// (15 adds per 16 pairs) to the classes of the tile-index bits, eight tiles
// at a time; the two lane halves are combined once per sample at the end.
#include "device_common.h"

namespace mdgmi {
namespace mfma {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr float kPadNorm = 60000.0f;   // padding rows: u = K - 60000 -> e = 0

// Operand split of the distance term: fp16 hi + lo (two products per
// coordinate, fp16 range) or bf16 in three parts (six products per
// coordinate, about 24 significant bits, FP32 range). Operands of either
// split travel as half8 registers (16 bytes); the bf16 MFMA reinterprets them.
constexpr int kSplitF16 = 0, kSplitBF16 = 1;

// K = 16 blocks per point: fp16 needs 2 for 8-D (K = 28), else 1; bf16 needs
// ceil((6 DIM + 6) / 16).
template <int DIM, int S = kSplitF16>
struct Blk {
    static constexpr int value = S == kSplitF16 ? (DIM == 8 ? 2 : 1) : (6 * DIM + 6 + 15) / 16;
};

__device__ __forceinline__ void split16(double v, _Float16& hi, _Float16& lo) {
    hi = (_Float16)v;
    lo = (_Float16)(v - (double)hi);
}
__device__ __forceinline__ void split16f(float v, _Float16& hi, _Float16& lo) {
    hi = (_Float16)v;
    lo = (_Float16)(v - (float)hi);
}

union H8 {
    half8 v;
    uint4 u;
    _Float16 h[8];
};

// A image of one (format, SNR): [tile][blk][half][row] of 8 halves (16 B);
// writes the entries of one slot (slot < ntiles * 32; slots >= M are padding
// rows whose exponentials vanish).
// bf16 layout: entry k of the K vector sits in block k / 16, lane half
// (k % 16) / 8, position k % 8. For each coordinate d the six products
// x1 y1, x1 y2, x2 y1, x1 y3, x2 y2, x3 y1 (dropped: x2 y3, x3 y2, x3 y3,
// ~2^-24 relative), then -n1 -n2 -n3 against ones and ones against K1 K2 K3.
template <int DIM>
struct Bf16K {
    static constexpr int K = 6 * DIM + 6;
};

__device__ __forceinline__ void split3_bf16(double v, __bf16& a, __bf16& b, __bf16& c) {
    a = (__bf16)v;
    const double r1 = v - (double)a;
    b = (__bf16)r1;
    c = (__bf16)(r1 - (double)b);
}
__device__ __forceinline__ void split3_bf16f(float v, __bf16& a, __bf16& b, __bf16& c) {
    a = (__bf16)v;
    const float r1 = v - (float)a;
    b = (__bf16)r1;
    c = (__bf16)(r1 - (float)b);
}

union B8 {
    half8 v;
    uint4 u;
    __bf16 h[8];
};

template <int DIM>
__device__ inline void image_slot_bf16(const double* __restrict__ X64, int M, double s, int slot,
                                       uint4* __restrict__ base) {
    constexpr int NB = Blk<DIM, kSplitBF16>::value;
    const int t = slot >> 5, row = slot & 31;
    __bf16 a[NB * 16];
#pragma unroll
    for (int k = 0; k < NB * 16; k++) a[k] = (__bf16)0.0f;
    const __bf16 one = (__bf16)1.0f;
    if (slot < M) {
        double n2 = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; d++) {
            const double x = X64[(size_t)slot * DIM + d];
            n2 += x * x;
            __bf16 x1, x2, x3;
            split3_bf16(2.0 * s * x, x1, x2, x3);
            a[6 * d + 0] = x1;
            a[6 * d + 1] = x1;
            a[6 * d + 2] = x2;
            a[6 * d + 3] = x1;
            a[6 * d + 4] = x2;
            a[6 * d + 5] = x3;
        }
        __bf16 n1, nb, n3;
        split3_bf16(-(s * n2), n1, nb, n3);
        a[6 * DIM + 0] = n1;
        a[6 * DIM + 1] = nb;
        a[6 * DIM + 2] = n3;
    } else {
        a[6 * DIM + 0] = (__bf16)(-kPadNorm);
    }
    a[6 * DIM + 3] = one;
    a[6 * DIM + 4] = one;
    a[6 * DIM + 5] = one;
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
        for (int h = 0; h < 2; h++) {
            B8 v;
#pragma unroll
            for (int i = 0; i < 8; i++) v.h[i] = a[16 * b + 8 * h + i];
            base[((t * NB + b) * 2 + h) * 32 + row] = v.u;
        }
}

template <int DIM, int S = kSplitF16>
__device__ inline void image_slot(const double* __restrict__ X64, int M, int ntiles, double s, int slot,
                                  uint4* __restrict__ base) {
    if (S == kSplitBF16) {
        image_slot_bf16<DIM>(X64, M, s, slot, base);
        return;
    }
    constexpr int NB = Blk<DIM>::value;
    const int t = slot >> 5, row = slot & 31;
    H8 a[NB][2];
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
        for (int h = 0; h < 2; h++)
#pragma unroll
            for (int i = 0; i < 8; i++) a[b][h].h[i] = (_Float16)0.0f;
    _Float16 xh[DIM], xl[DIM], nh, nl;
    if (slot < M) {
        double n2 = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; d++) {
            double x = X64[(size_t)slot * DIM + d];
            n2 += x * x;
            split16(2.0 * s * x, xh[d], xl[d]);
        }
        split16(s * n2, nh, nl);
        nh = -nh;
        nl = -nl;
    } else {
#pragma unroll
        for (int d = 0; d < DIM; d++) xh[d] = xl[d] = (_Float16)0.0f;
        nh = (_Float16)(-kPadNorm);
        nl = (_Float16)0.0f;
    }
    const _Float16 one = (_Float16)1.0f;
    if (DIM == 8) {
#pragma unroll
        for (int d = 0; d < 8; d++) {
            a[0][0].h[d] = xh[d];
            a[0][1].h[d] = xh[d];
            a[NB - 1][0].h[d] = xl[d];
        }
        a[NB - 1][1].h[0] = nh;
        a[NB - 1][1].h[1] = nl;
        a[NB - 1][1].h[2] = one;
        a[NB - 1][1].h[3] = one;
    } else if (DIM == 4) {
#pragma unroll
        for (int d = 0; d < 4; d++) {
            a[0][0].h[d] = xh[d];
            a[0][0].h[4 + d] = xl[d];
            a[0][1].h[d] = xh[d];
        }
        a[0][1].h[4] = nh;
        a[0][1].h[5] = nl;
        a[0][1].h[6] = one;
        a[0][1].h[7] = one;
    } else if (DIM == 2) {
        a[0][0].h[0] = xh[0];
        a[0][0].h[1] = xh[DIM - 1];
        a[0][0].h[2] = xl[0];
        a[0][0].h[3] = xl[DIM - 1];
        a[0][0].h[4] = xh[0];
        a[0][0].h[5] = xh[DIM - 1];
        a[0][1].h[0] = nh;
        a[0][1].h[1] = nl;
        a[0][1].h[2] = one;
        a[0][1].h[3] = one;
    } else {
        a[0][0].h[0] = xh[0];
        a[0][0].h[1] = xl[0];
        a[0][0].h[2] = xh[0];
        a[0][1].h[0] = nh;
        a[0][1].h[1] = nl;
        a[0][1].h[2] = one;
        a[0][1].h[3] = one;
    }
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
        for (int h = 0; h < 2; h++) base[((t * NB + b) * 2 + h) * 32 + row] = a[b][h].u;
    (void)ntiles;
}

// bf16 B operands of one sample column for lane half h (layout of Bf16K).
template <int DIM>
__device__ __forceinline__ void make_b_bf16(const float* yv, float K, int h, half8* bop) {
    constexpr int NB = Blk<DIM, kSplitBF16>::value;
    __bf16 b[NB * 16];
#pragma unroll
    for (int k = 0; k < NB * 16; k++) b[k] = (__bf16)0.0f;
    const __bf16 one = (__bf16)1.0f;
#pragma unroll
    for (int d = 0; d < DIM; d++) {
        __bf16 y1, y2, y3;
        split3_bf16f(yv[d], y1, y2, y3);
        b[6 * d + 0] = y1;
        b[6 * d + 1] = y2;
        b[6 * d + 2] = y1;
        b[6 * d + 3] = y3;
        b[6 * d + 4] = y2;
        b[6 * d + 5] = y1;
    }
    __bf16 k1, k2, k3;
    split3_bf16f(K, k1, k2, k3);
    b[6 * DIM + 0] = one;
    b[6 * DIM + 1] = one;
    b[6 * DIM + 2] = one;
    b[6 * DIM + 3] = k1;
    b[6 * DIM + 4] = k2;
    b[6 * DIM + 5] = k3;
#pragma unroll
    for (int blk = 0; blk < NB; blk++) {
        B8 v;
#pragma unroll
        for (int i = 0; i < 8; i++) v.h[i] = h ? b[16 * blk + 8 + i] : b[16 * blk + i];
        bop[blk] = v.v;
    }
}

// B operands of one sample column for lane half h.
template <int DIM, int S = kSplitF16>
__device__ __forceinline__ void make_b(const float* yv, float K, int h, half8* bop) {
    if (S == kSplitBF16) {
        make_b_bf16<DIM>(yv, K, h, bop);
        return;
    }
    _Float16 yh[DIM], yl[DIM], kh, kl;
#pragma unroll
    for (int d = 0; d < DIM; d++) split16f(yv[d], yh[d], yl[d]);
    split16f(K, kh, kl);
    const _Float16 one = (_Float16)1.0f, zero = (_Float16)0.0f;
    H8 b0, b1;
#pragma unroll
    for (int i = 0; i < 8; i++) b0.h[i] = b1.h[i] = zero;
    if (DIM == 8) {
#pragma unroll
        for (int d = 0; d < 8; d++) {
            b0.h[d] = h ? yl[d] : yh[d];
            b1.h[d] = yh[d];
        }
        if (h) {
            b1.h[0] = one;
            b1.h[1] = one;
            b1.h[2] = kh;
            b1.h[3] = kl;
#pragma unroll
            for (int i = 4; i < 8; i++) b1.h[i] = zero;
        }
        bop[0] = b0.v;
        bop[1] = b1.v;
    } else if (DIM == 4) {
        if (!h) {
#pragma unroll
            for (int d = 0; d < 4; d++) {
                b0.h[d] = yh[d];
                b0.h[4 + d] = yh[d];
            }
        } else {
#pragma unroll
            for (int d = 0; d < 4; d++) b0.h[d] = yl[d];
            b0.h[4] = one;
            b0.h[5] = one;
            b0.h[6] = kh;
            b0.h[7] = kl;
        }
        bop[0] = b0.v;
    } else if (DIM == 2) {
        if (!h) {
            b0.h[0] = yh[0];
            b0.h[1] = yh[DIM - 1];
            b0.h[2] = yh[0];
            b0.h[3] = yh[DIM - 1];
            b0.h[4] = yl[0];
            b0.h[5] = yl[DIM - 1];
        } else {
            b0.h[0] = one;
            b0.h[1] = one;
            b0.h[2] = kh;
            b0.h[3] = kl;
        }
        bop[0] = b0.v;
    } else {
        if (!h) {
            b0.h[0] = yh[0];
            b0.h[1] = yh[0];
            b0.h[2] = yl[0];
        } else {
            b0.h[0] = one;
            b0.h[1] = one;
            b0.h[2] = kh;
            b0.h[3] = kl;
        }
        bop[0] = b0.v;
    }
}

// Operands of one tile for this lane: p points at [tile][blk 0][half][row]
// of the lane's half and row; blocks are 64 uint4 apart.
template <int NB>
__device__ __forceinline__ void load_a_at(const uint4* __restrict__ p, half8* a) {
#pragma unroll
    for (int b = 0; b < NB; b++) {
        H8 tmp;
        tmp.u = p[b * 64];
        a[b] = tmp.v;
    }
}

// Values of a register in the lower (lanes 0-31) and upper (32-63) half of
// the wave, seen by every lane (v_permlane32_swap).
struct Halves {
    float lo, hi;
};
__device__ __forceinline__ Halves halves(float v) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return {__uint_as_float(r[0]), __uint_as_float(r[1])};
}
// lower + upper, formed in this order in every lane
__device__ __forceinline__ float half_sum(float v) {
    const Halves t = halves(v);
    return t.lo + t.hi;
}

template <int NB, int S = kSplitF16>
__device__ __forceinline__ f32x16 tile_mfma(const half8* a, const half8* b) {
    if (S == kSplitBF16) {
        f32x16 u = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[0]),
                                                           __builtin_bit_cast(bf16x8, b[0]), (f32x16){}, 0, 0, 0);
#pragma unroll
        for (int k = 1; k < NB; k++)
            u = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[k]),
                                                        __builtin_bit_cast(bf16x8, b[k]), u, 0, 0, 0);
        return u;
    }
    f32x16 u = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[0], b[0], (f32x16){}, 0, 0, 0);
    if (NB == 2) u = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[NB - 1], b[NB - 1], u, 0, 0, 0);
    return u;
}

// Exponentials of one or more sample columns against every tile of the A
// image, folded into a per-register bank (label bits in the register index)
// and per-group class sums of the tile-index bits (HiAcc).
//
// Software pipeline: the MFMA of tile t+1 is in flight while the
// exponentials of tile t issue, and the operands of tile t+2 are loaded
// meanwhile. Tile indices wrap (ntiles is a power of two and a multiple of
// G), so the last steps compute unused tiles instead of branching; the wrap
// is applied once per group through two base pointers (for G >= 2, tiles
// t + 2 past the group are the first two of the next group). CLAMP caps each
// exponent at 110 so that sums of up to 2^12 terms stay finite when the
// offset has been raised for far classes (only those classes are read then).
template <int DIM, int NCOL, int G, bool CLAMP, int MAXHI, bool TRACK = false, int S = kSplitF16>
__device__ __forceinline__ void tile_loop(const uint4* __restrict__ A, int ntiles, int h, int col,
                                          const half8 (&bop)[NCOL][Blk<DIM, S>::value], float (&bank)[NCOL][16],
                                          HiAcc<G, MAXHI> (&hi)[NCOL], float* umax = nullptr) {
    constexpr int NB = Blk<DIM, S>::value;
    constexpr int TS = NB * 64;  // uint4 per tile of the image
#pragma unroll
    for (int c = 0; c < NCOL; c++) {
#pragma unroll
        for (int r = 0; r < 16; r++) bank[c][r] = 0.0f;
        hi[c].zero();
        if (TRACK) umax[c] = -INFINITY;
    }
    const int tmask = ntiles - 1;
    const uint4* __restrict__ Al = A + h * 32 + col;
    half8 a_nxt[NB];
    f32x16 u_nxt[NCOL];
    load_a_at<NB>(Al, a_nxt);
#pragma unroll
    for (int c = 0; c < NCOL; c++) u_nxt[c] = tile_mfma<NB, S>(a_nxt, bop[c]);
    load_a_at<NB>(Al + (1 & tmask) * TS, a_nxt);
    for (int g0 = 0; g0 < ntiles; g0 += G) {
        const uint4* __restrict__ Acur = Al + g0 * TS;
        const uint4* __restrict__ Anxt = Al + ((g0 + G) & tmask) * TS;
        float T[NCOL][G];
#pragma unroll
        for (int i = 0; i < G; i++) {
            f32x16 u_cur[NCOL];
#pragma unroll
            for (int c = 0; c < NCOL; c++) {
                u_cur[c] = u_nxt[c];
                u_nxt[c] = tile_mfma<NB, S>(a_nxt, bop[c]);
            }
            if (G == 1)
                load_a_at<NB>(Al + ((g0 + 2) & tmask) * TS, a_nxt);
            else if (i + 2 < G)
                load_a_at<NB>(Acur + (i + 2) * TS, a_nxt);
            else
                load_a_at<NB>(Anxt + (i + 2 - G) * TS, a_nxt);
#pragma unroll
            for (int c = 0; c < NCOL; c++) {
                if (TRACK) {
                    // largest u of the tile (nearest point), a tree of 3-input maxima
                    const f32x16& u = u_cur[c];
                    const float a = fmaxf(fmaxf(u[0], u[1]), u[2]), b = fmaxf(fmaxf(u[3], u[4]), u[5]);
                    const float d = fmaxf(fmaxf(u[6], u[7]), u[8]), e = fmaxf(fmaxf(u[9], u[10]), u[11]);
                    const float g = fmaxf(fmaxf(u[12], u[13]), u[14]), q = fmaxf(fmaxf(u[15], a), b);
                    umax[c] = fmaxf(fmaxf(umax[c], q), fmaxf(fmaxf(d, e), g));
                }
                float ev[16];
#pragma unroll
                for (int r = 0; r < 16; r++) {
                    ev[r] = ex2(CLAMP ? fminf(u_cur[c][r], 110.0f) : u_cur[c][r]);
                    bank[c][r] += ev[r];
                }
                if (G > 1) {
#pragma unroll
                    for (int w = 1; w < 16; w <<= 1) {
#pragma unroll
                        for (int r = 0; r < 16; r += 2 * w) ev[r] += ev[r + w];
                    }
                    T[c][i] = ev[0];
                }
            }
            // keep one tile's accumulators in flight: without this fence the
            // independent MFMAs of the whole group are hoisted together
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int c = 0; c < NCOL; c++) hi[c].add_group(g0 / G, T[c]);
    }
}

// This lane's partial class sums p0[k], p1[k] (its 16 rows of every tile)
// from its bank and tile-bit sums. Label bits 0, 1, 3, 4 are bits 0..3 of
// the register index (folded by a register tree), bit 2 is the lane half
// (p0[2] = p1[2] = this half's total), bits 5.. come from the tile index.
// The bank is consumed.
template <int MAXHI, int G>
__device__ __forceinline__ void half_partials(float* b, const HiAcc<G, MAXHI>& hi, int m, float* p0, float* p1) {
    p0[0] = ((b[0] + b[2]) + (b[4] + b[6])) + ((b[8] + b[10]) + (b[12] + b[14]));
    p1[0] = ((b[1] + b[3]) + (b[5] + b[7])) + ((b[9] + b[11]) + (b[13] + b[15]));
#pragma unroll
    for (int j = 0; j < 8; j++) b[j] = b[2 * j] + b[2 * j + 1];
    p0[1] = (b[0] + b[2]) + (b[4] + b[6]);
    p1[1] = (b[1] + b[3]) + (b[5] + b[7]);
#pragma unroll
    for (int j = 0; j < 4; j++) b[j] = b[2 * j] + b[2 * j + 1];
    p0[3] = b[0] + b[2];
    p1[3] = b[1] + b[3];
    p0[4] = b[0] + b[1];
    p1[4] = b[2] + b[3];
    p0[2] = p1[2] = p0[4] + p1[4];
#pragma unroll
    for (int k = 5; k < MDGMI_MAX_BITS; k++) {
        p0[k] = k < m ? hi.R0[k - 5] : 1.0f;
        p1[k] = k < m ? hi.R1[k - 5] : 1.0f;
    }
}

// Full class sums of label bit k from both halves' partials, identical in
// every lane (all 64 lanes must take part).
__device__ __forceinline__ void full_sums(const float* p0, const float* p1, int k, float& S0k, float& S1k) {
    if (k == 2) {
        const Halves t = halves(p0[2]);
        S0k = t.lo;
        S1k = t.hi;
    } else {
        S0k = half_sum(p0[k]);
        S1k = half_sum(p1[k]);
    }
}

// LLR mode, a column tile where some sample has a class too far for the
// common offset (its sum below 2^kFarLog2): classes that were in range keep
// their first-pass sums; the far ones are summed again with the offset
// raised by 100 (the same fold, the exponents of the near points capped);
// classes still out of range, or non-finite inputs, take the exact
// per-class path. p0/p1 are the first pass's partials of this lane.
template <int DIM, int G, int MAXHI, int S = kSplitF16>
__device__ __forceinline__ void llr_far_pass(const uint4* __restrict__ A, const float* __restrict__ ys, int64_t n,
                                          int64_t i, int M, int m, int ntiles, float s,
                                          const float* __restrict__ X32, float* __restrict__ llr, const float* p0,
                                          const float* p1) {
    constexpr int NB = Blk<DIM, S>::value;
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, col = lane & 31;
    const float thr = ex2(kFarLog2);
    // first pass: this half's bits, near classes' log2 sums
    constexpr int NJ = (MDGMI_MAX_BITS + 1) / 2;
    float lnear0[NJ], lnear1[NJ];
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        lnear0[j] = lnear1[j] = 0.0f;
        if (2 * j < m) {
            const int ke = 2 * j, ko = ke + 1 < MDGMI_MAX_BITS ? ke + 1 : ke;
            float S0e, S1e, S0o = 1.0f, S1o = 1.0f;
            full_sums(p0, p1, ke, S0e, S1e);
            if (ko < m) full_sums(p0, p1, ko, S0o, S1o);
            const float s0 = h ? S0o : S0e, s1 = h ? S1o : S1e;
            lnear0[j] = s0 >= thr ? lg2(s0) : NAN;   // NaN marks a far (or non-finite) class
            lnear1[j] = s1 >= thr ? lg2(s1) : NAN;
        }
    }
    // second pass with the offset raised by 100
    half8 bop[1][NB];
    float yv[DIM];
    const bool valid = i < n;
    float ys2 = 0.0f;
#pragma unroll
    for (int d = 0; d < DIM; d++) {
        yv[d] = valid ? ys[i * DIM + d] : 0.0f;
        ys2 = fmaf(yv[d], yv[d], ys2);
    }
    make_b<DIM, S>(yv, fmaf(-s, ys2, kBias + 100.0f), h, bop[0]);
    float bank[1][16];
    HiAcc<G, MAXHI> hi[1];
    tile_loop<DIM, 1, G, true, MAXHI, false, S>(A, ntiles, h, col, bop, bank, hi);
    float q0[MDGMI_MAX_BITS], q1[MDGMI_MAX_BITS];
    half_partials<MAXHI, G>(bank[0], hi[0], m, q0, q1);
    float out[NJ];
    bool bad = false;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        out[j] = 0.0f;
        if (2 * j < m) {
            const int ke = 2 * j, ko = ke + 1 < MDGMI_MAX_BITS ? ke + 1 : ke;
            float S0e, S1e, S0o = 1.0f, S1o = 1.0f;
            full_sums(q0, q1, ke, S0e, S1e);
            if (ko < m) full_sums(q0, q1, ko, S0o, S1o);
            const int k = ke + h;
            if (k < m) {
                const float f0 = h ? S0o : S0e, f1 = h ? S1o : S1e;
                // log2 of each class sum at the common offset
                const float l0 = lnear0[j] == lnear0[j] ? lnear0[j] : lg2(f0) - 100.0f;
                const float l1 = lnear1[j] == lnear1[j] ? lnear1[j] : lg2(f1) - 100.0f;
                const bool r0 = lnear0[j] == lnear0[j] || f0 >= thr;
                const bool r1 = lnear1[j] == lnear1[j] || f1 >= thr;
                bad = bad || !(r0 && r1);
                out[j] = l1 - l0;
            }
        }
    }
    const Halves hb = halves(bad ? 1.0f : 0.0f);
    const bool any_bad = hb.lo + hb.hi > 0.0f;  // for this sample, over both halves
    if (!valid) return;
    if (!any_bad) {
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            const int k = 2 * j + h;
            if (k < m) llr[i * m + k] = out[j] * (float)kLn2;
        }
    } else if (h == 0) {
        float yc[DIM], ls0[MDGMI_MAX_BITS], ls1[MDGMI_MAX_BITS], ltot, ti;
#pragma unroll
        for (int d = 0; d < DIM; d++) yc[d] = ys[i * DIM + d];
        exact_classes_f32<DIM>(yc, X32, M, m, s, -1, ls0, ls1, ltot, ti);
#pragma unroll
        for (int k = 0; k < MDGMI_MAX_BITS; k++)
            if (k < m) llr[i * m + k] = (ls1[k] - ls0[k]) * (float)kLn2;
    }
}

// One column tile: NCOL x 32 samples starting at sample ct * NCOL * 32 of one
// (format, SNR) instance, against all points of its A image. Costs go to
// acc (GMI mode) or LLRs to llr (LLR mode). All 64 lanes of the wave must
// call it together (the MFMA and the half-wave swaps need every lane).
template <int DIM, int NCOL, int G, int MODE, int S = kSplitF16>
__device__ __forceinline__ void mfma_coltile(const uint4* __restrict__ A, const float* __restrict__ ys,
                                             const uint32_t* __restrict__ txs, int64_t n, int64_t ct, int M,
                                             int m, int ntiles, float s, const float* __restrict__ X32,
                                             const uint32_t* __restrict__ labels, float* __restrict__ llr,
                                             CostAcc& acc, HdAcc* hd = nullptr, float guard = 0.0f) {
    constexpr bool LLR = MODE == kModeLlr;
    constexpr bool HD = MODE == kModeHd;
    constexpr int NB = Blk<DIM, S>::value;
    constexpr int MAXHI = MDGMI_MAX_BITS - 5;
    constexpr int TS = NB * 64;
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, col = lane & 31;
    half8 bop[NCOL][NB];
    int64_t idx[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; c++) {
        idx[c] = (ct * NCOL + c) * 32 + col;
        const bool valid = idx[c] < n;
        float yv[DIM], ys2 = 0.0f;
#pragma unroll
        for (int d = 0; d < DIM; d++) {
            yv[d] = valid ? ys[idx[c] * DIM + d] : 0.0f;
            ys2 = fmaf(yv[d], yv[d], ys2);
        }
        const float K = fmaf(-s, ys2, kBias);
        make_b<DIM, S>(yv, K, h, bop[c]);
    }
    float bank[NCOL][16];
    HiAcc<G, MAXHI> hi[NCOL];
    float umax[NCOL];
    tile_loop<DIM, NCOL, G, false, MAXHI, HD, S>(A, ntiles, h, col, bop, bank, hi, umax);
    // ---- epilogue ----
    // Each lane folds its own 16 rows into per-bit partial class sums; the
    // two lane halves (rows differing in label bit 2) are combined with one
    // lane swap per value, summed in the same order in both halves so that
    // both hold identical class sums; each half then finishes every other
    // label bit (half h takes bits h, h + 2, ...). Bits are streamed in pairs
    // so that few class sums are live at a time.
#pragma unroll
    for (int c = 0; c < NCOL; c++) {
        const int64_t i = idx[c];
        float p0[MDGMI_MAX_BITS], p1[MDGMI_MAX_BITS];  // this half's partial class sums
        half_partials<MAXHI, G>(bank[c], hi[c], m, p0, p1);
        float S0t, S1t;
        full_sums(p0, p1, 2, S0t, S1t);
        const float tot = S0t + S1t;
        if (LLR) {
            float smin = INFINITY;
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++) {
                if (k < m) {
                    float S0k, S1k;
                    full_sums(p0, p1, k, S0k, S1k);
                    smin = fminf(smin, fminf(S0k, S1k));
                }
            }
            // a class of some sample of this column lies too far for the
            // common offset (or y is not finite): second pass for the column
            if (__ballot(!(smin >= ex2(kFarLog2))) != 0ull) {
                llr_far_pass<DIM, G, MAXHI, S>(A, ys, n, i, M, m, ntiles, s, X32, llr, p0, p1);
                continue;
            }
            constexpr int NJ = (MDGMI_MAX_BITS + 1) / 2;
            float lam[NJ];
            bool near0 = false;
#pragma unroll
            for (int j = 0; j < NJ; j++) {
                lam[j] = 0.0f;
                if (2 * j < m) {  // uniform
                    const int ke = 2 * j, ko = ke + 1 < MDGMI_MAX_BITS ? ke + 1 : ke;
                    float S0e, S1e, S0o = 1.0f, S1o = 1.0f;
                    if (ke == 2) {
                        S0e = S0t;
                        S1e = S1t;
                    } else {
                        full_sums(p0, p1, ke, S0e, S1e);
                    }
                    if (ko < m) full_sums(p0, p1, ko, S0o, S1o);
                    const int k = ke + h;
                    const float s0 = h ? S0o : S0e, s1 = h ? S1o : S1e;
                    lam[j] = log2_ratio_fast(s1, s0);
                    if (k < m) near0 = near0 || fabsf(lam[j]) < guard;
                }
            }
            // an LLR near zero at a large s (either half's bits): the whole
            // sample is recomputed on the per-class path by lane half 0
            const Halves hz = halves(near0 ? 1.0f : 0.0f);
            const bool redo = hz.lo + hz.hi > 0.0f;
            if (i >= n) continue;
            if (!redo) {
#pragma unroll
                for (int j = 0; j < NJ; j++) {
                    const int k = 2 * j + h;
                    if (k < m) llr[i * m + k] = lam[j] * (float)kLn2;
                }
            } else if (h == 0) {
                float yc[DIM], ls0[MDGMI_MAX_BITS], ls1[MDGMI_MAX_BITS], ltot, ti;
#pragma unroll
                for (int d = 0; d < DIM; d++) yc[d] = ys[i * DIM + d];
                exact_classes_f32<DIM>(yc, X32, M, m, s, -1, ls0, ls1, ltot, ti);
#pragma unroll
                for (int k = 0; k < MDGMI_MAX_BITS; k++)
                    if (k < m) llr[i * m + k] = (ls1[k] - ls0[k]) * (float)kLn2;
            }
            continue;
        }
        // a sent row outside [0, M) gives a NaN cost instead of a stray read
        const uint32_t row = i < n ? txs[i] : 0u;
        const bool row_ok = row < (uint32_t)M;
        const uint32_t lw = labels[row_ok ? row : 0u];
        const uint32_t slot = lw & kLabelMask;
        const bool twin = HD && (lw & kTwinBit) != 0u;  // a lower label shares the sent point
        // u of the sent point by the matrix cores themselves: one more MFMA
        // whose row r is the sent point of sample r puts u_i(y) on the
        // diagonal, bit-identical to the value inside the class sums, so the
        // MI cost log2 sum_j 2^(u_j - u_i) carries no recomputation error.
        // Diagonal element r sits in lane half (r >> 2) & 1, register
        // ((r >> 3) << 2) | (r & 3).
        half8 ad[NB];
        load_a_at<NB>(A + (int)(slot >> 5) * TS + h * 32 + (int)(slot & 31), ad);
        const f32x16 ud = tile_mfma<NB, S>(ad, bop[c]);
        const int q = ((col >> 3) << 2) | (col & 3);
        float dv = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; r++) dv = (r == q) ? ud[r] : dv;
        const Halves d = halves(dv);
        const float ui = ((col >> 2) & 1) ? d.hi : d.lo;
        // this half's class sums of its bit pair j (bit 2j + h)
        auto own_sums = [&](int j, float& s0, float& s1) {
            const int ke = 2 * j, ko = ke + 1 < MDGMI_MAX_BITS ? ke + 1 : ke;
            float S0e, S1e, S0o = 1.0f, S1o = 1.0f;
            if (ke == 2) {
                S0e = S0t;
                S1e = S1t;
            } else {
                full_sums(p0, p1, ke, S0e, S1e);
            }
            if (ko < m) full_sums(p0, p1, ko, S0o, S1o);
            s0 = h ? S0o : S0e;
            s1 = h ? S1o : S1e;
        };
        // GMI cost of this half's bits, sum_k log2(T / S_sent,k), as one
        // logarithm of the product of S_sent,k / T (cost_from_product)
        float cg = 0.0f, be = 0.0f, prod = 1.0f;
        const float rT = __builtin_amdgcn_rcpf(tot);
#pragma unroll
        for (int j = 0; j < (MDGMI_MAX_BITS + 1) / 2; j++) {
            if (2 * j < m) {  // uniform
                float s0, s1;
                own_sums(j, s0, s1);
                const int k = 2 * j + h;
                if (k < m) {
                    const bool bk = (slot >> k) & 1;
                    prod *= (bk ? s1 : s0) * rT;
                    if (HD) be += (s1 > s0) != bk ? 1.0f : 0.0f;  // bitwise MAP decision
                }
            }
        }
        const bool fast = prod >= 0x1p-120f;
        if (__ballot(!fast) == 0ull) {
            cost_from_product(prod, cg);
        } else {
            // some sample of the wave has a cost beyond 120 bits or a
            // non-finite sum: bit by bit, log2(1 + S_other / S_sent)
            asm volatile("" ::: "memory");  // keeps the rare path a real branch
#pragma unroll
            for (int j = 0; j < (MDGMI_MAX_BITS + 1) / 2; j++) {
                if (2 * j < m) {
                    float s0, s1;
                    own_sums(j, s0, s1);
                    const int k = 2 * j + h;
                    if (k < m) cg += bit_cost_sum2(s0 + s1, ((slot >> k) & 1) ? s1 : s0);
                }
            }
        }
        cg = half_sum(cg);
        float sym = 0.0f;
        if (HD) {
            be = half_sum(be);
            const Halves um = halves(umax[c]);
            // another point strictly nearer, or the sent point's coordinates
            // shared with a lower label (ties go to the lowest label)
            sym = fmaxf(um.lo, um.hi) > ui || twin ? 1.0f : 0.0f;
        }
        if (h != 0 || i >= n) continue;
        float cm;
        if (ui >= kFarLog2) {
            cm = mi_cost2(tot, ui);
        } else {
            // the sent point itself is far from y (or y is not finite)
            float yc[DIM], ls0[MDGMI_MAX_BITS], ls1[MDGMI_MAX_BITS], ltot, ti = 0.0f, tmin = 0.0f;
#pragma unroll
            for (int dd = 0; dd < DIM; dd++) yc[dd] = ys[i * DIM + dd];
            exact_classes_f32<DIM>(yc, X32, M, m, s, (int)slot, ls0, ls1, ltot, ti, HD ? &tmin : nullptr);
            cg = 0.0f;
            be = 0.0f;
            // the split factors may be out of range here: decide the symbol
            // from the FP32 distances as well
            if (HD) sym = tmin < ti || twin ? 1.0f : 0.0f;
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++) {
                if (k < m) {
                    const bool bk = (slot >> k) & 1;
                    cg += bit_cost2(bk ? ls0[k] - ls1[k] : ls1[k] - ls0[k]);
                    if (HD) be += (ls1[k] > ls0[k]) != bk ? 1.0f : 0.0f;  // from the exact logarithms
                }
            }
            cm = ltot + ti;
        }
        if (!row_ok) cg = cm = NAN;
        acc.add(cg, cm);
        if (HD) {
            const bool finite = cg == cg && cm == cm && ui == ui;
            hd->be += finite ? (double)be : (double)m;
            hd->se += finite ? (double)sym : 1.0;
        }
    }
}

// ---- max-log metrics --------------------------------------------------
// The max-log LLR needs, per bit, the largest u of each class: the same
// tile walk and fold as the exact sums with max in place of exponential and
// add (bank[r] = running max of register r, HiMax for the tile-index bits).
// Max is exact and order-free, so both lane halves hold identical class
// maxima whatever the combination order.
template <int DIM, int NCOL, int G, int MAXHI, int S = kSplitF16>
__device__ __forceinline__ void tile_loop_max(const uint4* __restrict__ A, int ntiles, int h, int col,
                                              const half8 (&bop)[NCOL][Blk<DIM, S>::value], float (&bank)[NCOL][16],
                                              HiMax<G, MAXHI> (&hi)[NCOL]) {
    constexpr int NB = Blk<DIM, S>::value;
    constexpr int TS = NB * 64;
#pragma unroll
    for (int c = 0; c < NCOL; c++) {
#pragma unroll
        for (int r = 0; r < 16; r++) bank[c][r] = -INFINITY;
        hi[c].zero();
    }
    const int tmask = ntiles - 1;
    const uint4* __restrict__ Al = A + h * 32 + col;
    half8 a_nxt[NB];
    f32x16 u_nxt[NCOL];
    load_a_at<NB>(Al, a_nxt);
#pragma unroll
    for (int c = 0; c < NCOL; c++) u_nxt[c] = tile_mfma<NB, S>(a_nxt, bop[c]);
    load_a_at<NB>(Al + (1 & tmask) * TS, a_nxt);
    for (int g0 = 0; g0 < ntiles; g0 += G) {
        const uint4* __restrict__ Acur = Al + g0 * TS;
        const uint4* __restrict__ Anxt = Al + ((g0 + G) & tmask) * TS;
        float T[NCOL][G];
#pragma unroll
        for (int i = 0; i < G; i++) {
            f32x16 u_cur[NCOL];
#pragma unroll
            for (int c = 0; c < NCOL; c++) {
                u_cur[c] = u_nxt[c];
                u_nxt[c] = tile_mfma<NB, S>(a_nxt, bop[c]);
            }
            if (G == 1)
                load_a_at<NB>(Al + ((g0 + 2) & tmask) * TS, a_nxt);
            else if (i + 2 < G)
                load_a_at<NB>(Acur + (i + 2) * TS, a_nxt);
            else
                load_a_at<NB>(Anxt + (i + 2 - G) * TS, a_nxt);
#pragma unroll
            for (int c = 0; c < NCOL; c++) {
                const f32x16& u = u_cur[c];
#pragma unroll
                for (int r = 0; r < 16; r++) bank[c][r] = fmaxf(bank[c][r], u[r]);
                if (G > 1) {
                    // tile maximum, a tree of 3-input maxima
                    const float a = fmaxf(fmaxf(u[0], u[1]), u[2]), b = fmaxf(fmaxf(u[3], u[4]), u[5]);
                    const float d = fmaxf(fmaxf(u[6], u[7]), u[8]), e = fmaxf(fmaxf(u[9], u[10]), u[11]);
                    const float g = fmaxf(fmaxf(u[12], u[13]), u[14]), q = fmaxf(fmaxf(u[15], a), b);
                    T[c][i] = fmaxf(fmaxf(q, d), fmaxf(e, g));
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int c = 0; c < NCOL; c++) hi[c].add_group(g0 / G, T[c]);
    }
}

// This lane's partial class maxima (the max counterpart of half_partials).
template <int MAXHI, int G>
__device__ __forceinline__ void half_partials_max(float* b, const HiMax<G, MAXHI>& hi, int m, float* p0,
                                                  float* p1) {
    p0[0] = fmaxf(fmaxf(fmaxf(b[0], b[2]), fmaxf(b[4], b[6])), fmaxf(fmaxf(b[8], b[10]), fmaxf(b[12], b[14])));
    p1[0] = fmaxf(fmaxf(fmaxf(b[1], b[3]), fmaxf(b[5], b[7])), fmaxf(fmaxf(b[9], b[11]), fmaxf(b[13], b[15])));
#pragma unroll
    for (int j = 0; j < 8; j++) b[j] = fmaxf(b[2 * j], b[2 * j + 1]);
    p0[1] = fmaxf(fmaxf(b[0], b[2]), fmaxf(b[4], b[6]));
    p1[1] = fmaxf(fmaxf(b[1], b[3]), fmaxf(b[5], b[7]));
#pragma unroll
    for (int j = 0; j < 4; j++) b[j] = fmaxf(b[2 * j], b[2 * j + 1]);
    p0[3] = fmaxf(b[0], b[2]);
    p1[3] = fmaxf(b[1], b[3]);
    p0[4] = fmaxf(b[0], b[1]);
    p1[4] = fmaxf(b[2], b[3]);
    p0[2] = p1[2] = fmaxf(p0[4], p1[4]);
#pragma unroll
    for (int k = 5; k < MDGMI_MAX_BITS; k++) {
        p0[k] = k < m ? hi.R0[k - 5] : 0.0f;
        p1[k] = k < m ? hi.R1[k - 5] : 0.0f;
    }
}

// Class maxima of label bit k over both halves, identical in every lane.
__device__ __forceinline__ void full_max(const float* p0, const float* p1, int k, float& U0, float& U1) {
    if (k == 2) {
        const Halves t = halves(p0[2]);
        U0 = t.lo;
        U1 = t.hi;
    } else {
        const Halves a = halves(p0[k]), b = halves(p1[k]);
        U0 = fmaxf(a.lo, a.hi);
        U1 = fmaxf(b.lo, b.hi);
    }
}

// One column tile with max-log metrics: MODE kModeMlLlr writes LLRs,
// kModeMlGmi adds the GMI cost of those LLRs to acc (no MI). A sample whose
// nearest point lies outside the exponent window, whose y is not finite, or
// (formats with padding rows, M < 32) whose class maximum could be a padding
// row, takes the FP32 per-class path.
template <int DIM, int NCOL, int G, int MODE, int S = kSplitF16>
__device__ __forceinline__ void mfma_coltile_ml(const uint4* __restrict__ A, const float* __restrict__ ys,
                                                const uint32_t* __restrict__ txs, int64_t n, int64_t ct, int M,
                                                int m, int ntiles, float s, const float* __restrict__ X32,
                                                const uint32_t* __restrict__ labels, float* __restrict__ llr,
                                                CostAcc& acc, float guard = 0.0f) {
    constexpr int NB = Blk<DIM, S>::value;
    constexpr int MAXHI = MDGMI_MAX_BITS - 5;
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, col = lane & 31;
    half8 bop[NCOL][NB];
    int64_t idx[NCOL];
    float Kc[NCOL];
    bool fin[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; c++) {
        idx[c] = (ct * NCOL + c) * 32 + col;
        const bool valid = idx[c] < n;
        float yv[DIM], ys2 = 0.0f;
        fin[c] = true;
#pragma unroll
        for (int d = 0; d < DIM; d++) {
            yv[d] = valid ? ys[idx[c] * DIM + d] : 0.0f;
            ys2 = fmaf(yv[d], yv[d], ys2);
            fin[c] = fin[c] && __builtin_isfinite(yv[d]);
        }
        Kc[c] = fmaf(-s, ys2, kBias);
        make_b<DIM, S>(yv, Kc[c], h, bop[c]);
    }
    float bank[NCOL][16];
    HiMax<G, MAXHI> hi[NCOL];
    tile_loop_max<DIM, NCOL, G, MAXHI, S>(A, ntiles, h, col, bop, bank, hi);
#pragma unroll
    for (int c = 0; c < NCOL; c++) {
        const int64_t i = idx[c];
        float p0[MDGMI_MAX_BITS], p1[MDGMI_MAX_BITS];
        half_partials_max<MAXHI, G>(bank[c], hi[c], m, p0, p1);
        float B0, B1;
        full_max(p0, p1, 2, B0, B1);
        const float best = fmaxf(B0, B1);
        bool far = !(best >= kFarLog2) || !fin[c];
        bool near0 = false;  // an LLR near zero at a large s (LLR output)
        float cg = 0.0f;
        constexpr int NJ = (MDGMI_MAX_BITS + 1) / 2;
        float lam[NJ];
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            lam[j] = 0.0f;
            if (2 * j < m) {  // uniform
                const int ke = 2 * j, ko = ke + 1 < MDGMI_MAX_BITS ? ke + 1 : ke;
                float U0e, U1e, U0o = 0.0f, U1o = 0.0f;
                full_max(p0, p1, ke, U0e, U1e);
                if (ko < m) full_max(p0, p1, ko, U0o, U1o);
                if (M < 32) {
                    // a class maximum near the padding rows' u = K - 60000
                    const float lim = Kc[c] - 0.5f * kPadNorm;
                    far = far || fminf(U0e, U1e) < lim || (ko < m && fminf(U0o, U1o) < lim);
                }
                const int k = ke + h;
                const float u0 = h ? U0o : U0e, u1 = h ? U1o : U1e;
                lam[j] = u1 - u0;  // log2 units
                if (MODE == kModeMlLlr && k < m) near0 = near0 || fabsf(lam[j]) < guard;
                if (MODE == kModeMlGmi && k < m) {
                    const uint32_t row = i < n ? txs[i] : 0u;
                    const uint32_t slot = labels[row < (uint32_t)M ? row : 0u];
                    cg += bit_cost2(((slot >> k) & 1) ? u0 - u1 : u1 - u0);
                }
            }
        }
        if (MODE == kModeMlGmi) cg = half_sum(cg);
        if (MODE == kModeMlLlr) {
            // either half's bits: both halves take the per-class path together
            const Halves hz = halves(near0 ? 1.0f : 0.0f);
            far = far || hz.lo + hz.hi > 0.0f;
        }
        if (i >= n) continue;
        if (!far) {
            if (MODE == kModeMlLlr) {
#pragma unroll
                for (int j = 0; j < NJ; j++) {
                    const int k = 2 * j + h;
                    if (k < m) llr[i * m + k] = lam[j] * (float)kLn2;
                }
            } else if (h == 0) {
                const uint32_t row = txs[i];
                acc.add(row < (uint32_t)M ? cg : NAN, 0.0f);
            }
            continue;
        }
        if (h != 0) continue;
        float yc[DIM], u0[MDGMI_MAX_BITS], u1[MDGMI_MAX_BITS];
#pragma unroll
        for (int d = 0; d < DIM; d++) yc[d] = ys[i * DIM + d];
        class_max_u_f32<DIM>(yc, X32, M, m, s, u0, u1);
        if (MODE == kModeMlLlr) {
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++)
                if (k < m) llr[i * m + k] = fin[c] ? (u1[k] - u0[k]) * (float)kLn2 : NAN;
        } else {
            const uint32_t row = txs[i];
            const bool row_ok = row < (uint32_t)M;
            const uint32_t slot = labels[row_ok ? row : 0u];
            float c2 = 0.0f;
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++)
                if (k < m) c2 += bit_cost2(((slot >> k) & 1) ? u0[k] - u1[k] : u1[k] - u0[k]);
            acc.add(row_ok && fin[c] ? c2 : NAN, 0.0f);
        }
    }
}

}  // namespace mfma
}  // namespace mdgmi
