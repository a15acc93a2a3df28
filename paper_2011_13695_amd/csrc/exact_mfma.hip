// FP32 exact demapper with the distance term on the matrix cores.
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
// with x' = 2 s x, n = s ||x||^2 and K = kBias - s ||y||^2.
//
// Output layout of the 32x32 MFMA: lane l, register r holds row
// p = 8 (r >> 2) + 4 (l >> 5) + (r & 3) of column l & 31. With points stored
// in label order, label bits 0, 1, 3, 4 of the point are bits of r, bit 2 is
// the lane half and bits 5.. are the tile index. Each lane keeps a running
// bank[r] of its 16 exponentials (one add per pair) and adds the tile total
// (15 adds per 16 pairs) to the classes of the tile-index bits; the two lane
// halves are combined once per sample at the end.
#include "device_common.h"

namespace mdgmi {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr float kPadNorm = 60000.0f;   // padding rows: u = K - 60000 -> e = 0

template <int DIM>
struct Blk {
    static constexpr int value = DIM == 8 ? 2 : 1;
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

// Per-SNR A image: [q][tile][blk][half][row] of 8 halves (16 bytes).
template <int DIM>
__global__ void k_mfma_image(const double* __restrict__ X64, int M, int ntiles, SnrArgs sa,
                             uint4* __restrict__ img) {
    constexpr int NB = Blk<DIM>::value;
    const int q = blockIdx.y;
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= ntiles * 32) return;
    const int t = slot >> 5, row = slot & 31;
    const double s = sa.s64[q];
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
    } else {
        a[0][0].h[0] = xh[0];
        a[0][0].h[1] = xh[1];
        a[0][0].h[2] = xl[0];
        a[0][0].h[3] = xl[1];
        a[0][0].h[4] = xh[0];
        a[0][0].h[5] = xh[1];
        a[0][1].h[0] = nh;
        a[0][1].h[1] = nl;
        a[0][1].h[2] = one;
        a[0][1].h[3] = one;
    }
    uint4* base = img + (size_t)q * ntiles * NB * 64;
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
        for (int h = 0; h < 2; h++) base[((t * NB + b) * 2 + h) * 32 + row] = a[b][h].u;
}

// B operands of one sample column for lane half h.
template <int DIM>
__device__ __forceinline__ void make_b(const float* yv, float K, int h, half8* bop) {
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
    } else {
        if (!h) {
            b0.h[0] = yh[0];
            b0.h[1] = yh[1];
            b0.h[2] = yh[0];
            b0.h[3] = yh[1];
            b0.h[4] = yl[0];
            b0.h[5] = yl[1];
        } else {
            b0.h[0] = one;
            b0.h[1] = one;
            b0.h[2] = kh;
            b0.h[3] = kl;
        }
        bop[0] = b0.v;
    }
}

template <int DIM, int NCOL, int WAVES, int G, bool LDS_IMG, bool LLR>
__global__ __launch_bounds__(WAVES * 64) void k_mfma(
    const float* __restrict__ y, const uint32_t* __restrict__ tx, const uint4* __restrict__ img,
    const float* __restrict__ X32, const float* __restrict__ n32, const uint32_t* __restrict__ labels,
    int64_t n, int M, int m, int ntiles, SnrArgs sa, float* __restrict__ llr, double* __restrict__ part) {
    constexpr int NB = Blk<DIM>::value;
    constexpr int MAXHI = MDGMI_MAX_BITS - 5;
    extern __shared__ uint4 lds_img[];
    const int q_snr = blockIdx.y;
    const float s = sa.s32[q_snr];
    const int64_t snr = sa.snr0 + q_snr;
    const uint4* __restrict__ gimg = img + (size_t)q_snr * ntiles * NB * 64;
    if (LDS_IMG) {
        const int cnt = ntiles * NB * 64;
        for (int k = threadIdx.x; k < cnt; k += blockDim.x) lds_img[k] = gimg[k];
        __syncthreads();
    }
    const uint4* A = LDS_IMG ? lds_img : gimg;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, col = lane & 31;
    const float* ys = y + snr * n * DIM;
    const uint32_t* txs = LLR ? nullptr : tx + snr * n;
    CostAcc acc;
    const int64_t ncoltiles = (n + 32 * NCOL - 1) / (32 * NCOL);
    for (int64_t ct = (int64_t)blockIdx.x * WAVES + wave; ct < ncoltiles; ct += (int64_t)gridDim.x * WAVES) {
        half8 bop[NCOL][NB];
        float yv[NCOL][DIM], Kc[NCOL];
        int64_t idx[NCOL];
#pragma unroll
        for (int c = 0; c < NCOL; c++) {
            idx[c] = (ct * NCOL + c) * 32 + col;
            const bool valid = idx[c] < n;
            float ys2 = 0.0f;
#pragma unroll
            for (int d = 0; d < DIM; d++) {
                yv[c][d] = valid ? ys[idx[c] * DIM + d] : 0.0f;
                ys2 = fmaf(yv[c][d], yv[c][d], ys2);
            }
            const float K = kBias - s * ys2;
            Kc[c] = K;
            make_b<DIM>(yv[c], K, h, bop[c]);
        }
        float bank[NCOL][16];
        HiAcc<G, MAXHI> hi[NCOL];
#pragma unroll
        for (int c = 0; c < NCOL; c++) {
#pragma unroll
            for (int r = 0; r < 16; r++) bank[c][r] = 0.0f;
            hi[c].zero();
        }
        for (int g0 = 0; g0 < ntiles; g0 += G) {
            float T[NCOL][G];
#pragma unroll
            for (int i = 0; i < G; i++) {
                const int t = g0 + i;
                half8 a[NB];
#pragma unroll
                for (int b = 0; b < NB; b++) {
                    H8 tmp;
                    tmp.u = A[((t * NB + b) * 2 + h) * 32 + col];
                    a[b] = tmp.v;
                }
#pragma unroll
                for (int c = 0; c < NCOL; c++) {
                    f32x16 u = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[0], bop[c][0], (f32x16){}, 0, 0, 0);
                    if (NB == 2) u = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[NB - 1], bop[c][NB - 1], u, 0, 0, 0);
                    float ev[16];
#pragma unroll
                    for (int r = 0; r < 16; r++) {
                        ev[r] = ex2(u[r]);
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
            }
#pragma unroll
            for (int c = 0; c < NCOL; c++) hi[c].add_group(g0 / G, T[c]);
        }
        // ---- epilogue: class sums, LLRs / costs ----
#pragma unroll
        for (int c = 0; c < NCOL; c++) {
            // lane-local sums over the row bits held in r: label bits 0,1,3,4
            float L0[4], L1[4], Lt = 0.0f;
#pragma unroll
            for (int q = 0; q < 4; q++) L0[q] = L1[q] = 0.0f;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                Lt += bank[c][r];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    if ((r >> q) & 1)
                        L1[q] += bank[c][r];
                    else
                        L0[q] += bank[c][r];
                }
            }
            float S0[MDGMI_MAX_BITS], S1[MDGMI_MAX_BITS];
            const int rbit_of_label[5] = {0, 1, -1, 2, 3};
#pragma unroll
            for (int k = 0; k < 5; k++) {
                if (k == 2) {
                    const float ot = __shfl_xor(Lt, 32, 64);
                    S0[2] = h ? ot : Lt;
                    S1[2] = h ? Lt : ot;
                } else {
                    const int q = rbit_of_label[k];
                    S0[k] = L0[q] + __shfl_xor(L0[q], 32, 64);
                    S1[k] = L1[q] + __shfl_xor(L1[q], 32, 64);
                }
            }
#pragma unroll
            for (int l = 0; l < MAXHI; l++) {
                S0[5 + l] = hi[c].R0[l] + __shfl_xor(hi[c].R0[l], 32, 64);
                S1[5 + l] = hi[c].R1[l] + __shfl_xor(hi[c].R1[l], 32, 64);
            }
            const float tot = Lt + __shfl_xor(Lt, 32, 64);
            if (h == 0 && idx[c] < n) {
                const int64_t i = idx[c];
                float ls0[MDGMI_MAX_BITS], ls1[MDGMI_MAX_BITS];
                float smin = INFINITY;
#pragma unroll
                for (int k = 0; k < MDGMI_MAX_BITS; k++) {
                    if (k < m) {
                        smin = fminf(smin, fminf(S0[k], S1[k]));
                        ls0[k] = lg2(S0[k]);
                        ls1[k] = lg2(S1[k]);
                    }
                }
                if (LLR) {
                    if (smin >= ex2(kFarLog2)) {
#pragma unroll
                        for (int k = 0; k < MDGMI_MAX_BITS; k++)
                            if (k < m) llr[i * m + k] = log2_ratio(S1[k], S0[k], ls1[k], ls0[k]) * (float)kLn2;
                    } else {
                        float ltot, ti;
                        exact_classes_f32<DIM>(yv[c], X32, M, m, s, -1, ls0, ls1, ltot, ti);
#pragma unroll
                        for (int k = 0; k < MDGMI_MAX_BITS; k++)
                            if (k < m) llr[i * m + k] = (ls1[k] - ls0[k]) * (float)kLn2;
                    }
                } else {
                    // a sent row outside [0, M) gives a NaN cost instead of a stray read
                    const uint32_t row = txs[i];
                    const bool row_ok = row < (uint32_t)M;
                    const uint32_t slot = labels[row_ok ? row : 0u];
                    // u of the sent point from the very fp16 operands the MFMA saw
                    // (every product is exact in FP32), so that the MI cost
                    // log2 sum_j 2^(u_j - u_i) is free of the split rounding
                    float ui = 0.0f;
                    {
                        half8 bb[2][NB];
                        make_b<DIM>(yv[c], Kc[c], 0, bb[0]);
                        make_b<DIM>(yv[c], Kc[c], 1, bb[1]);
                        const int ti = (int)(slot >> 5), pi = (int)(slot & 31);
#pragma unroll
                        for (int b = 0; b < NB; b++) {
#pragma unroll
                            for (int hh = 0; hh < 2; hh++) {
                                H8 av, bv;
                                av.u = A[((ti * NB + b) * 2 + hh) * 32 + pi];
                                bv.v = bb[hh][b];
#pragma unroll
                                for (int q = 0; q < 8; q++) ui = fmaf((float)av.h[q], (float)bv.h[q], ui);
                            }
                        }
                    }
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
                        float ltot, ti = 0.0f;
                        exact_classes_f32<DIM>(yv[c], X32, M, m, s, (int)slot, ls0, ls1, ltot, ti);
#pragma unroll
                        for (int k = 0; k < MDGMI_MAX_BITS; k++) {
                            if (k < m) {
                                bool b = (slot >> k) & 1;
                                cg += bit_cost2(b ? ls0[k] - ls1[k] : ls1[k] - ls0[k]);
                            }
                        }
                        cm = ltot + ti;
                    }
                    if (!row_ok) cg = cm = NAN;
                    acc.add((double)cg, (double)cm);
                }
            }
        }
    }
    if (!LLR) block_reduce_store(acc, part + ((int64_t)q_snr * gridDim.x + blockIdx.x) * kNPart);
}

struct MfmaVariant {
    int ncol, waves;
    bool lds;
};

int g_variant_override = -1;  // set through mdgmi_set_tuning for sweeps

template <int DIM, int NCOL, int WAVES, int G, bool LDS>
hipError_t launch_v(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n, const SnrArgs& sa,
                    bool llr_mode, float* llr, double* part, const uint4* img, int ntiles, int blocks,
                    hipStream_t st) {
    constexpr int NB = Blk<DIM>::value;
    dim3 grid(blocks, sa.n_snr), block(WAVES * 64);
    size_t lds = LDS ? (size_t)ntiles * NB * 64 * sizeof(uint4) : 0;
    if (LDS) {
        auto kfn = llr_mode ? (const void*)k_mfma<DIM, NCOL, WAVES, G, true, true>
                            : (const void*)k_mfma<DIM, NCOL, WAVES, G, true, false>;
        hipError_t e = hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (llr_mode)
        hipLaunchKernelGGL((k_mfma<DIM, NCOL, WAVES, G, LDS, true>), grid, block, lds, st, y, tx, img, f->d_X32,
                           f->d_n32, f->d_labels, n, f->M, f->m, ntiles, sa, llr, part);
    else
        hipLaunchKernelGGL((k_mfma<DIM, NCOL, WAVES, G, LDS, false>), grid, block, lds, st, y, tx, img, f->d_X32,
                           f->d_n32, f->d_labels, n, f->M, f->m, ntiles, sa, llr, part);
    return hipGetLastError();
}

// Variants: 0 = (1 col, 4 waves), 1 = (2 cols, 4 waves), 2 = (1 col, 8 waves),
// 3 = (2 cols, 8 waves); LDS staging when the image fits.
template <int DIM>
hipError_t launch_d(int var, bool lds, const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                    const SnrArgs& sa, bool llr_mode, float* llr, double* part, const uint4* img, int ntiles,
                    int blocks, hipStream_t st) {
#define MDGMI_VG(NC, W, G)                                                                                  \
    return lds ? launch_v<DIM, NC, W, G, true>(f, y, tx, n, sa, llr_mode, llr, part, img, ntiles, blocks, st) \
               : launch_v<DIM, NC, W, G, false>(f, y, tx, n, sa, llr_mode, llr, part, img, ntiles, blocks, st);
#define MDGMI_V(NC, W)             \
    if (ntiles >= 4) {             \
        MDGMI_VG(NC, W, 4)         \
    } else if (ntiles == 2) {      \
        MDGMI_VG(NC, W, 2)         \
    } else {                       \
        MDGMI_VG(NC, W, 1)         \
    }
    switch (var) {
        case 0:
            MDGMI_V(1, 4)
        case 1:
            MDGMI_V(2, 4)
        case 2:
            MDGMI_V(1, 8)
        default:
            MDGMI_V(2, 8)
    }
#undef MDGMI_V
#undef MDGMI_VG
}

const MfmaVariant kVariants[4] = {{1, 4, true}, {2, 4, true}, {1, 8, true}, {2, 8, true}};

int pick_variant(const mdgmi_format* f) {
    if (g_variant_override >= 0 && g_variant_override < 4) return g_variant_override;
    (void)f;
    return 3;
}

size_t image_bytes_per_snr(const mdgmi_format* f) {
    int ntiles = (f->M + 31) / 32;
    return (size_t)ntiles * (f->dim == 8 ? 2 : 1) * 64 * sizeof(uint4);
}

}  // namespace

bool mfma_supported(const mdgmi_format* f, double max_s) {
    // fp16 range of the split factors: 2 s |x| and s ||x||^2 must stay well
    // inside 65504 (the per-sample term K is checked in the kernel's range
    // through the far-point path).
    return 2.0 * max_s * f->max_abs < 30000.0 && max_s * f->max_norm2 < 30000.0;
}

size_t mfma_image_bytes(const mdgmi_format* f, int n_snr) { return (size_t)n_snr * image_bytes_per_snr(f); }

LaunchCfg mfma_cfg(const mdgmi_format* f, int64_t n, int n_snr) {
    const MfmaVariant& v = kVariants[pick_variant(f)];
    const int64_t cols = 32 * v.ncol;
    const int64_t tiles = (n + cols - 1) / cols;
    int64_t want = (tiles + v.waves - 1) / v.waves;
    // about 4 waves per SIMD in total, spread over the SNR points of a launch
    int64_t cap = (int64_t)device_cu_count() * 16 / v.waves;
    int snr_in_launch = n_snr < kMaxSnrPerLaunch ? n_snr : kMaxSnrPerLaunch;
    cap = (cap + snr_in_launch - 1) / snr_in_launch;
    if (cap < 1) cap = 1;
    LaunchCfg c;
    c.threads = v.waves * 64;
    c.blocks_per_snr = (int)(want < cap ? (want < 1 ? 1 : want) : cap);
    return c;
}

hipError_t launch_mfma(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                       const SnrArgs& sa, bool llr_mode, float* llr, double* part, void* image,
                       LaunchCfg cfg, hipStream_t st) {
    const int ntiles = (f->M + 31) / 32;
    uint4* img = (uint4*)image;
    dim3 g((ntiles * 32 + 255) / 256, sa.n_snr);
    switch (f->dim) {
        case 2:
            hipLaunchKernelGGL(k_mfma_image<2>, g, dim3(256), 0, st, f->d_X64, f->M, ntiles, sa, img);
            break;
        case 4:
            hipLaunchKernelGGL(k_mfma_image<4>, g, dim3(256), 0, st, f->d_X64, f->M, ntiles, sa, img);
            break;
        case 8:
            hipLaunchKernelGGL(k_mfma_image<8>, g, dim3(256), 0, st, f->d_X64, f->M, ntiles, sa, img);
            break;
        default:
            return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int var = pick_variant(f);
    const bool lds = image_bytes_per_snr(f) <= 128 * 1024;
    switch (f->dim) {
        case 2:
            return launch_d<2>(var, lds, f, y, tx, n, sa, llr_mode, llr, part, img, ntiles, cfg.blocks_per_snr, st);
        case 4:
            return launch_d<4>(var, lds, f, y, tx, n, sa, llr_mode, llr, part, img, ntiles, cfg.blocks_per_snr, st);
        default:
            return launch_d<8>(var, lds, f, y, tx, n, sa, llr_mode, llr, part, img, ntiles, cfg.blocks_per_snr, st);
    }
}

}  // namespace mdgmi

extern "C" int mdgmi_set_tuning(int mfma_variant) {
    mdgmi::g_variant_override = mfma_variant;
    return 0;
}
