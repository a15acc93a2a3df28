// FP32 exact demapper with the distance term on the vector ALUs.
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

namespace {

constexpr int kDirectThreads = 256;

template <int DIM>
struct DirectRec {
    static constexpr int value = ((DIM + 1 + 3) / 4) * 4;  // floats per point record
};

__global__ void k_direct_image(const double* __restrict__ X64, int M, int dim, int rec, SnrArgs sa,
                               float* __restrict__ img) {
    int q = blockIdx.y;
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    double s = sa.s64[q];
    double n2 = 0.0;
    float* r = img + ((size_t)q * M + j) * rec;
    for (int d = 0; d < dim; d++) {
        double x = X64[(size_t)j * dim + d];
        n2 += x * x;
        r[d] = (float)(2.0 * s * x);
    }
    r[dim] = (float)(s * n2);
    for (int d = dim + 1; d < rec; d++) r[d] = 0.0f;
}

template <int DIM, int CHB, int G, bool LLR>
__global__ __launch_bounds__(kDirectThreads) void k_direct(
    const float* __restrict__ y, const uint32_t* __restrict__ tx, const float* __restrict__ img,
    const float* __restrict__ X32, const uint32_t* __restrict__ labels, int64_t n, int M, int m, SnrArgs sa,
    float* __restrict__ llr, double* __restrict__ part) {
    constexpr int CH = 1 << CHB;
    constexpr int REC = DirectRec<DIM>::value;
    constexpr int MAXHI = MDGMI_MAX_BITS - CHB;
    const int q_snr = blockIdx.y;
    const float s = sa.s32[q_snr];
    const int64_t snr = sa.snr0 + q_snr;
    const float* __restrict__ im = img + (size_t)q_snr * M * REC;
    const float* ys = y + snr * n * DIM;
    const uint32_t* txs = LLR ? nullptr : tx + snr * n;
    const int nchunk = M >> CHB;
    CostAcc acc;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
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
            if (smin >= ex2(kFarLog2)) {
#pragma unroll
                for (int k = 0; k < MDGMI_MAX_BITS; k++)
                    if (k < m) llr[i * m + k] = log2_ratio(S1[k], S0[k], ls1[k], ls0[k]) * (float)kLn2;
            } else {
                // a class lies too far for the common offset (or y is not finite)
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
            const uint32_t slot = labels[row_ok ? row : 0u];
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
            }
            if (!row_ok) cg = cm = NAN;
            acc.add((double)cg, (double)cm);
        }
    }
    if (!LLR) block_reduce_store(acc, part + ((int64_t)q_snr * gridDim.x + blockIdx.x) * kNPart);
}

template <int DIM, int CHB, int G>
hipError_t launch_direct_t(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                           const SnrArgs& sa, bool llr_mode, float* llr, double* part, float* image,
                           LaunchCfg cfg, hipStream_t st) {
    dim3 grid(cfg.blocks_per_snr, sa.n_snr), block(cfg.threads);
    if (llr_mode)
        hipLaunchKernelGGL((k_direct<DIM, CHB, G, true>), grid, block, 0, st, y, tx, image, f->d_X32,
                           f->d_labels, n, f->M, f->m, sa, llr, part);
    else
        hipLaunchKernelGGL((k_direct<DIM, CHB, G, false>), grid, block, 0, st, y, tx, image, f->d_X32,
                           f->d_labels, n, f->M, f->m, sa, llr, part);
    return hipGetLastError();
}

template <int DIM>
hipError_t launch_direct_d(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                           const SnrArgs& sa, bool llr_mode, float* llr, double* part, float* image,
                           LaunchCfg cfg, hipStream_t st) {
    switch (f->m) {
        case 1:
            return launch_direct_t<DIM, 1, 1>(f, y, tx, n, sa, llr_mode, llr, part, image, cfg, st);
        case 2:
            return launch_direct_t<DIM, 2, 1>(f, y, tx, n, sa, llr_mode, llr, part, image, cfg, st);
        case 3:
            return launch_direct_t<DIM, 3, 1>(f, y, tx, n, sa, llr_mode, llr, part, image, cfg, st);
        case 4:
            return launch_direct_t<DIM, 4, 1>(f, y, tx, n, sa, llr_mode, llr, part, image, cfg, st);
        case 5:
            return launch_direct_t<DIM, 4, 2>(f, y, tx, n, sa, llr_mode, llr, part, image, cfg, st);
        default:
            return launch_direct_t<DIM, 4, 4>(f, y, tx, n, sa, llr_mode, llr, part, image, cfg, st);
    }
}

}  // namespace

size_t direct_image_bytes(const mdgmi_format* f, int n_snr) {
    int rec = ((f->dim + 1 + 3) / 4) * 4;
    return (size_t)n_snr * f->M * rec * sizeof(float);
}

LaunchCfg direct_cfg(const mdgmi_format* f, int64_t n) {
    (void)f;
    int64_t want = (n + kDirectThreads - 1) / kDirectThreads;
    int cap = device_cu_count() * 8;
    LaunchCfg c;
    c.threads = kDirectThreads;
    c.blocks_per_snr = (int)(want < cap ? (want < 1 ? 1 : want) : cap);
    return c;
}

hipError_t launch_direct(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                         const SnrArgs& sa, bool llr_mode, float* llr, double* part, float* image,
                         LaunchCfg cfg, hipStream_t st) {
    int rec = ((f->dim + 1 + 3) / 4) * 4;
    dim3 g((f->M + 255) / 256, sa.n_snr);
    hipLaunchKernelGGL(k_direct_image, g, dim3(256), 0, st, f->d_X64, f->M, f->dim, rec, sa, image);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (f->dim) {
        case 2:
            return launch_direct_d<2>(f, y, tx, n, sa, llr_mode, llr, part, image, cfg, st);
        case 4:
            return launch_direct_d<4>(f, y, tx, n, sa, llr_mode, llr, part, image, cfg, st);
        case 8:
            return launch_direct_d<8>(f, y, tx, n, sa, llr_mode, llr, part, image, cfg, st);
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace mdgmi
