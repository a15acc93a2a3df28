// Kernels and launch templates of the 32 x 32 MFMA demapper (arithmetic in
// mfma_core.h). Each (dimension, split) pair is instantiated in a source file
// of its own (exact_mfma_d<dim>_<split>.hip) so that they compile in parallel;
// exact_mfma.hip picks the shape and calls mfma_run.
#pragma once

#include "mfma_core.h"

namespace mdgmi {

// Launch shape chosen on the host: the tuned/default 32 x 32 variant (var,
// image in LDS or not), the fixed 1-column 16-wave shape, or the bf16
// split's two-column L2 shape.
struct MfmaShape {
    enum Kind { kVariant = 0, kFixed = 1, kWide = 2 } kind;
    int var;
    bool lds;
};

// Builds the per-SNR operand images, then runs the demapper kernel.
template <int DIM, int S>
hipError_t mfma_run(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n, const SnrArgs& sa, int mode,
                    float* llr, double* part, uint4* img, int ntiles, LaunchCfg cfg, MfmaShape shape, hipStream_t st);

#ifdef MDGMI_MFMA_KERNELS

namespace {

using namespace mfma;

// Per-SNR A images: [q][tile][blk][half][row].
template <int DIM, int S>
__global__ void k_mfma_image(const double* __restrict__ X64, int M, int ntiles, SnrArgs sa,
                             uint4* __restrict__ img) {
    constexpr int NB = Blk<DIM, S>::value;
    const int q = blockIdx.y;
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= ntiles * 32) return;
    image_slot<DIM, S>(X64, M, ntiles, sa.s64[q], slot, img + (size_t)q * ntiles * NB * 64);
}

template <int DIM, int NCOL, int WAVES, int G, bool LDS_IMG, int MODE, int S = kSplitF16>
__global__ __launch_bounds__(WAVES * 64) void k_mfma(
    const float* __restrict__ y, const uint32_t* __restrict__ tx, const uint4* __restrict__ img,
    const float* __restrict__ X32, const float* __restrict__ n32, const uint32_t* __restrict__ labels,
    int64_t n, int M, int m, int ntiles, SnrArgs sa, float max_n2, float* __restrict__ llr,
    double* __restrict__ part) {
    constexpr int NB = Blk<DIM, S>::value;
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
    const int wave = threadIdx.x >> 6;
    const float* ys = y + snr * n * DIM;
    const uint32_t* txs = mode_is_llr(MODE) ? nullptr : tx + snr * n;
    CostAcc acc;
    HdAcc hd;
    const float guard = mode_is_llr(MODE) ? llr_guard(s, max_n2) : 0.0f;
    const int64_t ncoltiles = (n + 32 * NCOL - 1) / (32 * NCOL);
    for (int64_t ct = (int64_t)blockIdx.x * WAVES + wave; ct < ncoltiles; ct += (int64_t)gridDim.x * WAVES) {
        if constexpr (mode_is_ml(MODE))
            mfma_coltile_ml<DIM, NCOL, G, MODE, S>(A, ys, txs, n, ct, M, m, ntiles, s, X32, labels, llr, acc,
                                                   guard);
        else
            mfma_coltile<DIM, NCOL, G, MODE, S>(A, ys, txs, n, ct, M, m, ntiles, s, X32, labels, llr, acc, &hd,
                                                guard);
    }
    (void)n32;
    double* dst = part + ((int64_t)q_snr * gridDim.x + blockIdx.x) * (MODE == kModeHd ? kNPartHd : kNPart);
    if (MODE == kModeGmi || MODE == kModeMlGmi) block_reduce_store(acc, dst);
    if (MODE == kModeHd) block_reduce_store_hd(acc, hd, dst);
}


template <int DIM, int NCOL, int WAVES, int G, bool LDS, int MODE, int S = kSplitF16>
hipError_t launch_vm(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n, const SnrArgs& sa,
                     float* llr, double* part, const uint4* img, int ntiles, int blocks, hipStream_t st) {
    constexpr int NB = Blk<DIM, S>::value;
    dim3 grid(blocks, sa.n_snr), block(WAVES * 64);
    size_t lds = LDS ? (size_t)ntiles * NB * 64 * sizeof(uint4) : 0;
    if (LDS) {
        hipError_t e = hipFuncSetAttribute((const void*)k_mfma<DIM, NCOL, WAVES, G, true, MODE, S>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_mfma<DIM, NCOL, WAVES, G, LDS, MODE, S>), grid, block, lds, st, y, tx, img, f->d_X32,
                       f->d_n32, MODE == kModeHd ? f->d_labels_hd : f->d_labels, n, f->M, f->m, ntiles, sa,
                       (float)f->max_norm2, llr, part);
    return hipGetLastError();
}

// GMI and LLR modes in every launch shape; hard decisions and max-log
// metrics only in the 1-column, 16-wave shape (launch_fixed).
template <int DIM, int NCOL, int WAVES, int G, bool LDS>
hipError_t launch_v(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n, const SnrArgs& sa,
                    int mode, float* llr, double* part, const uint4* img, int ntiles, int blocks,
                    hipStream_t st) {
    if (mode == kModeLlr)
        return launch_vm<DIM, NCOL, WAVES, G, LDS, kModeLlr>(f, y, tx, n, sa, llr, part, img, ntiles, blocks, st);
    return launch_vm<DIM, NCOL, WAVES, G, LDS, kModeGmi>(f, y, tx, n, sa, llr, part, img, ntiles, blocks, st);
}

template <int DIM, int MODE, int S>
hipError_t launch_fixed_m(bool lds, const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                          const SnrArgs& sa, float* llr, double* part, const uint4* img, int ntiles, int blocks,
                          hipStream_t st) {
#define MDGMI_FIXED_G(G)                                                                                       \
    return lds ? launch_vm<DIM, 1, 16, G, true, MODE, S>(f, y, tx, n, sa, llr, part, img, ntiles, blocks, st)  \
               : launch_vm<DIM, 1, 16, G, false, MODE, S>(f, y, tx, n, sa, llr, part, img, ntiles, blocks, st);
    if (ntiles >= 8) {
        MDGMI_FIXED_G(8)
    } else if (ntiles == 4) {
        MDGMI_FIXED_G(4)
    } else if (ntiles == 2) {
        MDGMI_FIXED_G(2)
    } else {
        MDGMI_FIXED_G(1)
    }
#undef MDGMI_FIXED_G
}

template <int DIM, int S = kSplitF16>
hipError_t launch_fixed(int mode, bool lds, const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                        const SnrArgs& sa, float* llr, double* part, const uint4* img, int ntiles, int blocks,
                        hipStream_t st) {
    if (mode == kModeGmi)
        return launch_fixed_m<DIM, kModeGmi, S>(lds, f, y, tx, n, sa, llr, part, img, ntiles, blocks, st);
    if (mode == kModeLlr)
        return launch_fixed_m<DIM, kModeLlr, S>(lds, f, y, tx, n, sa, llr, part, img, ntiles, blocks, st);
    if (mode == kModeHd)
        return launch_fixed_m<DIM, kModeHd, S>(lds, f, y, tx, n, sa, llr, part, img, ntiles, blocks, st);
    if (mode == kModeMlLlr)
        return launch_fixed_m<DIM, kModeMlLlr, S>(lds, f, y, tx, n, sa, llr, part, img, ntiles, blocks, st);
    return launch_fixed_m<DIM, kModeMlGmi, S>(lds, f, y, tx, n, sa, llr, part, img, ntiles, blocks, st);
}

// Variants (sample columns per wave, waves per block, A image in LDS):
// 0 = (1, 4), 1 = (2, 4), 2 = (1, 8), 3 = (2, 8), 4 = (1, 16), 5 = (1, 12)
// staged in LDS when the image fits; 6 = (1, 16), 7 = (1, 8) reading it from
// L2.
template <int DIM>
hipError_t launch_d(int var, bool lds, const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                    const SnrArgs& sa, int mode, float* llr, double* part, const uint4* img, int ntiles,
                    int blocks, hipStream_t st) {
#define MDGMI_VG(NC, W, G)                                                                                  \
    return lds ? launch_v<DIM, NC, W, G, true>(f, y, tx, n, sa, mode, llr, part, img, ntiles, blocks, st) \
               : launch_v<DIM, NC, W, G, false>(f, y, tx, n, sa, mode, llr, part, img, ntiles, blocks, st);
#define MDGMI_V(NC, W)             \
    if (ntiles >= 8) {             \
        MDGMI_VG(NC, W, 8)         \
    } else if (ntiles == 4) {      \
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
        case 3:
            MDGMI_V(2, 8)
        case 4:
        case 6:
            MDGMI_V(1, 16)
        case 5:
            MDGMI_V(1, 12)
        default:
            MDGMI_V(1, 8)
    }
#undef MDGMI_V
#undef MDGMI_VG
}

// bf16 images above the LDS budget are read from L2, 4 KB per tile and wave
// for 8-D: two sample columns per wave halve that traffic (8 waves per block
// for the registers). Such images have at least 32 tiles, so G = 8.
template <int DIM, int S>
hipError_t launch_wide_l2(int mode, const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                          const SnrArgs& sa, float* llr, double* part, const uint4* img, int ntiles, int blocks,
                          hipStream_t st) {
    switch (mode) {
        case kModeGmi:
            return launch_vm<DIM, 2, 8, 8, false, kModeGmi, S>(f, y, tx, n, sa, llr, part, img, ntiles, blocks, st);
        case kModeLlr:
            return launch_vm<DIM, 2, 8, 8, false, kModeLlr, S>(f, y, tx, n, sa, llr, part, img, ntiles, blocks, st);
        case kModeHd:
            return launch_vm<DIM, 2, 8, 8, false, kModeHd, S>(f, y, tx, n, sa, llr, part, img, ntiles, blocks, st);
        case kModeMlLlr:
            return launch_vm<DIM, 2, 8, 8, false, kModeMlLlr, S>(f, y, tx, n, sa, llr, part, img, ntiles, blocks,
                                                                  st);
        default:
            return launch_vm<DIM, 2, 8, 8, false, kModeMlGmi, S>(f, y, tx, n, sa, llr, part, img, ntiles, blocks,
                                                                  st);
    }
}

}  // namespace

template <int DIM, int S>
hipError_t mfma_run(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n, const SnrArgs& sa, int mode,
                    float* llr, double* part, uint4* img, int ntiles, LaunchCfg cfg, MfmaShape shape, hipStream_t st) {
    const dim3 g((ntiles * 32 + 255) / 256, sa.n_snr);
    hipLaunchKernelGGL((k_mfma_image<DIM, S>), g, dim3(256), 0, st, f->d_X64, f->M, ntiles, sa, img);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int b = cfg.blocks_per_snr;
    if constexpr (DIM > 1) {
        if (shape.kind == MfmaShape::kWide)
            return launch_wide_l2<DIM, S>(mode, f, y, tx, n, sa, llr, part, img, ntiles, b, st);
        if constexpr (S == kSplitF16) {
            if (shape.kind == MfmaShape::kVariant)
                return launch_d<DIM>(shape.var, shape.lds, f, y, tx, n, sa, mode, llr, part, img, ntiles, b, st);
        }
    }
    if (shape.kind != MfmaShape::kFixed) return hipErrorInvalidValue;
    return launch_fixed<DIM, S>(mode, shape.lds, f, y, tx, n, sa, llr, part, img, ntiles, b, st);
}

#endif  // MDGMI_MFMA_KERNELS

}  // namespace mdgmi
