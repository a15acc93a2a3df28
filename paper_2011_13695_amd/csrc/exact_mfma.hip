// FP32 exact demapper with the distance term on the matrix cores: per-SNR
// kernels over one format (see mfma_core.h for the arithmetic and layouts).
#include <algorithm>
#include <cmath>

#include "mfma_core.h"

namespace mdgmi {

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


struct MfmaVariant {
    int ncol, waves;
    bool lds;
};

int g_variant_override = -1;  // set through mdgmi_set_tuning for sweeps

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

constexpr int kNumVariants = 8;  // 32 x 32 shapes; kSmallVariant follows them
const MfmaVariant kVariants[kNumVariants] = {{1, 4, true},  {2, 4, true},  {1, 8, true},  {2, 8, true},
                                             {1, 16, true}, {1, 12, true}, {1, 16, false}, {1, 8, false}};

int blocks_of(int dim, int split) {
    if (split == kSplitBF16) return (6 * dim + 6 + 15) / 16;
    return dim == 8 ? 2 : 1;
}

size_t image_bytes_per_snr(const mdgmi_format* f, int split = kSplitF16) {
    int ntiles = (f->M + 31) / 32;
    return (size_t)ntiles * blocks_of(f->dim, split) * 64 * sizeof(uint4);
}

bool bf16_wide(const mdgmi_format* f, int split) {
    return split == kSplitBF16 && f->dim > 1 && image_bytes_per_snr(f, split) > 128 * 1024;
}


int pick_variant(const mdgmi_format* f) {
    if (g_variant_override >= 0 && g_variant_override < kNumVariants) return g_variant_override;
    const int t = tuned_mfma_variant(f->dim, f->M);
    if (t >= 0 && t < kNumVariants) return t;
    // untuned: a large image leaves room for one block per CU, so 16 waves
    // per block fill the CU; small images run several 8-wave blocks per CU
    return image_bytes_per_snr(f) > 32 * 1024 ? 4 : 2;
}

// The per-sample 4x4 shape serves small fp16-split formats unless a 32 x 32
// variant is asked for (override or tuning table).
bool use_small(const mdgmi_format* f, int split) {
    if (split != kSplitF16 || !small_shape_fits(f)) return false;
    int v = g_variant_override;
    if (v < 0 || v >= kMfmaVariants) v = tuned_mfma_variant(f->dim, f->M);
    return v < 0 || v >= kMfmaVariants || v == kSmallVariant;
}

}  // namespace

bool mfma_supported(const mdgmi_format* f, double max_s, int split) {
    // fp16 range of the split factors: 2 s |x| and s ||x||^2 must stay well
    // inside 65504 (the per-sample term K is checked in the kernel's range
    // through the far-point path). bf16 has the FP32 exponent range.
    if (split == kSplitBF16) return std::isfinite(max_s) && std::isfinite(f->max_norm2);
    return 2.0 * max_s * f->max_abs < 30000.0 && max_s * f->max_norm2 < 30000.0;
}

size_t mfma_image_bytes(const mdgmi_format* f, int n_snr, int split) {
    const size_t big = (size_t)n_snr * image_bytes_per_snr(f, split);
    // either shape may run (the choice follows tuning), so size for both
    if (split == kSplitF16 && small_shape_fits(f)) return std::max(big, small_image_bytes(f, n_snr));
    return big;
}

LaunchCfg mfma_cfg(const mdgmi_format* f, int64_t n, int n_snr, int mode, int split) {
    if (use_small(f, split)) return small_cfg(f, n, n_snr);
    // hard decisions, max-log metrics, 1-D formats and the bf16 split run the
    // 1-column, 16-wave shape only (LDS image if it fits)
    const bool fixed = mode == kModeHd || mode_is_ml(mode) || f->dim == 1 || split == kSplitBF16;
    const int var = fixed ? (image_bytes_per_snr(f, split) <= 128 * 1024 ? 4 : 6) : pick_variant(f);
    const MfmaVariant wide{2, 8, false};
    const MfmaVariant& v = bf16_wide(f, split) ? wide : kVariants[var];
    const int64_t cols = 32 * v.ncol;
    const int64_t tiles = (n + cols - 1) / cols;
    const int64_t want = (tiles + v.waves - 1) / v.waves;
    // One resident round of blocks over all CUs: blocks per CU limited by
    // the LDS image (160 KiB per CU) and by a target of 16 waves per CU.
    const size_t img = image_bytes_per_snr(f, split);
    const bool lds = v.lds && img <= 128 * 1024;
    const int by_lds = lds ? std::max(1, (int)((160 * 1024) / (img + 2048))) : 8;
    const int by_waves = std::max(1, 16 / v.waves);
    const int64_t total = (int64_t)device_cu_count() * std::min(by_lds, by_waves);
    const int snr_in_launch = n_snr < kMaxSnrPerLaunch ? n_snr : kMaxSnrPerLaunch;
    int64_t per = std::max<int64_t>(1, total / snr_in_launch);
    per = std::min<int64_t>(per, std::max<int64_t>(1, want));
    LaunchCfg c;
    c.threads = v.waves * 64;
    c.blocks_per_snr = (int)per;
    return c;
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

template <int S>
hipError_t image_and_fixed(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n, const SnrArgs& sa,
                           int mode, float* llr, double* part, uint4* img, int ntiles, LaunchCfg cfg,
                           hipStream_t st) {
    dim3 g((ntiles * 32 + 255) / 256, sa.n_snr);
    switch (f->dim) {
        case 1:
            hipLaunchKernelGGL((k_mfma_image<1, S>), g, dim3(256), 0, st, f->d_X64, f->M, ntiles, sa, img);
            break;
        case 2:
            hipLaunchKernelGGL((k_mfma_image<2, S>), g, dim3(256), 0, st, f->d_X64, f->M, ntiles, sa, img);
            break;
        case 4:
            hipLaunchKernelGGL((k_mfma_image<4, S>), g, dim3(256), 0, st, f->d_X64, f->M, ntiles, sa, img);
            break;
        case 8:
            hipLaunchKernelGGL((k_mfma_image<8, S>), g, dim3(256), 0, st, f->d_X64, f->M, ntiles, sa, img);
            break;
        default:
            return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const bool tuned_shape = S == kSplitF16 && !(mode == kModeHd || mode_is_ml(mode) || f->dim == 1);
    if (S == kSplitBF16 && bf16_wide(f, S)) {
        const int b = cfg.blocks_per_snr;
        switch (f->dim) {
            case 2:
                return launch_wide_l2<2, S>(mode, f, y, tx, n, sa, llr, part, img, ntiles, b, st);
            case 4:
                return launch_wide_l2<4, S>(mode, f, y, tx, n, sa, llr, part, img, ntiles, b, st);
            default:
                return launch_wide_l2<8, S>(mode, f, y, tx, n, sa, llr, part, img, ntiles, b, st);
        }
    }
    if (!tuned_shape) {
        const bool flds = image_bytes_per_snr(f, S) <= 128 * 1024;
        const int b = cfg.blocks_per_snr;
        switch (f->dim) {
            case 1:
                return launch_fixed<1, S>(mode, flds, f, y, tx, n, sa, llr, part, img, ntiles, b, st);
            case 2:
                return launch_fixed<2, S>(mode, flds, f, y, tx, n, sa, llr, part, img, ntiles, b, st);
            case 4:
                return launch_fixed<4, S>(mode, flds, f, y, tx, n, sa, llr, part, img, ntiles, b, st);
            default:
                return launch_fixed<8, S>(mode, flds, f, y, tx, n, sa, llr, part, img, ntiles, b, st);
        }
    }
    const int var = pick_variant(f);
    const bool lds = kVariants[var].lds && image_bytes_per_snr(f) <= 128 * 1024;
    switch (f->dim) {
        case 2:
            return launch_d<2>(var, lds, f, y, tx, n, sa, mode, llr, part, img, ntiles, cfg.blocks_per_snr, st);
        case 4:
            return launch_d<4>(var, lds, f, y, tx, n, sa, mode, llr, part, img, ntiles, cfg.blocks_per_snr, st);
        default:
            return launch_d<8>(var, lds, f, y, tx, n, sa, mode, llr, part, img, ntiles, cfg.blocks_per_snr, st);
    }
}

bool prefers_small(const mdgmi_format* f) { return use_small(f, kSplitF16); }

hipError_t launch_mfma(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                       const SnrArgs& sa, int mode, float* llr, double* part, void* image,
                       LaunchCfg cfg, hipStream_t st, int split) {
    const int ntiles = (f->M + 31) / 32;
    uint4* img = (uint4*)image;
    if (use_small(f, split)) return launch_small(f, y, tx, n, sa, mode, llr, part, image, cfg, st);
    if (split == kSplitBF16)
        return image_and_fixed<kSplitBF16>(f, y, tx, n, sa, mode, llr, part, img, ntiles, cfg, st);
    return image_and_fixed<kSplitF16>(f, y, tx, n, sa, mode, llr, part, img, ntiles, cfg, st);
}

}  // namespace mdgmi

extern "C" int mdgmi_set_tuning(int mfma_variant) {
    mdgmi::g_variant_override = mfma_variant;
    return 0;
}

extern "C" int mdgmi_get_tuning(void) { return mdgmi::g_variant_override; }
