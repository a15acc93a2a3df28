// FP32 exact demapper with the distance term on the matrix cores: per-SNR
// kernels over one format (see mfma_core.h for the arithmetic and layouts).
#include <algorithm>
#include <cmath>

#include "mfma_kernels.h"

namespace mdgmi {

namespace {

using namespace mfma;

struct MfmaVariant {
    int ncol, waves;
    bool lds;
};

int g_variant_override = -1;  // set through mdgmi_set_tuning for sweeps

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


// 32 x 32 launch shape for a launch of `total` samples over its SNR points.
int pick_variant(const mdgmi_format* f, int64_t total) {
    if (g_variant_override >= 0 && g_variant_override < kNumVariants) return g_variant_override;
    const int t = tuned_mfma_variant(f->dim, f->M, total);
    if (t >= 0 && t < kNumVariants) return t;
    // untuned: a large image leaves room for one block per CU, so 16 waves
    // per block fill the CU; small images run several 8-wave blocks per CU
    return image_bytes_per_snr(f) > 32 * 1024 ? 4 : 2;
}

// The per-sample 4x4 shape serves small fp16-split formats unless a 32 x 32
// variant is asked for (override or tuning table).
bool use_small(const mdgmi_format* f, int split, int64_t total) {
    if (split != kSplitF16 || !small_shape_fits(f)) return false;
    int v = g_variant_override;
    if (v < 0 || v >= kMfmaVariants) v = tuned_mfma_variant(f->dim, f->M, total);
    return v < 0 || v >= kMfmaVariants || v == kSmallVariant;
}

// Launch configuration of 32 x 32 shape var (-1: the bf16 split's
// two-column L2 shape).
LaunchCfg shape_cfg(const mdgmi_format* f, int64_t n, int n_snr, int split, int var) {
    const MfmaVariant wide{2, 8, false};
    const MfmaVariant& v = var < 0 ? wide : kVariants[var];
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
    c.variant = var;
    return c;
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
    const int64_t total = n * (int64_t)n_snr;
    if (use_small(f, split, total)) {
        LaunchCfg c = small_cfg(f, n, n_snr);
        c.variant = kSmallVariant;
        return c;
    }
    if (bf16_wide(f, split)) return shape_cfg(f, n, n_snr, split, -1);
    // hard decisions, max-log metrics, 1-D formats and the bf16 split run the
    // 1-column, 16-wave shape only (LDS image if it fits)
    const bool fixed = mode == kModeHd || mode_is_ml(mode) || f->dim == 1 || split == kSplitBF16;
    const int var = fixed ? (image_bytes_per_snr(f, split) <= 128 * 1024 ? 4 : 6) : pick_variant(f, total);
    return shape_cfg(f, n, n_snr, split, var);
}

int64_t mfma_blocks_bound(const mdgmi_format* f, int64_t n, int n_snr, int mode, int split) {
    // per shape, the blocks of a call over k of the n_snr points: the blocks
    // per point depend on k only up to kMaxSnrPerLaunch points per launch,
    // beyond which k times them grows with k, so k = 1..32 and k = n_snr
    int64_t b = (int64_t)n_snr * mfma_cfg(f, n, n_snr, mode, split).blocks_per_snr;
    for (int k = 1; k <= n_snr; k = (k < kMaxSnrPerLaunch || k == n_snr) ? k + 1 : n_snr) {
        if (split == kSplitF16 && small_shape_fits(f))
            b = std::max<int64_t>(b, (int64_t)k * small_cfg(f, n, k).blocks_per_snr);
        for (int v = -1; v < kNumVariants; v++)
            b = std::max<int64_t>(b, (int64_t)k * shape_cfg(f, n, k, split, v).blocks_per_snr);
    }
    return b;
}

template <int S>
hipError_t image_and_run(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n, const SnrArgs& sa,
                         int mode, float* llr, double* part, uint4* img, int ntiles, LaunchCfg cfg, hipStream_t st) {
    const bool tuned_shape = S == kSplitF16 && !(mode == kModeHd || mode_is_ml(mode) || f->dim == 1);
    MfmaShape shape{MfmaShape::kFixed, 0, image_bytes_per_snr(f, S) <= 128 * 1024};
    if (S == kSplitBF16 && bf16_wide(f, S)) {
        shape = {MfmaShape::kWide, 0, false};
    } else if (tuned_shape) {
        // the shape mfma_cfg chose for this launch (its block count matches)
        const int var = cfg.variant;
        if (var < 0 || var >= kNumVariants) return hipErrorInvalidValue;
        shape = {MfmaShape::kVariant, var, kVariants[var].lds && image_bytes_per_snr(f) <= 128 * 1024};
    }
    switch (f->dim) {
        case 1:
            return mfma_run<1, S>(f, y, tx, n, sa, mode, llr, part, img, ntiles, cfg, shape, st);
        case 2:
            return mfma_run<2, S>(f, y, tx, n, sa, mode, llr, part, img, ntiles, cfg, shape, st);
        case 4:
            return mfma_run<4, S>(f, y, tx, n, sa, mode, llr, part, img, ntiles, cfg, shape, st);
        case 8:
            return mfma_run<8, S>(f, y, tx, n, sa, mode, llr, part, img, ntiles, cfg, shape, st);
        default:
            return hipErrorInvalidValue;
    }
}

bool prefers_small(const mdgmi_format* f) { return use_small(f, kSplitF16, INT64_MAX); }

hipError_t launch_mfma(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                       const SnrArgs& sa, int mode, float* llr, double* part, void* image,
                       LaunchCfg cfg, hipStream_t st, int split) {
    const int ntiles = (f->M + 31) / 32;
    uint4* img = (uint4*)image;
    if (cfg.variant == kSmallVariant) return launch_small(f, y, tx, n, sa, mode, llr, part, image, cfg, st);
    if (split == kSplitBF16)
        return image_and_run<kSplitBF16>(f, y, tx, n, sa, mode, llr, part, img, ntiles, cfg, st);
    return image_and_run<kSplitF16>(f, y, tx, n, sa, mode, llr, part, img, ntiles, cfg, st);
}

}  // namespace mdgmi

extern "C" int mdgmi_set_tuning(int mfma_variant) {
    mdgmi::g_variant_override = mfma_variant;
    return 0;
}

extern "C" int mdgmi_get_tuning(void) { return mdgmi::g_variant_override; }
