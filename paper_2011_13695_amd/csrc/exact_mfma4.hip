// Per-SNR kernels of the per-sample 4x4-block MFMA demapper for small
// constellations (the arithmetic is in small_core.h).
#include <algorithm>

#include "small_core.h"

namespace mdgmi {

namespace {

using namespace small;

// largest formats served: at these sizes the shape still beat 32 x 32 tiles
// (4-D M = 512: 0.339 against 0.355 ms; 8-D M = 256: 0.232 against 0.264 ms
// for 2^22 samples)
constexpr int kSmallMaxM = 512, kSmallMaxM8 = 256;

template <int DIM>
__global__ void k_small_image(const double* __restrict__ X64, int M, SnrArgs sa, uint2* __restrict__ img) {
    const int q = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    image_slot<DIM>(X64, sa.s64[q], j, img + ((size_t)q * M + j) * Nk4<DIM>::value);
}

template <int DIM, int NG, int MODE>
__global__ __launch_bounds__(kSmallThreads) void k_small(const float* __restrict__ y, const uint32_t* __restrict__ tx,
                                                         const uint2* __restrict__ img, const float* __restrict__ X32,
                                                         const uint32_t* __restrict__ labels, int64_t n, SnrArgs sa,
                                                         float max_n2, float* __restrict__ llr,
                                                         double* __restrict__ part) {
    constexpr int NK = Nk4<DIM>::value;
    constexpr int M = 4 * NG;
    // the wave index is uniform: keep the batch loop on the scalar unit
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q_snr = blockIdx.y;
    const float s = sa.s32[q_snr];
    const int64_t snr = sa.snr0 + q_snr;
    const uint2* __restrict__ gimg = img + (size_t)q_snr * M * NK;
    const float* ys = y + snr * n * DIM;
    const uint32_t* txs = mode_is_llr(MODE) ? nullptr : tx + snr * n;
    half4 a[Sets<NG>::value][NK];
    load_image<DIM, NG>(gimg, M, a);
    CostAcc acc;
    HdAcc hd;
    const float guard = mode_is_llr(MODE) ? llr_guard(s, max_n2) : 0.0f;
    const int waves = kSmallThreads / 64;
    const int64_t nbat = (n + 63) / 64;
    // wave-uniform loop over batches of 64 consecutive samples
    for (int64_t b = (int64_t)blockIdx.x * waves + wave; b < nbat; b += (int64_t)gridDim.x * waves)
        small_sample<DIM, NG, MODE>(a, gimg, ys, txs, b * 64 + lane, n, s, X32, labels, llr, acc, hd, guard);
    double* dst = part + ((int64_t)q_snr * gridDim.x + blockIdx.x) * (MODE == kModeHd ? kNPartHd : kNPart);
    if (MODE == kModeGmi || MODE == kModeMlGmi) block_reduce_store(acc, dst);
    if (MODE == kModeHd) block_reduce_store_hd(acc, hd, dst);
}

template <int DIM, int NG>
hipError_t launch_small_t(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n, const SnrArgs& sa,
                          int mode, float* llr, double* part, const uint2* img, int blocks, hipStream_t st) {
    const dim3 grid(blocks, sa.n_snr), block(kSmallThreads);
#define MDGMI_SMALL(MD)                                                                                      \
    hipLaunchKernelGGL((k_small<DIM, NG, MD>), grid, block, 0, st, y, tx, img, f->d_X32,                    \
                       MD == kModeHd ? f->d_labels_hd : f->d_labels, n, sa, (float)f->max_norm2, llr, part); \
    break;
    switch (mode) {
        case kModeLlr:
            MDGMI_SMALL(kModeLlr)
        case kModeHd:
            MDGMI_SMALL(kModeHd)
        case kModeMlLlr:
            MDGMI_SMALL(kModeMlLlr)
        case kModeMlGmi:
            MDGMI_SMALL(kModeMlGmi)
        default:
            MDGMI_SMALL(kModeGmi)
    }
#undef MDGMI_SMALL
    return hipGetLastError();
}

template <int DIM>
hipError_t launch_small_d(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n, const SnrArgs& sa,
                          int mode, float* llr, double* part, const uint2* img, int blocks, hipStream_t st) {
    switch (f->M) {
        case 4:
            return launch_small_t<DIM, 1>(f, y, tx, n, sa, mode, llr, part, img, blocks, st);
        case 8:
            return launch_small_t<DIM, 2>(f, y, tx, n, sa, mode, llr, part, img, blocks, st);
        case 16:
            return launch_small_t<DIM, 4>(f, y, tx, n, sa, mode, llr, part, img, blocks, st);
        case 32:
            return launch_small_t<DIM, 8>(f, y, tx, n, sa, mode, llr, part, img, blocks, st);
        case 64:
            return launch_small_t<DIM, 16>(f, y, tx, n, sa, mode, llr, part, img, blocks, st);
        case 128:
            return launch_small_t<DIM, 32>(f, y, tx, n, sa, mode, llr, part, img, blocks, st);
        case 256:
            return launch_small_t<DIM, 64>(f, y, tx, n, sa, mode, llr, part, img, blocks, st);
        default:
            if constexpr (DIM < 8) {
                if (f->M == 512) return launch_small_t<DIM, 128>(f, y, tx, n, sa, mode, llr, part, img, blocks, st);
            }
            return hipErrorInvalidValue;
    }
}

}  // namespace

bool small_shape_fits(const mdgmi_format* f) {
    const int M = f->M;
    return M >= 4 && (M & (M - 1)) == 0 && (f->dim < 8 ? M <= kSmallMaxM : M <= kSmallMaxM8) &&
           (f->dim == 1 || f->dim == 2 || f->dim == 4 || f->dim == 8);
}

size_t small_image_bytes(const mdgmi_format* f, int n_snr) {
    const int nk = (3 * f->dim + 2 + 3) / 4;
    return (size_t)n_snr * f->M * nk * sizeof(uint2);
}

LaunchCfg small_cfg(const mdgmi_format* f, int64_t n, int n_snr) {
    (void)f;
    const int64_t batches = (n + 63) / 64;
    const int64_t want = (batches + kSmallThreads / 64 - 1) / (kSmallThreads / 64);
    // about four blocks per CU over the launch's SNR points
    const int snr_in_launch = n_snr < kMaxSnrPerLaunch ? n_snr : kMaxSnrPerLaunch;
    int64_t per = std::max<int64_t>(1, (int64_t)device_cu_count() * 4 / snr_in_launch);
    per = std::min<int64_t>(per, std::max<int64_t>(1, want));
    LaunchCfg c;
    c.threads = kSmallThreads;
    c.blocks_per_snr = (int)per;
    return c;
}

hipError_t launch_small(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n, const SnrArgs& sa,
                        int mode, float* llr, double* part, void* image, LaunchCfg cfg, hipStream_t st) {
    if (!small_shape_fits(f)) return hipErrorInvalidValue;
    uint2* img = (uint2*)image;
    const dim3 g((f->M + 63) / 64, sa.n_snr);
    switch (f->dim) {
        case 1:
            hipLaunchKernelGGL(k_small_image<1>, g, dim3(64), 0, st, f->d_X64, f->M, sa, img);
            break;
        case 2:
            hipLaunchKernelGGL(k_small_image<2>, g, dim3(64), 0, st, f->d_X64, f->M, sa, img);
            break;
        case 4:
            hipLaunchKernelGGL(k_small_image<4>, g, dim3(64), 0, st, f->d_X64, f->M, sa, img);
            break;
        default:
            hipLaunchKernelGGL(k_small_image<8>, g, dim3(64), 0, st, f->d_X64, f->M, sa, img);
            break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int b = cfg.blocks_per_snr;
    switch (f->dim) {
        case 1:
            return launch_small_d<1>(f, y, tx, n, sa, mode, llr, part, img, b, st);
        case 2:
            return launch_small_d<2>(f, y, tx, n, sa, mode, llr, part, img, b, st);
        case 4:
            return launch_small_d<4>(f, y, tx, n, sa, mode, llr, part, img, b, st);
        default:
            return launch_small_d<8>(f, y, tx, n, sa, mode, llr, part, img, b, st);
    }
}

}  // namespace mdgmi
