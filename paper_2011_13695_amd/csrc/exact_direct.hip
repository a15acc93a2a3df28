// FP32 exact demapper with the distance term on the vector ALUs: per-SNR
// kernels over one format (see direct_core.h for the arithmetic).
#include "direct_core.h"

namespace mdgmi {

namespace {

using namespace direct;

constexpr int kDirectThreads = 256;

template <int DIM, int CHB, int G, int MODE>
__global__ __launch_bounds__(kDirectThreads) void k_direct(
    const float* __restrict__ y, const uint32_t* __restrict__ tx, const float* __restrict__ img,
    const float* __restrict__ X32, const uint32_t* __restrict__ labels, int64_t n, int M, int m, SnrArgs sa,
    float max_n2, float* __restrict__ llr, double* __restrict__ part) {
    constexpr int REC = DirectRec<DIM>::value;
    const int q_snr = blockIdx.y;
    const float s = sa.s32[q_snr];
    const int64_t snr = sa.snr0 + q_snr;
    const float* __restrict__ im = img + (size_t)q_snr * M * REC;
    const float* ys = y + snr * n * DIM;
    const uint32_t* txs = mode_is_llr(MODE) ? nullptr : tx + snr * n;
    CostAcc acc;
    HdAcc hd;
    const float guard = mode_is_llr(MODE) ? llr_guard(s, max_n2) : 0.0f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if constexpr (mode_is_ml(MODE))
            direct_sample_ml<DIM, CHB, G, MODE>(im, ys, txs, i, M, m, s, X32, labels, llr, acc, guard);
        else
            direct_sample<DIM, CHB, G, MODE>(im, ys, txs, i, M, m, s, X32, labels, llr, acc, &hd, guard);
    }
    double* dst = part + ((int64_t)q_snr * gridDim.x + blockIdx.x) * (MODE == kModeHd ? kNPartHd : kNPart);
    if (MODE == kModeGmi || MODE == kModeMlGmi) block_reduce_store(acc, dst);
    if (MODE == kModeHd) block_reduce_store_hd(acc, hd, dst);
}

__global__ void k_direct_image(const double* __restrict__ X64, int M, int dim, int rec, SnrArgs sa,
                               float* __restrict__ img) {
    const int q = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    direct_record(X64, dim, rec, sa.s64[q], j, img + ((size_t)q * M + j) * rec);
}


template <int DIM, int CHB, int G>
hipError_t launch_direct_t(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                           const SnrArgs& sa, int mode, float* llr, double* part, float* image,
                           LaunchCfg cfg, hipStream_t st) {
    dim3 grid(cfg.blocks_per_snr, sa.n_snr), block(cfg.threads);
    if (mode == kModeLlr)
        hipLaunchKernelGGL((k_direct<DIM, CHB, G, kModeLlr>), grid, block, 0, st, y, tx, image, f->d_X32,
                           f->d_labels, n, f->M, f->m, sa, (float)f->max_norm2, llr, part);
    else if (mode == kModeMlLlr)
        hipLaunchKernelGGL((k_direct<DIM, CHB, G, kModeMlLlr>), grid, block, 0, st, y, tx, image, f->d_X32,
                           f->d_labels, n, f->M, f->m, sa, (float)f->max_norm2, llr, part);
    else if (mode == kModeMlGmi)
        hipLaunchKernelGGL((k_direct<DIM, CHB, G, kModeMlGmi>), grid, block, 0, st, y, tx, image, f->d_X32,
                           f->d_labels, n, f->M, f->m, sa, (float)f->max_norm2, llr, part);
    else if (mode == kModeHd)
        hipLaunchKernelGGL((k_direct<DIM, CHB, G, kModeHd>), grid, block, 0, st, y, tx, image, f->d_X32,
                           f->d_labels_hd, n, f->M, f->m, sa, (float)f->max_norm2, llr, part);
    else
        hipLaunchKernelGGL((k_direct<DIM, CHB, G, kModeGmi>), grid, block, 0, st, y, tx, image, f->d_X32,
                           f->d_labels, n, f->M, f->m, sa, (float)f->max_norm2, llr, part);
    return hipGetLastError();
}

template <int DIM>
hipError_t launch_direct_d(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                           const SnrArgs& sa, int mode, float* llr, double* part, float* image,
                           LaunchCfg cfg, hipStream_t st) {
    switch (f->m) {
        case 1:
            return launch_direct_t<DIM, 1, 1>(f, y, tx, n, sa, mode, llr, part, image, cfg, st);
        case 2:
            return launch_direct_t<DIM, 2, 1>(f, y, tx, n, sa, mode, llr, part, image, cfg, st);
        case 3:
            return launch_direct_t<DIM, 3, 1>(f, y, tx, n, sa, mode, llr, part, image, cfg, st);
        case 4:
            return launch_direct_t<DIM, 4, 1>(f, y, tx, n, sa, mode, llr, part, image, cfg, st);
        case 5:
            return launch_direct_t<DIM, 4, 2>(f, y, tx, n, sa, mode, llr, part, image, cfg, st);
        default:
            return launch_direct_t<DIM, 4, 4>(f, y, tx, n, sa, mode, llr, part, image, cfg, st);
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
                         const SnrArgs& sa, int mode, float* llr, double* part, float* image,
                         LaunchCfg cfg, hipStream_t st) {
    int rec = ((f->dim + 1 + 3) / 4) * 4;
    dim3 g((f->M + 255) / 256, sa.n_snr);
    hipLaunchKernelGGL(k_direct_image, g, dim3(256), 0, st, f->d_X64, f->M, f->dim, rec, sa, image);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (f->dim) {
        case 1:
            return launch_direct_d<1>(f, y, tx, n, sa, mode, llr, part, image, cfg, st);
        case 2:
            return launch_direct_d<2>(f, y, tx, n, sa, mode, llr, part, image, cfg, st);
        case 4:
            return launch_direct_d<4>(f, y, tx, n, sa, mode, llr, part, image, cfg, st);
        case 8:
            return launch_direct_d<8>(f, y, tx, n, sa, mode, llr, part, image, cfg, st);
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace mdgmi
