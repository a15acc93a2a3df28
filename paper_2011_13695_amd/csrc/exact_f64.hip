// FP64 exact demapper: one lane per sample, every class with its own
// reference (its nearest point), so no class sum can underflow.
//
// Pass 1 over the constellation finds the per-class minima of
// t_j = ||y - x_j||^2 / (2 sigma2); pass 2 sums e^{cmin(k,b) - t_j} into the
// class of every label bit. The constellation is read through uniform
// (scalar) loads; the sample stays in registers.
#include "device_common.h"

namespace mdgmi {

namespace {

constexpr int kF64Threads = 256;

template <int DIM>
__device__ __forceinline__ double dist2(const double* yv, const double* __restrict__ X, int j) {
    double d = 0.0;
#pragma unroll
    for (int q = 0; q < DIM; q++) {
        double e = yv[q] - X[j * DIM + q];
        d = fma(e, e, d);
    }
    return d;
}

template <int DIM, int MODE>
__global__ __launch_bounds__(kF64Threads) void k_exact_f64(const double* __restrict__ y,
                                                           const uint32_t* __restrict__ tx,
                                                           const double* __restrict__ X,
                                                           const uint32_t* __restrict__ labels, int64_t n,
                                                           int M, int m, SnrArgs sa, double* __restrict__ llr,
                                                           double* __restrict__ part) {
    const int q_snr = blockIdx.y;
    const double inv2s2 = sa.inv2s2[q_snr];
    const int64_t snr = sa.snr0 + q_snr;
    const double* ys = y + snr * n * DIM;
    constexpr bool LLR = MODE == kModeLlr;
    const uint32_t* txs = mode_is_llr(MODE) ? nullptr : tx + snr * n;
    CostAcc acc;
    HdAcc hd;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double yv[DIM];
#pragma unroll
        for (int q = 0; q < DIM; q++) yv[q] = ys[i * DIM + q];
        // class (k, 0) and class (k, 1) kept in separate arrays: j is uniform,
        // so the bit tests below are uniform branches, not register indexing.
        double cmin0[MDGMI_MAX_BITS], cmin1[MDGMI_MAX_BITS];
#pragma unroll
        for (int k = 0; k < MDGMI_MAX_BITS; k++) cmin0[k] = cmin1[k] = INFINITY;
        double tmin = INFINITY;
        for (int j = 0; j < M; j++) {
            double t = dist2<DIM>(yv, X, j) * inv2s2;
            tmin = fmin(tmin, t);
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++) {
                if (k < m) {
                    if ((j >> k) & 1)
                        cmin1[k] = fmin(cmin1[k], t);
                    else
                        cmin0[k] = fmin(cmin0[k], t);
                }
            }
        }
        if (mode_is_ml(MODE)) {
            // max-log: lambda_k = min over class 0 of t - min over class 1 of t
            if (MODE == kModeMlLlr) {
#pragma unroll
                for (int k = 0; k < MDGMI_MAX_BITS; k++)
                    if (k < m) llr[i * m + k] = cmin0[k] - cmin1[k];
            } else {
                const uint32_t row = txs[i];
                const bool row_ok = row < (uint32_t)M;
                const uint32_t slot = labels[row_ok ? row : 0u];
                double cg = 0.0;
#pragma unroll
                for (int k = 0; k < MDGMI_MAX_BITS; k++) {
                    if (k < m) {
                        const double lam = cmin0[k] - cmin1[k];
                        const double u = ((slot >> k) & 1) ? -lam : lam;
                        cg += fmax(u, 0.0) + log1p(exp(-fabs(u)));
                    }
                }
                if (!row_ok) cg = NAN;
                acc.add(cg * kLog2e, 0.0);
            }
            continue;
        }
        double S0[MDGMI_MAX_BITS], S1[MDGMI_MAX_BITS];
#pragma unroll
        for (int k = 0; k < MDGMI_MAX_BITS; k++) S0[k] = S1[k] = 0.0;
        double tot = 0.0;
        for (int j = 0; j < M; j++) {
            double t = dist2<DIM>(yv, X, j) * inv2s2;
            tot += exp(tmin - t);
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++) {
                if (k < m) {
                    if ((j >> k) & 1)
                        S1[k] += exp(cmin1[k] - t);
                    else
                        S0[k] += exp(cmin0[k] - t);
                }
            }
        }
        // ln sum_{class} e^{-t} = ln S - cmin
        if (LLR) {
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++) {
                if (k < m) llr[i * m + k] = (log(S1[k]) - cmin1[k]) - (log(S0[k]) - cmin0[k]);
            }
        } else {
            // a sent row outside [0, M) gives a NaN cost instead of a stray read
            const uint32_t row = txs[i];
            const bool row_ok = row < (uint32_t)M;
            const uint32_t lw = labels[row_ok ? row : 0u];
            const uint32_t slot = lw & kLabelMask;
            double cg = 0.0;
#pragma unroll
            for (int k = 0; k < MDGMI_MAX_BITS; k++) {
                if (k < m) {
                    double l1 = log(S1[k]) - cmin1[k], l0 = log(S0[k]) - cmin0[k];
                    // u = ln S_(not sent) - ln S_(sent) ; cost = softplus(u)
                    double u = ((slot >> k) & 1) ? l0 - l1 : l1 - l0;
                    cg += fmax(u, 0.0) + log1p(exp(-fabs(u)));
                }
            }
            double ti = dist2<DIM>(yv, X, (int)slot) * inv2s2;
            double cm = ti - tmin + log(tot);
            if (!row_ok) cg = cm = NAN;
            acc.add(cg * kLog2e, cm * kLog2e);
            if (MODE == kModeHd) {
                // bitwise MAP decisions (sign of the LLR) and the nearest
                // point (some other point strictly nearer than the sent one,
                // or its coordinates shared with a lower label: ties go to
                // the lowest label)
                int be = 0;
#pragma unroll
                for (int k = 0; k < MDGMI_MAX_BITS; k++) {
                    if (k < m) {
                        const double lam = (log(S1[k]) - cmin1[k]) - (log(S0[k]) - cmin0[k]);
                        const int bk = (int)((slot >> k) & 1u);
                        be += (lam == lam) ? ((lam > 0.0 ? 1 : 0) != bk) : 1;
                    }
                }
                const bool finite = cg == cg && cm == cm;
                hd.be += finite ? (double)be : (double)m;
                const bool twin = (lw & kTwinBit) != 0u;
                hd.se += (finite && !(tmin < ti) && !twin) ? 0.0 : 1.0;
            }
        }
    }
    double* dst = part + ((int64_t)q_snr * gridDim.x + blockIdx.x) * (MODE == kModeHd ? kNPartHd : kNPart);
    if (MODE == kModeGmi || MODE == kModeMlGmi) block_reduce_store(acc, dst);
    if (MODE == kModeHd) block_reduce_store_hd(acc, hd, dst);
}

}  // namespace

LaunchCfg f64_cfg(const mdgmi_format* f, int64_t n) {
    (void)f;
    int64_t want = (n + kF64Threads - 1) / kF64Threads;
    int cap = device_cu_count() * 8;
    LaunchCfg c;
    c.threads = kF64Threads;
    c.blocks_per_snr = (int)(want < cap ? (want < 1 ? 1 : want) : cap);
    return c;
}

hipError_t launch_f64(const mdgmi_format* f, const double* y, const uint32_t* tx, int64_t n,
                      const SnrArgs& sa, int mode, double* llr, double* part, LaunchCfg cfg,
                      hipStream_t st) {
    dim3 grid(cfg.blocks_per_snr, sa.n_snr), block(cfg.threads);
    // part points at the first block row of this launch's first SNR.
#define MDGMI_F64_CASE(D)                                                                              \
    case D:                                                                                            \
        if (mode == kModeLlr)                                                                          \
            hipLaunchKernelGGL((k_exact_f64<D, kModeLlr>), grid, block, 0, st, y, tx, f->d_X64,       \
                               f->d_labels, n, f->M, f->m, sa, llr, part);                             \
        else if (mode == kModeHd)                                                                      \
            hipLaunchKernelGGL((k_exact_f64<D, kModeHd>), grid, block, 0, st, y, tx, f->d_X64,        \
                               f->d_labels_hd, n, f->M, f->m, sa, llr, part);                          \
        else if (mode == kModeMlLlr)                                                                   \
            hipLaunchKernelGGL((k_exact_f64<D, kModeMlLlr>), grid, block, 0, st, y, tx, f->d_X64,     \
                               f->d_labels, n, f->M, f->m, sa, llr, part);                             \
        else if (mode == kModeMlGmi)                                                                   \
            hipLaunchKernelGGL((k_exact_f64<D, kModeMlGmi>), grid, block, 0, st, y, tx, f->d_X64,     \
                               f->d_labels, n, f->M, f->m, sa, llr, part);                             \
        else                                                                                           \
            hipLaunchKernelGGL((k_exact_f64<D, kModeGmi>), grid, block, 0, st, y, tx, f->d_X64,       \
                               f->d_labels, n, f->M, f->m, sa, llr, part);                             \
        break;
    switch (f->dim) {
        MDGMI_F64_CASE(1)
        MDGMI_F64_CASE(2)
        MDGMI_F64_CASE(4)
        MDGMI_F64_CASE(8)
        default:
            return hipErrorInvalidValue;
    }
#undef MDGMI_F64_CASE
    return hipGetLastError();
}

}  // namespace mdgmi
