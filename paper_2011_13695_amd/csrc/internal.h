// Internal declarations of libmdgmi (HIP, gfx950). Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <cstddef>

#include "../../include/mdgmi.h"
#include "format_host.h"

struct mdgmi_format {
    int32_t M = 0, dim = 0, m = 0;
    int device = 0;
    // Label-ordered copies: slot j holds the point whose label is j, so the
    // label bits of a slot are the bits of its index.
    double* d_X64 = nullptr;      // [M][dim]
    float* d_X32 = nullptr;       // [M][dim]
    float* d_n32 = nullptr;       // [M] ||x||^2
    uint32_t* d_labels = nullptr; // [M] caller row -> label (= slot)
    // [M] as d_labels, with kTwinBit set on rows whose point has the same
    // coordinates as a point with a lower label (hard-decision launches read
    // this copy: the nearest-point decision goes to the lowest label)
    uint32_t* d_labels_hd = nullptr;
    double energy = 0.0;          // mean_j ||x_j||^2 (SNR = energy / (dim sigma2))
    // learned demapper attached by mdgmi_learned_calibrate (mlp.hip)
    struct LearnedBinding* learned = nullptr;
    double max_abs = 0.0;         // max_j,d |x_jd|
    double max_norm2 = 0.0;       // max_j ||x_j||^2
    double* h_X64 = nullptr;      // host copy, label-ordered [M][dim]
};

namespace mdgmi {

constexpr int kMfmaVariants = 9;     // MFMA launch shapes (see mdgmi_set_tuning)
constexpr int kSmallVariant = 8;     // ... the last: one sample per lane, 4x4 MFMA blocks
constexpr int kNPart = 5;           // per-block FP64 partials: sum cG, sum cG^2, sum cM, sum cM^2, nonfinite
constexpr int kNPartHd = kNPart + 2; // ... and, with hard decisions, bit errors and symbol errors
// What a demapper launch produces: GMI/MI partials, LLRs, or GMI/MI partials
// with hard-decision error counts.
constexpr int kModeGmi = 0, kModeLlr = 1, kModeHd = 2;
// max-log metrics: LLR output, or the GMI of those LLRs (no MI)
constexpr int kModeMlLlr = 3, kModeMlGmi = 4;
__host__ __device__ constexpr bool mode_is_llr(int mode) { return mode == kModeLlr || mode == kModeMlLlr; }
__host__ __device__ constexpr bool mode_is_ml(int mode) { return mode == kModeMlLlr || mode == kModeMlGmi; }
// what the final reduction writes: GMI/MI, + hard decisions, or GMI only
constexpr int kReduceGmi = 0, kReduceHd = 1, kReduceMl = 2;
constexpr int kMaxSnrPerLaunch = 32;
// Exponents are taken relative to a fixed offset: e_j = 2^(kBias - t_j) with
// t_j = ||y - x_j||^2 / (2 sigma2) * log2(e) >= 0, so no term can overflow
// (M * 2^kBias < 2^128) and any class whose nearest point lies within
// 2 * kBias of y is summed without underflow.
constexpr float kBias = 100.0f;
constexpr float kFarLog2 = -100.0f;  // class sums below 2^-100 take the per-class path
// LLR outputs at large s max||x||^2: u = K - s||x||^2 + <2 s x, y> cancels
// terms of that size, so an LLR carries an absolute error of up to about
// 2.3e-7 s max||x||^2 nats (fp16 split; FP32 rounding alone is a quarter of
// that). Above kLlrGuardS the LLR modes of the per-lane kernels recompute a
// sample on the per-class path (distances from differences) when one of
// its LLRs is below llr_guard() (log2 units), which keeps that error under
// half of the 1e-3 max(|lambda|, 1) bar: |lambda| > 4.6e-4 s max||x||^2
// nats, i.e. 6.6e-4 s max||x||^2 log2 units, and at least 3.
constexpr float kLlrGuardS = 1000.0f;
__host__ __device__ inline float llr_guard(float s, float max_n2) {
    const float sn = s * max_n2;
    return sn > kLlrGuardS ? fmaxf(3.0f, 6.6e-4f * sn) : 0.0f;
}
constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;

struct SnrArgs {
    int n_snr;                 // SNR points in this launch
    int snr0;                  // index of the first one in the caller's arrays
    float s32[kMaxSnrPerLaunch];   // s = log2(e) / (2 sigma2)
    double s64[kMaxSnrPerLaunch];
    double inv2s2[kMaxSnrPerLaunch];  // 1 / (2 sigma2)
};

struct LaunchCfg {
    int blocks_per_snr;
    int threads;
    int variant = -1;          // MFMA paths: the launch shape chosen by mfma_cfg
};

// ---- launchers (each in the .hip file holding the kernel) ----
hipError_t launch_generate(const mdgmi_format* f, uint64_t seed, const double* sigma2, int n_snr,
                           int64_t n, int snr_slot0, void* y, uint32_t* tx, bool f64, hipStream_t st);

LaunchCfg f64_cfg(const mdgmi_format* f, int64_t n);
hipError_t launch_f64(const mdgmi_format* f, const double* y, const uint32_t* tx, int64_t n,
                      const SnrArgs& sa, int mode, double* llr, double* part, LaunchCfg cfg,
                      hipStream_t st);

LaunchCfg direct_cfg(const mdgmi_format* f, int64_t n);
size_t direct_image_bytes(const mdgmi_format* f, int n_snr);
hipError_t launch_direct(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                         const SnrArgs& sa, int mode, float* llr, double* part, float* image,
                         LaunchCfg cfg, hipStream_t st);

// Per-sample 4x4-block shape of the fp16-split path for 4 <= M <= 512
// (8-D: M <= 256), exact_mfma4.hip; used by launch_mfma where it applies.
bool small_shape_fits(const mdgmi_format* f);
// whether the fp16-split path runs f on that shape in launches of many
// samples (tuning table, override): the ragged batch's choice
bool prefers_small(const mdgmi_format* f);
size_t small_image_bytes(const mdgmi_format* f, int n_snr);
LaunchCfg small_cfg(const mdgmi_format* f, int64_t n, int n_snr);
hipError_t launch_small(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n, const SnrArgs& sa,
                        int mode, float* llr, double* part, void* image, LaunchCfg cfg, hipStream_t st);

// split: 0 = fp16 hi + lo operands, 1 = bf16 in three parts (see mfma_core.h)
bool mfma_supported(const mdgmi_format* f, double max_s, int split = 0);
LaunchCfg mfma_cfg(const mdgmi_format* f, int64_t n, int n_snr, int mode = kModeGmi, int split = 0);
// the most blocks, over all SNR points, that any MFMA launch shape takes for
// n samples at n_snr points or at any subset of them: a partial-sum
// workspace that holds whichever shape the tuning table picks
int64_t mfma_blocks_bound(const mdgmi_format* f, int64_t n, int n_snr, int mode = kModeGmi, int split = 0);
size_t mfma_image_bytes(const mdgmi_format* f, int n_snr, int split = 0);
hipError_t launch_mfma(const mdgmi_format* f, const float* y, const uint32_t* tx, int64_t n,
                       const SnrArgs& sa, int mode, float* llr, double* part, void* image,
                       LaunchCfg cfg, hipStream_t st, int split = 0);

// Host-side planning shared by the entry points (api.hip).
size_t align_up(size_t v);
bool finite_pos(double v);
int check_device(const mdgmi_format* f);
// Resolve MDGMI_PATH_AUTO and check that the path can serve the format at
// the largest s = log2(e) / (2 sigma2) of the call; total = samples of the
// call over all its SNR points (selects the tuning regime).
int resolve_path(const mdgmi_format* f, int path, double max_s, int* out, int64_t total = INT64_MAX);
double s_of(double sigma2);
int part_stride(int mode);
struct GmiPlan {
    int path;
    LaunchCfg cfg;
    size_t part_bytes, image_bytes, total;
};
GmiPlan plan_gmi(const mdgmi_format* f, int64_t n, int n_snr, int path, int mode = kModeGmi);
SnrArgs snr_args(const double* sigma2, int q0, int cnt);
// One demapper launch on the resolved path (image built inside).
hipError_t launch_exact(const mdgmi_format* f, int path, const void* y, const uint32_t* tx, int64_t n,
                        const SnrArgs& sa, int mode, void* llr, double* part, void* image, LaunchCfg cfg,
                        hipStream_t st);

size_t sopt_workspace_bytes(int64_t n);
size_t bits_workspace_bytes(int64_t n);
hipError_t launch_bits(const mdgmi_format* f, const void* llr, bool f64, const uint32_t* tx, int64_t n, double* out,
                       void* ws, hipStream_t st);
hipError_t launch_sopt(const mdgmi_format* f, const void* llr, bool f64, const uint32_t* tx, int64_t n, double* out,
                       void* ws, hipStream_t st);
hipError_t launch_reduce(const double* part, int n_snr, int blocks_per_snr, int64_t n, int m,
                         double* out, hipStream_t st, int kind = kReduceGmi);

int device_cu_count();

// MDGMI_PATH_LEARNED_BF16 in mdgmi_gmi / mdgmi_llr and their workspace
// sizes (mlp.hip): the attached network where calibration routed the SNR
// point to it, the exact fallback path elsewhere.
int learned_gmi_workspace_size(const mdgmi_format* fmt, int64_t n, int32_t n_snr, size_t* bytes);
int learned_gmi(const mdgmi_format* fmt, const float* y, const uint32_t* tx_idx, int64_t n, const double* sigma2_host,
                int32_t n_snr, double* out, void* ws, size_t ws_bytes, void* stream);
int learned_llr_workspace_size(const mdgmi_format* fmt, int64_t n, size_t* bytes);
int learned_llr(const mdgmi_format* fmt, const float* y, int64_t n, double sigma2, float* llr, void* ws,
                size_t ws_bytes, void* stream);
void learned_free(mdgmi_format* fmt);

// mdgmi_gmi on a given workspace (the no-allocation entry point passes its
// static scratch array here)
int gmi_with_workspace(const mdgmi_format* fmt, const void* y, const uint32_t* tx_idx, int64_t n,
                       const double* sigma2_host, int32_t n_snr, int32_t path, double* out, void* ws, size_t ws_bytes,
                       void* stream);

// autotuner table (autotune.hip), per (dim, M) and sample-count regime of
// the launch (total samples over its SNR points below kTuneShortSamples:
// the short regime); -1 where (dim, M) is untuned
constexpr int64_t kTuneShortSamples = MDGMI_TUNE_SHORT_SAMPLES;
inline int tune_regime(int64_t total) { return total < kTuneShortSamples ? 1 : 0; }
int tuned_path(int dim, int M, int64_t total);
int tuned_mfma_variant(int dim, int M, int64_t total);

}  // namespace mdgmi
