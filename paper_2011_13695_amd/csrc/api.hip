// C ABI of libmdgmi: argument checks on the host, format staging, workspace
// carving and kernel dispatch. Every check happens before the first launch.
#include <algorithm>
#include <limits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace mdgmi {

int device_cu_count() {
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> g(mu);
    if (cache[dev] == 0) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
            cu = 256;
        cache[dev] = cu;
    }
    return cache[dev];
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int check_device(const mdgmi_format* f) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return MDGMI_E_HIP;
    return dev == f->device ? MDGMI_OK : MDGMI_E_DEVICE;
}

// Resolve MDGMI_PATH_AUTO and check that the path can serve the format at
// the largest s = log2(e) / (2 sigma2) of the call.
int resolve_path(const mdgmi_format* f, int path, double max_s, int* out, int64_t total) {
    switch (path) {
        case MDGMI_PATH_F64:
        case MDGMI_PATH_F32_DIRECT:
            *out = path;
            return MDGMI_OK;
        case MDGMI_PATH_F32_MFMA_F16SPLIT:
            if (!mfma_supported(f, max_s)) return MDGMI_E_UNSUPPORTED;
            *out = path;
            return MDGMI_OK;
        case MDGMI_PATH_F32_MFMA_BF16SPLIT:
            if (!mfma_supported(f, max_s, 1)) return MDGMI_E_UNSUPPORTED;
            *out = path;
            return MDGMI_OK;
        case MDGMI_PATH_AUTO: {
            const bool small = small_shape_fits(f);
            const bool mfma_ok = (f->M >= 32 || small) && mfma_supported(f, max_s);
            const int t = tuned_path(f->dim, f->M, total);
            // untuned: the per-sample 4x4 shape for small formats, the 32 x 32
            // shape from 128 points; between them the vector-ALU kernel
            const bool want_mfma = t == MDGMI_PATH_F32_MFMA_F16SPLIT || (t < 0 && (f->M >= 128 || small));
            if (t == MDGMI_PATH_F32_DIRECT)
                *out = t;
            else if (want_mfma && mfma_ok)
                *out = MDGMI_PATH_F32_MFMA_F16SPLIT;
            else if (want_mfma && f->M >= 128 && mfma_supported(f, max_s, 1))
                *out = MDGMI_PATH_F32_MFMA_BF16SPLIT;  // beyond the fp16 range: the bf16 split
            else
                *out = MDGMI_PATH_F32_DIRECT;
            return MDGMI_OK;
        }
        default:
            return MDGMI_E_ARG;
    }
}

double s_of(double sigma2) { return kLog2e / (2.0 * sigma2); }

int part_stride(int mode) { return mode == kModeHd ? kNPartHd : kNPart; }

GmiPlan plan_gmi(const mdgmi_format* f, int64_t n, int n_snr, int path, int mode) {
    GmiPlan p{};
    p.path = path;
    const int per_launch = std::min(n_snr, kMaxSnrPerLaunch);
    if (path == MDGMI_PATH_F64) {
        p.cfg = f64_cfg(f, n);
        p.image_bytes = 0;
    } else if (path == MDGMI_PATH_F32_DIRECT) {
        p.cfg = direct_cfg(f, n);
        p.image_bytes = direct_image_bytes(f, per_launch);
    } else {
        const int split = path == MDGMI_PATH_F32_MFMA_BF16SPLIT ? 1 : 0;
        p.cfg = mfma_cfg(f, n, n_snr, mode, split);
        p.image_bytes = mfma_image_bytes(f, per_launch, split);
    }
    int64_t blocks = (int64_t)n_snr * p.cfg.blocks_per_snr;
    // MFMA launch shapes follow the tuning table, per sample-count regime:
    // room for whichever shape a call over these samples (or a subset of
    // the SNR points) may take
    if (path == MDGMI_PATH_F32_MFMA_F16SPLIT || path == MDGMI_PATH_F32_MFMA_BF16SPLIT)
        blocks = std::max(blocks, mfma_blocks_bound(f, n, n_snr, mode, path == MDGMI_PATH_F32_MFMA_BF16SPLIT ? 1 : 0));
    p.part_bytes = (size_t)blocks * part_stride(mode) * sizeof(double);
    p.total = align_up(p.part_bytes) + align_up(p.image_bytes);
    return p;
}

SnrArgs snr_args(const double* sigma2, int q0, int cnt) {
    SnrArgs sa{};
    sa.n_snr = cnt;
    sa.snr0 = q0;
    for (int q = 0; q < cnt; q++) {
        const double s2 = sigma2[q0 + q];
        sa.s64[q] = s_of(s2);
        sa.s32[q] = (float)sa.s64[q];
        sa.inv2s2[q] = 1.0 / (2.0 * s2);
    }
    return sa;
}

hipError_t launch_exact(const mdgmi_format* f, int path, const void* y, const uint32_t* tx, int64_t n,
                        const SnrArgs& sa, int mode, void* llr, double* part, void* image, LaunchCfg cfg,
                        hipStream_t st) {
    if (path == MDGMI_PATH_F64)
        return launch_f64(f, (const double*)y, tx, n, sa, mode, (double*)llr, part, cfg, st);
    if (path == MDGMI_PATH_F32_DIRECT)
        return launch_direct(f, (const float*)y, tx, n, sa, mode, (float*)llr, part, (float*)image, cfg, st);
    return launch_mfma(f, (const float*)y, tx, n, sa, mode, (float*)llr, part, image, cfg, st,
                       path == MDGMI_PATH_F32_MFMA_BF16SPLIT ? 1 : 0);
}

namespace {


int gmi_workspace_size(const mdgmi_format* fmt, int64_t n, int32_t n_snr, int32_t path, int mode, size_t* bytes) {
    if (!fmt || !bytes) return MDGMI_E_NULL;
    if (n < 1 || n_snr < 1) return MDGMI_E_SHAPE;
    int p = path;
    if (p == MDGMI_PATH_AUTO) p = MDGMI_PATH_F32_MFMA_F16SPLIT;
    if (p != MDGMI_PATH_F64 && p != MDGMI_PATH_F32_DIRECT && p != MDGMI_PATH_F32_MFMA_F16SPLIT &&
        p != MDGMI_PATH_F32_MFMA_BF16SPLIT)
        return MDGMI_E_ARG;
    GmiPlan pl = plan_gmi(fmt, n, n_snr, p, mode);
    // AUTO resolves per call (format size, tuning, fp16 range); size for
    // whichever of the two FP32 paths it may take.
    if (path == MDGMI_PATH_AUTO)
        pl.total = std::max({pl.total, plan_gmi(fmt, n, n_snr, MDGMI_PATH_F32_DIRECT, mode).total,
                             plan_gmi(fmt, n, n_snr, MDGMI_PATH_F32_MFMA_BF16SPLIT, mode).total});
    // mdgmi_gmi_maxlog shares mdgmi_gmi's size: its launch shape may differ
    if (mode == kModeGmi) {
        size_t ml = 0;
        gmi_workspace_size(fmt, n, n_snr, path, kModeMlGmi, &ml);
        pl.total = std::max(pl.total, ml);
    }
    *bytes = pl.total;
    return MDGMI_OK;
}

// One pass over n samples at n_snr noise levels: per-block partial sums
// (launches of at most kMaxSnrPerLaunch SNR points), then the FP64 reduce.
int run_gmi(const mdgmi_format* fmt, const void* y, const uint32_t* tx_idx, int64_t n, const double* sigma2_host,
            int32_t n_snr, int32_t path, int mode, double* out, void* ws, size_t ws_bytes, void* stream) {
    if (!fmt || !y || !tx_idx || !sigma2_host || !out) return MDGMI_E_NULL;
    if (n < 1 || n_snr < 1) return MDGMI_E_SHAPE;
    double max_s = 0.0;
    for (int q = 0; q < n_snr; q++) {
        if (!finite_pos(sigma2_host[q])) return MDGMI_E_SIGMA2;
        max_s = std::max(max_s, s_of(sigma2_host[q]));
    }
    int p = 0;
    int rc = resolve_path(fmt, path, max_s, &p, n * (int64_t)n_snr);
    if (rc != MDGMI_OK) return rc;
    GmiPlan pl = plan_gmi(fmt, n, n_snr, p, mode);
    if (!ws || ws_bytes < pl.total) return MDGMI_E_WORKSPACE;
    rc = check_device(fmt);
    if (rc != MDGMI_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    double* part = (double*)ws;
    void* image = (char*)ws + align_up(pl.part_bytes);
    for (int q0 = 0; q0 < n_snr; q0 += kMaxSnrPerLaunch) {
        const int cnt = std::min(kMaxSnrPerLaunch, n_snr - q0);
        SnrArgs sa = snr_args(sigma2_host, q0, cnt);
        double* pq = part + (size_t)q0 * pl.cfg.blocks_per_snr * part_stride(mode);
        if (launch_exact(fmt, p, y, tx_idx, n, sa, mode, nullptr, pq, image, pl.cfg, st) != hipSuccess)
            return MDGMI_E_HIP;
    }
    const int kind = mode == kModeHd ? kReduceHd : (mode == kModeMlGmi ? kReduceMl : kReduceGmi);
    hipError_t e = launch_reduce(part, n_snr, pl.cfg.blocks_per_snr, n, fmt->m, out, st, kind);
    return e == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}


// Per-bit LLRs of n samples at one noise level (exact or max-log metrics).
int run_llr(const mdgmi_format* fmt, const void* y, int64_t n, double sigma2, void* llr, int32_t path, int mode,
            void* ws, size_t ws_bytes, void* stream) {
    if (!fmt || !y || !llr) return MDGMI_E_NULL;
    if (n < 1) return MDGMI_E_SHAPE;
    if (!finite_pos(sigma2)) return MDGMI_E_SIGMA2;
    int p = 0;
    int rc = resolve_path(fmt, path, s_of(sigma2), &p, n);
    if (rc != MDGMI_OK) return rc;
    size_t need = 0;
    rc = mdgmi_llr_workspace_size(fmt, n, p, &need);
    if (rc != MDGMI_OK) return rc;
    if (need > 0 && (!ws || ws_bytes < need)) return MDGMI_E_WORKSPACE;
    rc = check_device(fmt);
    if (rc != MDGMI_OK) return rc;
    SnrArgs sa = snr_args(&sigma2, 0, 1);
    hipStream_t st = (hipStream_t)stream;
    const GmiPlan pl = plan_gmi(fmt, n, 1, p, mode);
    hipError_t e = launch_exact(fmt, p, y, nullptr, n, sa, mode, llr, nullptr, ws, pl.cfg, st);
    return e == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}
}  // namespace

int gmi_with_workspace(const mdgmi_format* fmt, const void* y, const uint32_t* tx_idx, int64_t n,
                       const double* sigma2_host, int32_t n_snr, int32_t path, double* out, void* ws, size_t ws_bytes,
                       void* stream) {
    if (path == MDGMI_PATH_LEARNED_BF16)
        return learned_gmi(fmt, (const float*)y, tx_idx, n, sigma2_host, n_snr, out, ws, ws_bytes, stream);
    return run_gmi(fmt, y, tx_idx, n, sigma2_host, n_snr, path, kModeGmi, out, ws, ws_bytes, stream);
}
}  // namespace mdgmi

using namespace mdgmi;

extern "C" {

const char* mdgmi_status_string(int status) {
    switch (status) {
        case MDGMI_OK: return "ok";
        case MDGMI_E_NULL: return "a required pointer is NULL";
        case MDGMI_E_SHAPE: return "n, n_snr, dim or M out of range";
        case MDGMI_E_LABELS: return "labels are not a permutation of [0, M)";
        case MDGMI_E_SIGMA2: return "sigma2 must be finite and > 0";
        case MDGMI_E_UNSUPPORTED: return "path not available for this format / SNR";
        case MDGMI_E_WORKSPACE: return "workspace missing or too small";
        case MDGMI_E_HIP: return "HIP runtime error";
        case MDGMI_E_DEVICE: return "current device differs from the format's device";
        case MDGMI_E_ARG: return "argument out of range";
        default: return "unknown status";
    }
}

int mdgmi_format_create(const double* X_host, const uint32_t* labels_host, int32_t M, int32_t dim,
                        mdgmi_format** out) {
    if (!X_host || !labels_host || !out) return MDGMI_E_NULL;
    *out = nullptr;
    FormatHost fh;
    const int rc = prepare_format(X_host, labels_host, M, dim, fh);
    if (rc != MDGMI_OK) return rc;
    mdgmi_format* f = new mdgmi_format();
    f->M = M;
    f->dim = dim;
    f->m = fh.m;
    f->energy = fh.energy;
    f->max_abs = fh.max_abs;
    f->max_norm2 = fh.max_norm2;
    if (hipGetDevice(&f->device) != hipSuccess) {
        delete f;
        return MDGMI_E_HIP;
    }
    const std::vector<double>& X64 = fh.X64;
    const std::vector<float>& X32 = fh.X32;
    const std::vector<float>& n32 = fh.n32;
    const std::vector<uint32_t>& lab_hd = fh.labels_hd;
    f->h_X64 = new double[(size_t)M * dim];
    std::memcpy(f->h_X64, X64.data(), sizeof(double) * X64.size());
    bool ok = hipMalloc(&f->d_X64, sizeof(double) * X64.size()) == hipSuccess &&
              hipMalloc(&f->d_X32, sizeof(float) * X32.size()) == hipSuccess &&
              hipMalloc(&f->d_n32, sizeof(float) * n32.size()) == hipSuccess &&
              hipMalloc(&f->d_labels, sizeof(uint32_t) * (size_t)M) == hipSuccess &&
              hipMalloc(&f->d_labels_hd, sizeof(uint32_t) * (size_t)M) == hipSuccess;
    ok = ok && hipMemcpy(f->d_X64, X64.data(), sizeof(double) * X64.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(f->d_X32, X32.data(), sizeof(float) * X32.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(f->d_n32, n32.data(), sizeof(float) * n32.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(f->d_labels, labels_host, sizeof(uint32_t) * (size_t)M, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(f->d_labels_hd, lab_hd.data(), sizeof(uint32_t) * (size_t)M, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        mdgmi_format_destroy(f);
        return MDGMI_E_HIP;
    }
    *out = f;
    return MDGMI_OK;
}

int mdgmi_format_destroy(mdgmi_format* f) {
    if (!f) return MDGMI_E_NULL;
    if (f->d_X64) (void)hipFree(f->d_X64);
    if (f->d_X32) (void)hipFree(f->d_X32);
    if (f->d_n32) (void)hipFree(f->d_n32);
    if (f->d_labels) (void)hipFree(f->d_labels);
    if (f->d_labels_hd) (void)hipFree(f->d_labels_hd);
    learned_free(f);
    delete[] f->h_X64;
    delete f;
    return MDGMI_OK;
}

int mdgmi_generate(const mdgmi_format* fmt, uint64_t seed, const double* sigma2_host, int32_t n_snr, int64_t n,
                   int32_t snr_slot0, void* y, uint32_t* tx_idx, int32_t y_is_f64, void* stream) {
    if (!fmt || !sigma2_host || !y || !tx_idx) return MDGMI_E_NULL;
    if (n < 1 || n_snr < 1) return MDGMI_E_SHAPE;
    if (snr_slot0 < 0) return MDGMI_E_ARG;
    for (int q = 0; q < n_snr; q++)
        if (!finite_pos(sigma2_host[q])) return MDGMI_E_SIGMA2;
    int rc = check_device(fmt);
    if (rc != MDGMI_OK) return rc;
    hipError_t e = launch_generate(fmt, seed, sigma2_host, n_snr, n, snr_slot0, y, tx_idx, y_is_f64 != 0,
                                   (hipStream_t)stream);
    return e == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

int mdgmi_llr_workspace_size(const mdgmi_format* fmt, int64_t n, int32_t path, size_t* bytes) {
    if (!fmt || !bytes) return MDGMI_E_NULL;
    if (n < 1) return MDGMI_E_SHAPE;
    if (path == MDGMI_PATH_LEARNED_BF16) return learned_llr_workspace_size(fmt, n, bytes);
    int p = path == MDGMI_PATH_AUTO ? (fmt->M >= 32 ? MDGMI_PATH_F32_MFMA_F16SPLIT : MDGMI_PATH_F32_DIRECT) : path;
    if (p == MDGMI_PATH_F64)
        *bytes = 0;
    else if (p == MDGMI_PATH_F32_DIRECT)
        *bytes = align_up(direct_image_bytes(fmt, 1));
    else if (p == MDGMI_PATH_F32_MFMA_F16SPLIT)  // (AUTO may also resolve to direct or bf16)
        *bytes = align_up(std::max({mfma_image_bytes(fmt, 1), direct_image_bytes(fmt, 1),
                                    path == MDGMI_PATH_AUTO ? mfma_image_bytes(fmt, 1, 1) : size_t(0)}));
    else if (p == MDGMI_PATH_F32_MFMA_BF16SPLIT)
        *bytes = align_up(mfma_image_bytes(fmt, 1, 1));
    else
        return MDGMI_E_ARG;
    return MDGMI_OK;
}

int mdgmi_llr(const mdgmi_format* fmt, const void* y, int64_t n, double sigma2, void* llr, int32_t path, void* ws,
              size_t ws_bytes, void* stream) {
    if (path == MDGMI_PATH_LEARNED_BF16) return learned_llr(fmt, (const float*)y, n, sigma2, (float*)llr, ws, ws_bytes, stream);
    return run_llr(fmt, y, n, sigma2, llr, path, kModeLlr, ws, ws_bytes, stream);
}

int mdgmi_llr_maxlog(const mdgmi_format* fmt, const void* y, int64_t n, double sigma2, void* llr, int32_t path,
                     void* ws, size_t ws_bytes, void* stream) {
    return run_llr(fmt, y, n, sigma2, llr, path, kModeMlLlr, ws, ws_bytes, stream);
}

int mdgmi_gmi_workspace_size(const mdgmi_format* fmt, int64_t n, int32_t n_snr, int32_t path, size_t* bytes) {
    if (path == MDGMI_PATH_LEARNED_BF16) {
        if (!fmt || !bytes) return MDGMI_E_NULL;
        return learned_gmi_workspace_size(fmt, n, n_snr, bytes);
    }
    return gmi_workspace_size(fmt, n, n_snr, path, kModeGmi, bytes);
}

int mdgmi_gmi(const mdgmi_format* fmt, const void* y, const uint32_t* tx_idx, int64_t n, const double* sigma2_host,
              int32_t n_snr, int32_t path, double* out, void* ws, size_t ws_bytes, void* stream) {
    return gmi_with_workspace(fmt, y, tx_idx, n, sigma2_host, n_snr, path, out, ws, ws_bytes, stream);
}

int mdgmi_gmi_hd_workspace_size(const mdgmi_format* fmt, int64_t n, int32_t n_snr, int32_t path, size_t* bytes) {
    return gmi_workspace_size(fmt, n, n_snr, path, kModeHd, bytes);
}

int mdgmi_gmi_hd(const mdgmi_format* fmt, const void* y, const uint32_t* tx_idx, int64_t n,
                 const double* sigma2_host, int32_t n_snr, int32_t path, double* out, void* ws, size_t ws_bytes,
                 void* stream) {
    return run_gmi(fmt, y, tx_idx, n, sigma2_host, n_snr, path, kModeHd, out, ws, ws_bytes, stream);
}

int mdgmi_gmi_maxlog(const mdgmi_format* fmt, const void* y, const uint32_t* tx_idx, int64_t n,
                     const double* sigma2_host, int32_t n_snr, int32_t path, double* out, void* ws, size_t ws_bytes,
                     void* stream) {
    return run_gmi(fmt, y, tx_idx, n, sigma2_host, n_snr, path, kModeMlGmi, out, ws, ws_bytes, stream);
}

int mdgmi_gmi_sopt_workspace_size(int64_t n, size_t* bytes) {
    if (!bytes) return MDGMI_E_NULL;
    if (n < 1) return MDGMI_E_SHAPE;
    *bytes = sopt_workspace_bytes(n);
    return MDGMI_OK;
}

int mdgmi_gmi_sopt(const mdgmi_format* fmt, const void* llr, int32_t llr_is_f64, const uint32_t* tx_idx, int64_t n,
                   double* out, void* ws, size_t ws_bytes, void* stream) {
    if (!fmt || !llr || !tx_idx || !out) return MDGMI_E_NULL;
    if (n < 1) return MDGMI_E_SHAPE;
    if (llr_is_f64 != 0 && llr_is_f64 != 1) return MDGMI_E_ARG;
    if (!ws || ws_bytes < sopt_workspace_bytes(n)) return MDGMI_E_WORKSPACE;
    int rc = check_device(fmt);
    if (rc != MDGMI_OK) return rc;
    hipError_t e = launch_sopt(fmt, llr, llr_is_f64 == 1, tx_idx, n, out, ws, (hipStream_t)stream);
    return e == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

int mdgmi_gmi_bits_workspace_size(int64_t n, size_t* bytes) {
    if (!bytes) return MDGMI_E_NULL;
    if (n < 1) return MDGMI_E_SHAPE;
    *bytes = bits_workspace_bytes(n);
    return MDGMI_OK;
}

int mdgmi_gmi_bits(const mdgmi_format* fmt, const void* llr, int32_t llr_is_f64, const uint32_t* tx_idx, int64_t n,
                   double* out, void* ws, size_t ws_bytes, void* stream) {
    if (!fmt || !llr || !tx_idx || !out) return MDGMI_E_NULL;
    if (n < 1) return MDGMI_E_SHAPE;
    if (llr_is_f64 != 0 && llr_is_f64 != 1) return MDGMI_E_ARG;
    if (!ws || ws_bytes < bits_workspace_bytes(n)) return MDGMI_E_WORKSPACE;
    int rc = check_device(fmt);
    if (rc != MDGMI_OK) return rc;
    hipError_t e = launch_bits(fmt, llr, llr_is_f64 == 1, tx_idx, n, out, ws, (hipStream_t)stream);
    return e == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

double mdgmi_q_factor_db(double ber) {
    if (!(ber >= 0.0 && ber <= 0.5)) return std::numeric_limits<double>::quiet_NaN();
    if (ber == 0.0) return std::numeric_limits<double>::infinity();
    if (ber == 0.5) return -std::numeric_limits<double>::infinity();
    // erfc^-1(2 ber) by bisection on the decreasing erfc over [0, 28]
    // (erfc(28) is below the smallest positive double)
    const double target = 2.0 * ber;
    double lo = 0.0, hi = 28.0;
    for (int it = 0; it < 200; it++) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (std::erfc(mid) > target)
            lo = mid;
        else
            hi = mid;
    }
    return 20.0 * std::log10(std::sqrt(2.0) * 0.5 * (lo + hi));
}

}  // extern "C"
