// Streaming GMI/MI monitor: fixed-size buffers of received samples (with
// the transmitted rows) evaluated as they arrive, on several HIP streams.
//
// The paper's receiver cuts the ADC stream into fixed buffers of 2^22
// samples, each processed on one of several streams with events ordering the
// work that crosses buffers (real-time GPU receiver architecture section).
// Here every lane (one HIP stream, its own device buffers and partials)
// takes every n_lanes-th buffer: the host-to-device copy of the buffer when
// it comes from host memory, then the exact demapper with its per-block FP64
// partials. An accumulation stream waits for each buffer's event in push
// order, reduces its partials in a fixed order into the buffer's result row
// (a ring on the device) and adds its sums to the running totals, so totals
// are bit-identical whatever the number of lanes. A lane reuses its
// partials only after the accumulation of its previous buffer (event).
#include <algorithm>
#include <cmath>
#include <vector>

#include "device_common.h"

struct mdgmi_stream {
    const mdgmi_format* fmt = nullptr;
    int path = 0;
    int device = 0;
    double sigma2 = 0.0;
    int64_t buffer_n = 0;
    int n_lanes = 0;
    int ring = 0;
    int64_t pushed = 0;
    mdgmi::SnrArgs sa{};
    hipStream_t acc_stream = nullptr;
    std::vector<hipStream_t> lane;
    std::vector<hipEvent_t> ev_done, ev_acc;  // per lane
    std::vector<hipEvent_t> ev_ring;          // per result slot: its accumulation has run
    std::vector<void*> d_y, d_tx, d_ws;      // per lane: input buffers, workspace (partials + image)
    std::vector<int> lane_blocks;            // blocks of the lane's last launch
    size_t part_bytes = 0;                   // partials region of a lane workspace
    size_t ws_bytes = 0;                     // whole lane workspace (partials + image)
    int max_blocks = 0;                      // blocks per launch the partials region holds
    double* d_results = nullptr;  // [ring][MDGMI_NFIELDS]
    double* d_total = nullptr;    // [kNPart + 1]: running sums and sample count
};

namespace mdgmi {

namespace {

constexpr int kStreamMaxLanes = 8;

// One block: reduce a buffer's per-block partials in a fixed order, write its
// result row and add its sums to the running totals.
__global__ __launch_bounds__(256) void k_stream_accumulate(const double* __restrict__ part, int blocks, int64_t n,
                                                           int m, double* __restrict__ row,
                                                           double* __restrict__ total) {
    double v[kNPart] = {};
    for (int b = threadIdx.x; b < blocks; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < kNPart; k++) v[k] += part[(size_t)b * kNPart + k];
    }
    __shared__ double tot[kNPart];
    block_reduce_vals<kNPart>(v, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double N = (double)n;
    row[MDGMI_F_GMI] = m - tot[0] / N;
    row[MDGMI_F_MI] = m - tot[2] / N;
    const double vg = n > 1 ? (tot[1] - tot[0] * tot[0] / N) / (N - 1.0) : 0.0;
    const double vm = n > 1 ? (tot[3] - tot[2] * tot[2] / N) / (N - 1.0) : 0.0;
    row[MDGMI_F_SE_GMI] = sqrt(fmax(vg, 0.0) / N);
    row[MDGMI_F_SE_MI] = sqrt(fmax(vm, 0.0) / N);
    row[MDGMI_F_N] = N;
    row[MDGMI_F_NONFINITE] = tot[4];
#pragma unroll
    for (int k = 0; k < kNPart; k++) total[k] += tot[k];
    total[kNPart] += N;
}

__global__ void k_stream_zero(double* __restrict__ total) {
    if (threadIdx.x <= kNPart) total[threadIdx.x] = 0.0;
}

void destroy_stream(mdgmi_stream* s) {
    if (!s) return;
    int prev = 0;
    const bool switched = hipGetDevice(&prev) == hipSuccess && prev != s->device && hipSetDevice(s->device) == hipSuccess;
    for (auto& st : s->lane)
        if (st) (void)hipStreamSynchronize(st);
    if (s->acc_stream) (void)hipStreamSynchronize(s->acc_stream);
    for (auto* p : s->d_y) (void)hipFree(p);
    for (auto* p : s->d_tx) (void)hipFree(p);
    for (auto* p : s->d_ws) (void)hipFree(p);
    (void)hipFree(s->d_results);
    (void)hipFree(s->d_total);
    for (auto e : s->ev_done) (void)hipEventDestroy(e);
    for (auto e : s->ev_acc) (void)hipEventDestroy(e);
    for (auto e : s->ev_ring) (void)hipEventDestroy(e);
    for (auto& st : s->lane)
        if (st) (void)hipStreamDestroy(st);
    if (s->acc_stream) (void)hipStreamDestroy(s->acc_stream);
    if (switched) (void)hipSetDevice(prev);
    delete s;
}

}  // namespace
}  // namespace mdgmi

using namespace mdgmi;

extern "C" {

int mdgmi_stream_create(const mdgmi_format* fmt, double sigma2, int64_t buffer_n, int32_t n_lanes, int32_t path,
                        int32_t ring, mdgmi_stream** out) {
    if (!fmt || !out) return MDGMI_E_NULL;
    *out = nullptr;
    if (buffer_n < 1 || buffer_n > (int64_t(1) << 31) || n_lanes < 1 || n_lanes > kStreamMaxLanes || ring < 1 ||
        ring > (1 << 20))
        return MDGMI_E_SHAPE;
    if (!finite_pos(sigma2)) return MDGMI_E_SIGMA2;
    int p = 0;
    int rc = resolve_path(fmt, path, s_of(sigma2), &p, buffer_n);
    if (rc != MDGMI_OK) return rc;
    rc = check_device(fmt);
    if (rc != MDGMI_OK) return rc;
    mdgmi_stream* s = new mdgmi_stream();
    s->fmt = fmt;
    s->path = p;
    s->device = fmt->device;
    s->sigma2 = sigma2;
    s->buffer_n = buffer_n;
    s->n_lanes = n_lanes;
    s->ring = ring;
    s->sa = snr_args(&sigma2, 0, 1);
    const GmiPlan pl = plan_gmi(fmt, buffer_n, 1, p);
    s->part_bytes = align_up(pl.part_bytes);
    s->ws_bytes = pl.total;
    s->max_blocks = pl.cfg.blocks_per_snr;
    const size_t ybytes = (size_t)buffer_n * fmt->dim * (p == MDGMI_PATH_F64 ? sizeof(double) : sizeof(float));
    bool ok = hipStreamCreateWithFlags(&s->acc_stream, hipStreamNonBlocking) == hipSuccess;
    s->lane.assign(n_lanes, nullptr);
    s->ev_done.assign(n_lanes, nullptr);
    s->ev_acc.assign(n_lanes, nullptr);
    s->d_y.assign(n_lanes, nullptr);
    s->d_tx.assign(n_lanes, nullptr);
    s->d_ws.assign(n_lanes, nullptr);
    s->lane_blocks.assign(n_lanes, 0);
    for (int k = 0; k < n_lanes && ok; k++) {
        ok = hipStreamCreateWithFlags(&s->lane[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&s->ev_done[k], hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&s->ev_acc[k], hipEventDisableTiming) == hipSuccess &&
             hipMalloc(&s->d_y[k], ybytes) == hipSuccess &&
             hipMalloc(&s->d_tx[k], (size_t)buffer_n * sizeof(uint32_t)) == hipSuccess &&
             hipMalloc(&s->d_ws[k], pl.total) == hipSuccess;
    }
    s->ev_ring.assign(ring, nullptr);
    for (int r = 0; r < ring && ok; r++)
        ok = hipEventCreateWithFlags(&s->ev_ring[r], hipEventDisableTiming) == hipSuccess;
    ok = ok && hipMalloc(&s->d_results, (size_t)ring * MDGMI_NFIELDS * sizeof(double)) == hipSuccess &&
         hipMalloc(&s->d_total, (kNPart + 1) * sizeof(double)) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_stream_zero, dim3(1), dim3(64), 0, s->acc_stream, s->d_total);
        ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(s->acc_stream) == hipSuccess;
    }
    if (!ok) {
        destroy_stream(s);
        return MDGMI_E_HIP;
    }
    *out = s;
    return MDGMI_OK;
}

int mdgmi_stream_push(mdgmi_stream* s, const void* y, const uint32_t* tx_idx, int64_t n, int32_t from_host,
                      int64_t* index) {
    if (!s || !y || !tx_idx) return MDGMI_E_NULL;
    if (n < 1 || n > s->buffer_n) return MDGMI_E_SHAPE;
    if (from_host != 0 && from_host != 1) return MDGMI_E_ARG;
    int rc = check_device(s->fmt);
    if (rc != MDGMI_OK) return rc;
    // the plan of this buffer (as mdgmi_gmi would launch it), held to the
    // workspace sized at create: a tuning change since then could ask for
    // more blocks or a larger image
    GmiPlan pl = plan_gmi(s->fmt, n, 1, s->path);
    if (pl.cfg.blocks_per_snr > s->max_blocks) pl.cfg.blocks_per_snr = s->max_blocks;
    if (align_up(pl.image_bytes) > s->ws_bytes - s->part_bytes) return MDGMI_E_WORKSPACE;
    const int64_t b = s->pushed;
    const int k = (int)(b % s->n_lanes);
    hipStream_t st = s->lane[k];
    const size_t ybytes = (size_t)n * s->fmt->dim * (s->path == MDGMI_PATH_F64 ? sizeof(double) : sizeof(float));
    const void* yd = y;
    const uint32_t* td = tx_idx;
    if (from_host) {
        if (hipMemcpyAsync(s->d_y[k], y, ybytes, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(s->d_tx[k], tx_idx, (size_t)n * sizeof(uint32_t), hipMemcpyHostToDevice, st) != hipSuccess)
            return MDGMI_E_HIP;
        yd = s->d_y[k];
        td = (const uint32_t*)s->d_tx[k];
    }
    // the lane's partials are free once its previous buffer was accumulated
    if (b >= s->n_lanes && hipStreamWaitEvent(st, s->ev_acc[k], 0) != hipSuccess) return MDGMI_E_HIP;
    double* part = (double*)s->d_ws[k];
    void* image = (char*)s->d_ws[k] + s->part_bytes;
    if (launch_exact(s->fmt, s->path, yd, td, n, s->sa, kModeGmi, nullptr, part, image, pl.cfg, st) != hipSuccess)
        return MDGMI_E_HIP;
    s->lane_blocks[k] = pl.cfg.blocks_per_snr;
    if (hipEventRecord(s->ev_done[k], st) != hipSuccess) return MDGMI_E_HIP;
    // accumulation in push order
    if (hipStreamWaitEvent(s->acc_stream, s->ev_done[k], 0) != hipSuccess) return MDGMI_E_HIP;
    const int slot = (int)(b % s->ring);
    hipLaunchKernelGGL(k_stream_accumulate, dim3(1), dim3(256), 0, s->acc_stream, part, pl.cfg.blocks_per_snr, n,
                       s->fmt->m, s->d_results + (size_t)slot * MDGMI_NFIELDS, s->d_total);
    if (hipGetLastError() != hipSuccess || hipEventRecord(s->ev_acc[k], s->acc_stream) != hipSuccess ||
        hipEventRecord(s->ev_ring[slot], s->acc_stream) != hipSuccess)
        return MDGMI_E_HIP;
    s->pushed = b + 1;
    if (index) *index = b;
    return MDGMI_OK;
}

int mdgmi_stream_wait(mdgmi_stream* s, int64_t index) {
    if (!s) return MDGMI_E_NULL;
    if (index >= s->pushed) return MDGMI_E_ARG;
    if (index < 0 || index < s->pushed - s->ring)
        return hipStreamSynchronize(s->acc_stream) == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
    return hipEventSynchronize(s->ev_ring[index % s->ring]) == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

int mdgmi_stream_result(mdgmi_stream* s, int64_t index, double* out_host) {
    if (!s || !out_host) return MDGMI_E_NULL;
    if (index < 0 || index >= s->pushed || index < s->pushed - s->ring) return MDGMI_E_ARG;
    int rc = mdgmi_stream_wait(s, index);
    if (rc != MDGMI_OK) return rc;
    return hipMemcpy(out_host, s->d_results + (size_t)(index % s->ring) * MDGMI_NFIELDS,
                     MDGMI_NFIELDS * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess
               ? MDGMI_OK
               : MDGMI_E_HIP;
}

int mdgmi_stream_total(mdgmi_stream* s, double* out_host) {
    if (!s || !out_host) return MDGMI_E_NULL;
    if (hipStreamSynchronize(s->acc_stream) != hipSuccess) return MDGMI_E_HIP;
    double t[kNPart + 1];
    if (hipMemcpy(t, s->d_total, sizeof(t), hipMemcpyDeviceToHost) != hipSuccess) return MDGMI_E_HIP;
    const double N = t[kNPart];
    const int m = s->fmt->m;
    for (int k = 0; k < MDGMI_NFIELDS; k++) out_host[k] = 0.0;
    if (N > 0.0) {
        out_host[MDGMI_F_GMI] = m - t[0] / N;
        out_host[MDGMI_F_MI] = m - t[2] / N;
        const double vg = N > 1.0 ? (t[1] - t[0] * t[0] / N) / (N - 1.0) : 0.0;
        const double vm = N > 1.0 ? (t[3] - t[2] * t[2] / N) / (N - 1.0) : 0.0;
        out_host[MDGMI_F_SE_GMI] = std::sqrt(std::max(vg, 0.0) / N);
        out_host[MDGMI_F_SE_MI] = std::sqrt(std::max(vm, 0.0) / N);
    }
    out_host[MDGMI_F_N] = N;
    out_host[MDGMI_F_NONFINITE] = t[4];
    return MDGMI_OK;
}

int mdgmi_stream_reset(mdgmi_stream* s) {
    if (!s) return MDGMI_E_NULL;
    hipLaunchKernelGGL(k_stream_zero, dim3(1), dim3(64), 0, s->acc_stream, s->d_total);
    return hipGetLastError() == hipSuccess && hipStreamSynchronize(s->acc_stream) == hipSuccess ? MDGMI_OK
                                                                                              : MDGMI_E_HIP;
}

int mdgmi_stream_info(const mdgmi_stream* s, int64_t* pushed, int32_t* path) {
    if (!s) return MDGMI_E_NULL;
    if (pushed) *pushed = s->pushed;
    if (path) *path = s->path;
    return MDGMI_OK;
}

int mdgmi_stream_destroy(mdgmi_stream* s) {
    if (!s) return MDGMI_E_NULL;
    destroy_stream(s);
    return MDGMI_OK;
}

}  // extern "C"
