// MLP demapper: parameters, training step and inference on the GPU.
//
// The network maps features x = [y, (SNR_dB - 9.5) / 4.5] through hidden
// layers with GELU to m logits read as LLRs in nats. FP32 master weights
// (flat, [W_1 b_1 W_2 b_2 ...], W_l row-major [out][in]) with bf16 copies of
// every W_l and W_l^T for the GEMMs; bf16 activations and gradients, FP32
// accumulation; Adam on the FP32 masters. Loss: binary cross-entropy with
// logits against targets p = sigmoid(lambda_exact), summed over bits and
// averaged over samples.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "device_common.h"
#include "mlp_gemm.h"
#include "mlp_layout.h"

using mdgmi::mlp::GemmArgs;

struct mdgmi_mlp {
    int L = 0;
    int sizes[MDGMI_MLP_MAX_LAYERS + 1] = {0};
    int64_t P = 0;
    int64_t woff[MDGMI_MLP_MAX_LAYERS] = {0}, boff[MDGMI_MLP_MAX_LAYERS] = {0};
    float* d_params = nullptr;  // FP32 masters
    float* d_m = nullptr;
    float* d_v = nullptr;
    float* d_grad = nullptr;
    __bf16* d_w[MDGMI_MLP_MAX_LAYERS] = {nullptr};   // [out][in]
    __bf16* d_wt[MDGMI_MLP_MAX_LAYERS] = {nullptr};  // [in][out]
    __bf16* d_wf[4] = {nullptr};                     // fused-inference layout (fused shapes only)
    bool fused = false;
    int64_t step = 0;
    int device = 0;
    int width = 0;  // widest layer
};

namespace mdgmi {

// mlp_fused.hip
bool fused_shape_ok(const int* sizes, int L);
size_t fused_weight_bytes(int layer);
hipError_t build_fused_weights(const float* const* W, const int* out, const int* in, __bf16* const* dst,
                               hipStream_t st);
int fused_grid();
extern int g_fused_waves;
hipError_t launch_mlp_gmi_fused(__bf16* const* wf, const float* const* bias, int in_dim, int out_dim, const float* y,
                                int dim, const uint32_t* tx, const uint32_t* labels, int M, int64_t n, float snr_feat,
                                double* part, int grid, hipStream_t st);

namespace {

using namespace mlp;

constexpr int64_t kKSplit = 256;  // samples per split-K slice of the weight gradients (at least)
constexpr int64_t kMaxSplits = 64;

int64_t al(int64_t v) { return (v + 255) / 256 * 256; }

// chunk length of the bias-gradient column sums (at most 65535 chunks: grid.y)
// Samples per split-K slice of the weight gradients: kKSplit, or more so
// that there are at most kMaxSplits slices (a multiple of the GEMM's K step).
int64_t split_len(int64_t n) {
    const int64_t s = std::max<int64_t>(kKSplit, (n + kMaxSplits - 1) / kMaxSplits);
    return (s + mlp::kKStep - 1) / mlp::kKStep * mlp::kKStep;
}


// ---- elementwise kernels ----
// out [n][cols] = bf16(x), and xt [cols][n] (if not null) the transposed copy
__global__ void k_to_bf16(const float* __restrict__ x, int64_t n, int cols, __bf16* __restrict__ out,
                          __bf16* __restrict__ xt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * cols) return;
    const __bf16 b = (__bf16)x[i];
    out[i] = b;
    if (xt) xt[(i % cols) * n + i / cols] = b;
}

__global__ void k_features(const float* __restrict__ y, int64_t n, int dim, float snr_feature,
                           float* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int d = 0; d < dim; d++) x[i * (dim + 1) + d] = y[i * dim + d];
    x[i * (dim + 1) + dim] = snr_feature;
}

// D = (sigmoid(z) - sigmoid(lambda)) / n in bf16 (and its transpose Dt
// [out][n]), and per-block FP64 loss partials sum_k softplus(z) - p z.
__global__ __launch_bounds__(256) void k_bce(const float* __restrict__ logits, const float* __restrict__ target_llr,
                                             int64_t n, int out, __bf16* __restrict__ D, __bf16* __restrict__ Dt,
                                             double* __restrict__ part) {
    const int64_t cnt = n * out;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
        const float z = logits[i];
        const float p = 1.0f / (1.0f + expf(-target_llr[i]));
        const float sz = 1.0f / (1.0f + expf(-z));
        const __bf16 d = (__bf16)((sz - p) / (float)n);
        D[i] = d;
        Dt[(i % out) * n + i / out] = d;
        const double sp = (z > 0.0f ? (double)z : 0.0) + log1p(exp(-(double)fabsf(z)));
        acc += sp - (double)p * (double)z;
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss = sum of the block partials / n: thread t adds partials t, t + 64,
// ... in turn, then a fixed tree over the 64 threads.
__global__ __launch_bounds__(64) void k_sum_loss(const double* __restrict__ part, int nb, int64_t n,
                                                 double* __restrict__ loss) {
    __shared__ double red[64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 64) s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (double)n;
}

// The weight and bias gradients of one layer, one launch. Blocks below nr:
// grad[o * in + i] = sum over the split-K slices of partial[s][o][i], in
// slice order, four consecutive i per thread (16-byte loads where the count
// and the pointer allow). The next `out` blocks: db[o] = sum_s D^T[o][s],
// thread t of the block adding samples 8t .. 8t + 7, then 8t + 2048 .. in
// turn (16-byte loads where n and the row allow), then a fixed tree over the
// 256 threads.
__global__ __launch_bounds__(256) void k_grad_finish(const float* __restrict__ partial, int splits, int64_t cnt,
                                                     float* __restrict__ grad, int nr, const __bf16* __restrict__ Dt,
                                                     int64_t n, float* __restrict__ db) {
    if ((int)blockIdx.x < nr) {
        const int64_t i = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
        if (i >= cnt) return;
        if (i + 4 <= cnt && cnt % 4 == 0 && ((uintptr_t)grad & 15) == 0) {
            float4 s = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            for (int k = 0; k < splits; k++) {
                const float4 v = *(const float4*)(partial + (int64_t)k * cnt + i);
                s.x += v.x;
                s.y += v.y;
                s.z += v.z;
                s.w += v.w;
            }
            *(float4*)(grad + i) = s;
        } else {
            for (int64_t j = i; j < i + 4 && j < cnt; j++) {
                float s = 0.0f;
                for (int k = 0; k < splits; k++) s += partial[(int64_t)k * cnt + j];
                grad[j] = s;
            }
        }
        return;
    }
    __shared__ float red[256];
    const int64_t o = blockIdx.x - nr;
    const __bf16* row = Dt + o * n;
    const bool vec = n % 8 == 0 && ((uintptr_t)row & 15) == 0;
    float s = 0.0f;
    for (int64_t i = 8 * (int64_t)threadIdx.x; i < n; i += 8 * 256) {
        if (vec) {
            union {
                uint4 u;
                __bf16 h[8];
            } p;
            p.u = *(const uint4*)(row + i);
#pragma unroll
            for (int j = 0; j < 8; j++) s += (float)p.h[j];
        } else {
            for (int64_t j = i; j < i + 8 && j < n; j++) s += (float)row[j];
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[o] = red[0];
}

// Adam on every parameter, and the bf16 copies of each updated weight in
// the same thread: W [out][in], W^T [in][out] and, for the fused shape, its
// element of the fused inference layout (the layout's padding stays as the
// whole-layout build wrote it).
struct AdamArgs {
    float* p;
    const float* g;
    float* m;
    float* v;
    int64_t P;
    float lr, b1, b2, eps, c1, c2;
};

struct CopyArgs {
    int L;
    bool fused;
    int64_t woff[MDGMI_MLP_MAX_LAYERS];
    int out[MDGMI_MLP_MAX_LAYERS], in[MDGMI_MLP_MAX_LAYERS];
    __bf16* w[MDGMI_MLP_MAX_LAYERS];
    __bf16* wt[MDGMI_MLP_MAX_LAYERS];
    __bf16* wf[4];
};

__global__ void k_adam(AdamArgs a, CopyArgs c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.P) return;
    const float gi = a.g[i];
    const float mi = a.b1 * a.m[i] + (1.0f - a.b1) * gi;
    const float vi = a.b2 * a.v[i] + (1.0f - a.b2) * gi * gi;
    a.m[i] = mi;
    a.v[i] = vi;
    const float pi = a.p[i] - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
    a.p[i] = pi;
    for (int l = 0; l < c.L; l++) {
        const int64_t j = i - c.woff[l];
        if (j < 0 || j >= (int64_t)c.out[l] * c.in[l]) continue;
        const int o = (int)(j / c.in[l]), k = (int)(j % c.in[l]);
        const __bf16 b = (__bf16)pi;
        c.w[l][j] = b;
        c.wt[l][(int64_t)k * c.out[l] + o] = b;
        if (c.fused) c.wf[l][fused::fused_offset(l, o, k, c.in[l])] = (__bf16)(pi * fused::layer_scale(l));
    }
}

// bf16 copies W [out][in] and W^T [in][out] of every layer, one launch
// (blockIdx.y = layer)
struct RefreshArgs {
    const float* W[MDGMI_MLP_MAX_LAYERS];
    __bf16* w[MDGMI_MLP_MAX_LAYERS];
    __bf16* wt[MDGMI_MLP_MAX_LAYERS];
    int out[MDGMI_MLP_MAX_LAYERS], in[MDGMI_MLP_MAX_LAYERS];
};

__global__ void k_refresh(RefreshArgs a) {
    const int l = blockIdx.y, out = a.out[l], in = a.in[l];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)out * in) return;
    const int o = (int)(i / in), j = (int)(i % in);
    const __bf16 b = (__bf16)a.W[l][i];
    a.w[l][i] = b;
    a.wt[l][(int64_t)j * out + o] = b;
}

// ---- GEMM launch ----
template <int EPI>
hipError_t gemm(const GemmArgs& g, bool a_kc, bool b_kc, int splits, hipStream_t st) {
    dim3 grid((g.N + kTile - 1) / kTile, (g.M + kTile - 1) / kTile, splits);
    if (a_kc && b_kc)
        hipLaunchKernelGGL((k_gemm<true, true, EPI>), grid, dim3(256), 0, st, g);
    else if (a_kc)
        hipLaunchKernelGGL((k_gemm<true, false, EPI>), grid, dim3(256), 0, st, g);
    else if (b_kc)
        hipLaunchKernelGGL((k_gemm<false, true, EPI>), grid, dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL((k_gemm<false, false, EPI>), grid, dim3(256), 0, st, g);
    return hipGetLastError();
}

GemmArgs gargs() {
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    return g;
}

// Workspace layout for n samples.
struct MlpWs {
    int64_t x0, z[MDGMI_MLP_MAX_LAYERS], h[MDGMI_MLP_MAX_LAYERS], logits, d0, d1, dt, ht[MDGMI_MLP_MAX_LAYERS], part,
        lpart, total;
};

MlpWs mlp_ws(const mdgmi_mlp* net, int64_t n) {
    MlpWs w{};
    int64_t o = 0;
    w.x0 = o;
    o += al(n * net->sizes[0] * 2);
    for (int l = 0; l < net->L; l++) {
        w.z[l] = o;
        o += al(n * net->sizes[l + 1] * 4);
        w.h[l] = o;
        o += al(n * net->sizes[l + 1] * 2);
    }
    w.logits = w.z[net->L - 1];
    w.d0 = o;
    o += al(n * net->width * 2);
    w.d1 = o;
    o += al(n * net->width * 2);
    // transposed copies [features][n] of D and of every layer's input for
    // the weight gradients (the sample axis is their K axis), written by the
    // kernels that produce D and the inputs
    w.dt = o;
    o += al(n * net->width * 2);
    for (int l = 0; l < net->L; l++) {
        w.ht[l] = o;
        o += al(n * net->sizes[l] * 2);
    }
    const int64_t splits = (n + split_len(n) - 1) / split_len(n);
    w.part = o;
    o += al(splits * (int64_t)net->width * net->width * 4);
    w.lpart = o;
    o += al(1024 * 8);
    w.total = o;
    return w;
}

// Forward pass of n samples: Z_l (FP32) and H_l (bf16) of every layer into
// the workspace; the last layer's Z is the logits. With `transposed`, each
// layer's input is also stored as [features][n] for the weight gradients.
hipError_t forward(const mdgmi_mlp* net, const float* x, int64_t n, char* ws, const MlpWs& w, hipStream_t st,
                   bool transposed = false) {
    const int in0 = net->sizes[0];
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n * in0 + 255) / 256)), dim3(256), 0, st, x, n, in0,
                       (__bf16*)(ws + w.x0), transposed ? (__bf16*)(ws + w.ht[0]) : nullptr);
    const __bf16* prev = (const __bf16*)(ws + w.x0);
    for (int l = 0; l < net->L; l++) {
        const int in = net->sizes[l], out = net->sizes[l + 1];
        GemmArgs g = gargs();
        g.A = prev;
        g.a_sm = in;
        g.a_sk = 1;
        g.B = net->d_w[l];
        g.b_sk = 1;
        g.b_sn = in;
        g.M = (int)n;
        g.N = out;
        g.K = in;
        g.k_per_split = ((in + kKStep - 1) / kKStep) * kKStep;
        g.bias = net->d_params + net->boff[l];
        g.C = (float*)(ws + w.z[l]);
        g.ldc = out;
        hipError_t e;
        if (l < net->L - 1) {
            g.H = (__bf16*)(ws + w.h[l]);
            g.ldh = out;
            if (transposed) {
                g.Ht = (__bf16*)(ws + w.ht[l + 1]);
                g.ldht = n;
            }
            e = gemm<kEpiGeluBf16>(g, true, true, 1, st);
        } else {
            e = gemm<kEpiF32>(g, true, true, 1, st);
        }
        if (e != hipSuccess) return e;
        prev = (const __bf16*)(ws + w.h[l]);
    }
    return hipSuccess;
}

void refresh_all(mdgmi_mlp* net, hipStream_t st) {
    RefreshArgs a{};
    int64_t most = 0;
    const float* W[MDGMI_MLP_MAX_LAYERS];
    for (int l = 0; l < net->L; l++) {
        W[l] = a.W[l] = net->d_params + net->woff[l];
        a.w[l] = net->d_w[l];
        a.wt[l] = net->d_wt[l];
        a.out[l] = net->sizes[l + 1];
        a.in[l] = net->sizes[l];
        most = std::max<int64_t>(most, (int64_t)a.out[l] * a.in[l]);
    }
    hipLaunchKernelGGL(k_refresh, dim3((unsigned)((most + 255) / 256), (unsigned)net->L), dim3(256), 0, st, a);
    if (net->fused) (void)build_fused_weights(W, a.out, a.in, net->d_wf, st);
}

bool ok_sizes(const int32_t* sizes, int L) {
    if (L < 1 || L > MDGMI_MLP_MAX_LAYERS) return false;
    for (int l = 0; l <= L; l++)
        if (sizes[l] < 1 || sizes[l] > 4096) return false;
    return true;
}

}  // namespace
}  // namespace mdgmi

using namespace mdgmi;

extern "C" {

int mdgmi_mlp_create(const int32_t* sizes, int32_t n_layers, uint64_t seed, mdgmi_mlp** out) {
    if (!sizes || !out) return MDGMI_E_NULL;
    *out = nullptr;
    if (!ok_sizes(sizes, n_layers)) return MDGMI_E_SHAPE;
    mdgmi_mlp* net = new mdgmi_mlp();
    net->L = n_layers;
    int64_t p = 0;
    for (int l = 0; l <= n_layers; l++) {
        net->sizes[l] = sizes[l];
        net->width = std::max(net->width, (int)sizes[l]);
    }
    for (int l = 0; l < n_layers; l++) {
        net->woff[l] = p;
        p += (int64_t)sizes[l + 1] * sizes[l];
        net->boff[l] = p;
        p += sizes[l + 1];
    }
    net->P = p;
    (void)hipGetDevice(&net->device);
    // PyTorch-style default init of a linear layer: W, b ~ U(-1/sqrt(in), 1/sqrt(in)),
    // drawn from a 64-bit Mersenne twister seeded with `seed`.
    std::vector<float> h(p);
    std::mt19937_64 rng(seed);
    for (int l = 0; l < n_layers; l++) {
        const double bound = 1.0 / std::sqrt((double)sizes[l]);
        for (int64_t i = net->woff[l]; i < net->boff[l] + sizes[l + 1]; i++)
            h[i] = (float)((2.0 * ((rng() >> 11) * (1.0 / 9007199254740992.0)) - 1.0) * bound);
    }
    bool ok = hipMalloc(&net->d_params, sizeof(float) * p) == hipSuccess &&
              hipMalloc(&net->d_m, sizeof(float) * p) == hipSuccess &&
              hipMalloc(&net->d_v, sizeof(float) * p) == hipSuccess &&
              hipMalloc(&net->d_grad, sizeof(float) * p) == hipSuccess;
    for (int l = 0; ok && l < n_layers; l++) {
        const int64_t cnt = (int64_t)sizes[l + 1] * sizes[l];
        ok = hipMalloc(&net->d_w[l], 2 * cnt) == hipSuccess && hipMalloc(&net->d_wt[l], 2 * cnt) == hipSuccess;
    }
    net->fused = fused_shape_ok(net->sizes, net->L);
    for (int l = 0; ok && net->fused && l < 4; l++) ok = hipMalloc(&net->d_wf[l], fused_weight_bytes(l)) == hipSuccess;
    ok = ok && hipMemcpy(net->d_params, h.data(), sizeof(float) * p, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(net->d_m, 0, sizeof(float) * p) == hipSuccess &&
         hipMemset(net->d_v, 0, sizeof(float) * p) == hipSuccess &&
         hipMemset(net->d_grad, 0, sizeof(float) * p) == hipSuccess;
    if (ok) {
        refresh_all(net, nullptr);
        ok = hipDeviceSynchronize() == hipSuccess;
    }
    if (!ok) {
        mdgmi_mlp_destroy(net);
        return MDGMI_E_HIP;
    }
    *out = net;
    return MDGMI_OK;
}

int mdgmi_mlp_destroy(mdgmi_mlp* net) {
    if (!net) return MDGMI_E_NULL;
    (void)hipFree(net->d_params);
    (void)hipFree(net->d_m);
    (void)hipFree(net->d_v);
    (void)hipFree(net->d_grad);
    for (int l = 0; l < net->L; l++) {
        (void)hipFree(net->d_w[l]);
        (void)hipFree(net->d_wt[l]);
    }
    for (int l = 0; l < 4; l++)
        if (net->d_wf[l]) (void)hipFree(net->d_wf[l]);
    delete net;
    return MDGMI_OK;
}

int mdgmi_mlp_param_count(const mdgmi_mlp* net, int64_t* count) {
    if (!net || !count) return MDGMI_E_NULL;
    *count = net->P;
    return MDGMI_OK;
}

int mdgmi_mlp_get_params(const mdgmi_mlp* net, float* host, int64_t count, int32_t which) {
    if (!net || !host) return MDGMI_E_NULL;
    if (count != net->P) return MDGMI_E_SHAPE;
    const float* src = which == 0 ? net->d_params : which == 1 ? net->d_grad : which == 2 ? net->d_m : which == 3 ? net->d_v : nullptr;
    if (!src) return MDGMI_E_ARG;
    return hipMemcpy(host, src, sizeof(float) * count, hipMemcpyDeviceToHost) == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

int mdgmi_mlp_set_params(mdgmi_mlp* net, const float* host, int64_t count) {
    if (!net || !host) return MDGMI_E_NULL;
    if (count != net->P) return MDGMI_E_SHAPE;
    if (hipMemcpy(net->d_params, host, sizeof(float) * count, hipMemcpyHostToDevice) != hipSuccess) return MDGMI_E_HIP;
    refresh_all(net, nullptr);
    return hipDeviceSynchronize() == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

int mdgmi_mlp_workspace_size(const mdgmi_mlp* net, int64_t n, size_t* bytes) {
    if (!net || !bytes) return MDGMI_E_NULL;
    if (n < 1 || n > (int64_t)1 << 30) return MDGMI_E_SHAPE;
    *bytes = (size_t)mlp_ws(net, n).total;
    return MDGMI_OK;
}

int mdgmi_mlp_features(const float* y, int64_t n, int32_t dim, double snr_db, float* x, void* stream) {
    if (!y || !x) return MDGMI_E_NULL;
    if (n < 1 || dim < 1 || dim > 16) return MDGMI_E_SHAPE;
    const float feat = (float)((snr_db - 9.5) / 4.5);
    hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, y, n, dim,
                       feat, x);
    return hipGetLastError() == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

int mdgmi_mlp_forward(const mdgmi_mlp* net, const float* x, int64_t n, float* logits, void* ws, size_t ws_bytes,
                      void* stream) {
    if (!net || !x || !logits || !ws) return MDGMI_E_NULL;
    if (n < 1 || n > (int64_t)1 << 30) return MDGMI_E_SHAPE;
    const MlpWs w = mlp_ws(net, n);
    if (ws_bytes < (size_t)w.total) return MDGMI_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    if (forward(net, x, n, (char*)ws, w, st) != hipSuccess) return MDGMI_E_HIP;
    const int out = net->sizes[net->L];
    return hipMemcpyAsync(logits, (char*)ws + w.logits, sizeof(float) * n * out, hipMemcpyDeviceToDevice, st) ==
                   hipSuccess
               ? MDGMI_OK
               : MDGMI_E_HIP;
}

int mdgmi_mlp_loss_grad(mdgmi_mlp* net, const float* x, const float* target_llr, int64_t n, double* loss, void* ws,
                        size_t ws_bytes, void* stream) {
    if (!net || !x || !target_llr || !loss || !ws) return MDGMI_E_NULL;
    if (n < 1 || n > (int64_t)1 << 30) return MDGMI_E_SHAPE;
    const MlpWs w = mlp_ws(net, n);
    if (ws_bytes < (size_t)w.total) return MDGMI_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    if (forward(net, x, n, base, w, st, true) != hipSuccess) return MDGMI_E_HIP;
    const int L = net->L, outL = net->sizes[L];
    const int nb = (int)std::min<int64_t>(1024, (n * outL + 255) / 256);
    hipLaunchKernelGGL(k_bce, dim3(nb), dim3(256), 0, st, (const float*)(base + w.logits), target_llr, n, outL,
                       (__bf16*)(base + w.d0), (__bf16*)(base + w.dt), (double*)(base + w.lpart));
    hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(64), 0, st, (const double*)(base + w.lpart), nb, n, loss);
    __bf16* D = (__bf16*)(base + w.d0);
    __bf16* Dn = (__bf16*)(base + w.d1);
    const int64_t slen = split_len(n);
    const int splits = (int)((n + slen - 1) / slen);
    for (int l = L - 1; l >= 0; l--) {
        const int in = net->sizes[l], out = net->sizes[l + 1];
        // dW_l [out][in] = sum_s D[s][o] Hprev[s][i]  (split over samples),
        // on the copies with the sample axis contiguous: D^T [out][n], Hprev^T [in][n]
        const __bf16* Dt = (const __bf16*)(base + w.dt);
        const __bf16* Ht = (const __bf16*)(base + w.ht[l]);
        GemmArgs g = gargs();
        g.A = Dt;
        g.a_sm = n;
        g.a_sk = 1;
        g.B = Ht;
        g.b_sk = 1;
        g.b_sn = n;
        g.M = out;
        g.N = in;
        g.K = n;
        g.k_per_split = slen;
        g.C = (float*)(base + w.part);
        if (gemm<kEpiPartial>(g, true, true, splits, st) != hipSuccess) return MDGMI_E_HIP;
        // dW_l from the slices and db_l [out] = sum_s D[s][o] from the same transposed copy
        const int64_t cnt = (int64_t)out * in;
        const int nr = (int)((cnt + 1023) / 1024);
        hipLaunchKernelGGL(k_grad_finish, dim3((unsigned)(nr + out)), dim3(256), 0, st,
                           (const float*)(base + w.part), splits, cnt, net->d_grad + net->woff[l], nr,
                           (const __bf16*)Dt, n, net->d_grad + net->boff[l]);
        if (l > 0) {
            // D_prev [n][in] = (D [n][out] W_l [out][in]) * gelu'(Z_{l-1})
            GemmArgs h = gargs();
            h.A = D;
            h.a_sm = out;
            h.a_sk = 1;
            h.B = net->d_wt[l];  // B(k = o, n = i) = W^T[i][o]
            h.b_sk = 1;
            h.b_sn = out;
            h.M = (int)n;
            h.N = in;
            h.K = out;
            h.k_per_split = ((out + kKStep - 1) / kKStep) * kKStep;
            h.H = Dn;
            h.ldh = in;
            h.Z = (const float*)(base + w.z[l - 1]);
            h.ldz = in;
            h.Ht = (__bf16*)(base + w.dt);  // D_{l-1}^T for the next weight gradient (this layer's uses are done)
            h.ldht = n;
            if (gemm<kEpiGeluGrad>(h, true, true, 1, st) != hipSuccess) return MDGMI_E_HIP;
            std::swap(D, Dn);
        }
    }
    return hipGetLastError() == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

int mdgmi_mlp_adam_step(mdgmi_mlp* net, float lr, float beta1, float beta2, float eps, void* stream) {
    if (!net) return MDGMI_E_NULL;
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return MDGMI_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    net->step++;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)net->step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)net->step));
    const AdamArgs a{net->d_params, net->d_grad, net->d_m, net->d_v, net->P, lr, beta1, beta2, eps, c1, c2};
    CopyArgs c{};
    c.L = net->L;
    c.fused = net->fused;
    for (int l = 0; l < net->L; l++) {
        c.woff[l] = net->woff[l];
        c.out[l] = net->sizes[l + 1];
        c.in[l] = net->sizes[l];
        c.w[l] = net->d_w[l];
        c.wt[l] = net->d_wt[l];
        if (l < 4) c.wf[l] = net->d_wf[l];
    }
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((net->P + 255) / 256)), dim3(256), 0, st, a, c);
    return hipGetLastError() == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

int mdgmi_mlp_save(const mdgmi_mlp* net, const char* path) {
    if (!net || !path) return MDGMI_E_NULL;
    std::vector<float> p(net->P), m(net->P), v(net->P);
    if (hipMemcpy(p.data(), net->d_params, 4 * net->P, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(m.data(), net->d_m, 4 * net->P, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(v.data(), net->d_v, 4 * net->P, hipMemcpyDeviceToHost) != hipSuccess)
        return MDGMI_E_HIP;
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return MDGMI_E_ARG;
    const char magic[8] = {'M', 'D', 'G', 'M', 'I', 'M', 'L', '1'};
    int32_t hdr[2 + MDGMI_MLP_MAX_LAYERS + 1] = {net->L};
    for (int l = 0; l <= net->L; l++) hdr[1 + l] = net->sizes[l];
    bool ok = std::fwrite(magic, 1, 8, fp) == 8 && std::fwrite(hdr, sizeof(hdr), 1, fp) == 1 &&
              std::fwrite(&net->step, sizeof(int64_t), 1, fp) == 1 &&
              std::fwrite(p.data(), 4, net->P, fp) == (size_t)net->P &&
              std::fwrite(m.data(), 4, net->P, fp) == (size_t)net->P &&
              std::fwrite(v.data(), 4, net->P, fp) == (size_t)net->P;
    std::fclose(fp);
    return ok ? MDGMI_OK : MDGMI_E_ARG;
}

int mdgmi_mlp_load(mdgmi_mlp* net, const char* path) {
    if (!net || !path) return MDGMI_E_NULL;
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return MDGMI_E_ARG;
    char magic[8];
    int32_t hdr[2 + MDGMI_MLP_MAX_LAYERS + 1];
    int64_t step = 0;
    std::vector<float> p(net->P), m(net->P), v(net->P);
    bool ok = std::fread(magic, 1, 8, fp) == 8 && std::memcmp(magic, "MDGMIML1", 8) == 0 &&
              std::fread(hdr, sizeof(hdr), 1, fp) == 1 && hdr[0] == net->L;
    for (int l = 0; ok && l <= net->L; l++) ok = hdr[1 + l] == net->sizes[l];
    ok = ok && std::fread(&step, sizeof(int64_t), 1, fp) == 1 && std::fread(p.data(), 4, net->P, fp) == (size_t)net->P &&
         std::fread(m.data(), 4, net->P, fp) == (size_t)net->P && std::fread(v.data(), 4, net->P, fp) == (size_t)net->P;
    std::fclose(fp);
    if (!ok) return MDGMI_E_ARG;
    if (hipMemcpy(net->d_params, p.data(), 4 * net->P, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net->d_m, m.data(), 4 * net->P, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net->d_v, v.data(), 4 * net->P, hipMemcpyHostToDevice) != hipSuccess)
        return MDGMI_E_HIP;
    net->step = step;
    refresh_all(net, nullptr);
    return hipDeviceSynchronize() == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

}  // extern "C"

// ---------------------------------------------------------------- learned GMI
namespace mdgmi {
namespace {

// Per-sample GMI cost of the logits (read as LLRs, nats) in bits, summed per
// block in FP64: partials {sum c, sum c^2, 0, 0, non-finite count}.
__global__ __launch_bounds__(256) void k_learned_cost(const float* __restrict__ logits, const uint32_t* __restrict__ tx,
                                                      const uint32_t* __restrict__ labels, int64_t n, int M, int m,
                                                      double* __restrict__ part) {
    double s = 0.0, s2 = 0.0, bad = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t row = tx[i];
        float c;
        if (row < (uint32_t)M) {
            const uint32_t lab = labels[row];
            c = 0.0f;
            for (int k = 0; k < m; k++) {
                const float z = logits[i * m + k] * 1.4426950408889634f;  // to log2 units
                const float x = ((lab >> k) & 1) ? -z : z;                 // log2(S_other / S_sent)
                c += fmaxf(x, 0.0f) + __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f(-fabsf(x)));
            }
        } else {
            c = NAN;
        }
        const double d = (double)c;
        s += d;
        s2 += d * d;
        bad += __builtin_isfinite(d) ? 0.0 : 1.0;
    }
    CostAcc a;
    a.sg = s;
    a.sg2 = s2;
    a.bad = bad;
    block_reduce_store(a, part + (size_t)blockIdx.x * kNPart);
}

// Sums of the nb block partials in a fixed order (thread t adds blocks t,
// t + 64, ... in turn, then a fixed tree over the 64 threads), then the GMI
// estimate and its standard error.
__global__ __launch_bounds__(64) void k_learned_finish(const double* __restrict__ part, int nb, int64_t n, int m,
                                                       double* __restrict__ out) {
    __shared__ double red[3][64];
    const int t = threadIdx.x;
    double s = 0.0, s2 = 0.0, bad = 0.0;
    for (int b = t; b < nb; b += 64) {
        s += part[(size_t)b * kNPart + 0];
        s2 += part[(size_t)b * kNPart + 1];
        bad += part[(size_t)b * kNPart + 4];
    }
    red[0][t] = s;
    red[1][t] = s2;
    red[2][t] = bad;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (t < w) {
            red[0][t] += red[0][t + w];
            red[1][t] += red[1][t + w];
            red[2][t] += red[2][t + w];
        }
        __syncthreads();
    }
    if (t != 0) return;
    s = red[0][0];
    s2 = red[1][0];
    const double N = (double)n;
    out[MDGMI_F_GMI] = m - s / N;
    out[MDGMI_F_MI] = NAN;  // the learned demapper gives bit metrics only
    const double v = n > 1 ? (s2 - s * s / N) / (N - 1.0) : 0.0;
    out[MDGMI_F_SE_GMI] = sqrt(fmax(v, 0.0) / N);
    out[MDGMI_F_SE_MI] = NAN;
    out[MDGMI_F_N] = N;
    out[MDGMI_F_NONFINITE] = red[2][0];
}

constexpr int kLearnedBlocks = 1024;

}  // namespace
}  // namespace mdgmi

extern "C" {

int mdgmi_mlp_gmi_workspace_size(const mdgmi_mlp* net, int64_t chunk, size_t* bytes) {
    if (!net || !bytes) return MDGMI_E_NULL;
    if (chunk < 1 || chunk > (int64_t)1 << 26) return MDGMI_E_SHAPE;
    const MlpWs w = mlp_ws(net, chunk);
    *bytes = (size_t)(al(chunk * net->sizes[0] * 4) + w.total + al(kLearnedBlocks * kNPart * 8));
    return MDGMI_OK;
}

int mdgmi_mlp_gmi(const mdgmi_mlp* net, const mdgmi_format* fmt, const float* y, const uint32_t* tx_idx, int64_t n,
                  const double* snr_db_host, int32_t n_snr, int64_t chunk, double* out, void* ws, size_t ws_bytes,
                  void* stream) {
    if (!net || !fmt || !y || !tx_idx || !snr_db_host || !out || !ws) return MDGMI_E_NULL;
    if (n < 1 || n_snr < 1 || chunk < 1) return MDGMI_E_SHAPE;
    if (net->sizes[0] != fmt->dim + 1 || net->sizes[net->L] != fmt->m) return MDGMI_E_SHAPE;
    for (int q = 0; q < n_snr; q++)
        if (!std::isfinite(snr_db_host[q])) return MDGMI_E_ARG;
    size_t need = 0;
    int rc = mdgmi_mlp_gmi_workspace_size(net, chunk, &need);
    if (rc != MDGMI_OK) return rc;
    if (ws_bytes < need) return MDGMI_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    float* x = (float*)base;
    char* mws = base + al(chunk * net->sizes[0] * 4);
    const MlpWs w = mlp_ws(net, chunk);
    double* part = (double*)(mws + w.total);
    const int dim = fmt->dim, m = fmt->m;
    if (net->fused && g_fused_waves != 0 && fused_grid() <= kLearnedBlocks) {
        const float* bias[4] = {net->d_params + net->boff[0], net->d_params + net->boff[1],
                                net->d_params + net->boff[2], net->d_params + net->boff[3]};
        const int grid = fused_grid();
        for (int q = 0; q < n_snr; q++) {
            const float feat = (float)((snr_db_host[q] - 9.5) / 4.5);
            if (launch_mlp_gmi_fused(net->d_wf, bias, net->sizes[0], net->sizes[4], y + (size_t)q * n * dim, dim,
                                     tx_idx + (size_t)q * n, fmt->d_labels, fmt->M, n, feat, part, grid, st) !=
                hipSuccess)
                return MDGMI_E_HIP;
            hipLaunchKernelGGL(k_learned_finish, dim3(1), dim3(64), 0, st, part, grid, n, m,
                               out + (size_t)q * MDGMI_NFIELDS);
        }
        return hipGetLastError() == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
    }
    for (int q = 0; q < n_snr; q++) {
        const float* yq = y + (size_t)q * n * dim;
        const uint32_t* tq = tx_idx + (size_t)q * n;
        // chunks are processed in order; each writes its own block partials
        const int64_t nchunks = (n + chunk - 1) / chunk;
        const int per = std::max<int>(1, kLearnedBlocks / (int)std::min<int64_t>(nchunks, kLearnedBlocks));
        int used = 0;
        for (int64_t c0 = 0; c0 < n; c0 += chunk) {
            const int64_t nc = std::min(chunk, n - c0);
            if ((rc = mdgmi_mlp_features(yq + c0 * dim, nc, dim, snr_db_host[q], x, stream)) != MDGMI_OK) return rc;
            if (forward(net, x, nc, mws, w, st) != hipSuccess) return MDGMI_E_HIP;
            const int nb = (int)std::min<int64_t>(per, (nc + 255) / 256);
            if (used + nb > kLearnedBlocks) return MDGMI_E_SHAPE;  // too many chunks for the partial table
            hipLaunchKernelGGL(k_learned_cost, dim3(nb), dim3(256), 0, st, (const float*)(mws + w.logits), tq + c0,
                               fmt->d_labels, nc, fmt->M, m, part + (size_t)used * kNPart);
            used += nb;
        }
        hipLaunchKernelGGL(k_learned_finish, dim3(1), dim3(64), 0, st, part, used, n, m,
                           out + (size_t)q * MDGMI_NFIELDS);
        if (hipGetLastError() != hipSuccess) return MDGMI_E_HIP;
    }
    return MDGMI_OK;
}

}  // extern "C"

// ------------------------------------------ training step, LLRs, learned path
namespace mdgmi {

hipError_t launch_mlp_llr_fused(__bf16* const* wf, const float* const* bias, int in_dim, int out_dim, const float* y,
                                int dim, int64_t n, const float* snr_db, float snr_feat, float* llr, int grid,
                                hipStream_t st);

namespace {

// x [n][dim + 1] = [y, (snr_db[i] - 9.5) / 4.5] (snr_db per sample), or the
// scalar feature when snr_db is null.
__global__ void k_features_snr(const float* __restrict__ y, int64_t n, int dim, const float* __restrict__ snr_db,
                               float snr_feat, float* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int d = 0; d < dim; d++) x[i * (dim + 1) + d] = y[i * dim + d];
    // in FP64 like the host-side scalar feature, so both agree exactly
    x[i * (dim + 1) + dim] = snr_db ? (float)(((double)snr_db[i] - 9.5) / 4.5) : snr_feat;
}

hipError_t features(const float* y, int64_t n, int dim, const float* snr_db, float snr_feat, float* x,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_features_snr, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, y, n, dim, snr_db,
                       snr_feat, x);
    return hipGetLastError();
}

// SNR feature of a noise variance: SNR = E||x||^2 / (dim sigma2) in dB.
float snr_feature(const mdgmi_format* f, double sigma2) {
    const double snr_db = 10.0 * std::log10(f->energy / (f->dim * sigma2));
    return (float)((snr_db - 9.5) / 4.5);
}

void fused_biases(const mdgmi_mlp* net, const float* (&bias)[4]) {
    for (int l = 0; l < 4; l++) bias[l] = net->d_params + net->boff[l];
}

}  // namespace
}  // namespace mdgmi

// A learned demapper attached to a format, with the per-SNR route found by
// calibration (noise variances and whether each uses the network).
struct LearnedBinding {
    const mdgmi_mlp* net = nullptr;
    int exact_path = MDGMI_PATH_AUTO;
    double max_loss = 0.01;
    std::vector<double> s2;
    std::vector<uint8_t> route;
};

namespace mdgmi {
namespace {

// 1 if sigma2 was calibrated to the network, else 0 (exact fallback).
int routed(const LearnedBinding* b, double sigma2) {
    for (size_t k = 0; k < b->s2.size(); k++)
        if (std::fabs(b->s2[k] - sigma2) <= 1e-12 * sigma2) return b->route[k];
    return 0;
}

bool use_fused(const mdgmi_mlp* net) { return net->fused && g_fused_waves != 0 && fused_grid() <= kLearnedBlocks; }

int64_t learned_chunk(int64_t n) { return std::min<int64_t>(n, (int64_t)1 << 20); }

// Workspace of the network's GMI over n samples of one SNR point: block
// partials of the fused kernel, or the layer-by-layer path's buffers.
size_t learned_ws_bytes(const mdgmi_mlp* net, int64_t n) {
    if (use_fused(net)) return (size_t)al((int64_t)fused_grid() * kNPart * 8);
    size_t b = 0;
    mdgmi_mlp_gmi_workspace_size(net, learned_chunk(n), &b);
    return b;
}

int check_net_for(const mdgmi_format* f, const mdgmi_mlp* net) {
    if (net->sizes[0] != f->dim + 1 || net->sizes[net->L] != f->m) return MDGMI_E_SHAPE;
    return MDGMI_OK;
}

double snr_db_of(const mdgmi_format* f, double sigma2) { return 10.0 * std::log10(f->energy / (f->dim * sigma2)); }

// Learned GMI of one SNR point into out_row.
int learned_gmi_one(const mdgmi_format* fmt, const mdgmi_mlp* net, const float* yq, const uint32_t* tq, int64_t n,
                    double sigma2, void* ws, size_t ws_bytes, double* out_row, hipStream_t st) {
    if (!use_fused(net)) {
        const double snr = snr_db_of(fmt, sigma2);
        return mdgmi_mlp_gmi(net, fmt, yq, tq, n, &snr, 1, learned_chunk(n), out_row, ws, ws_bytes, st);
    }
    const float* bias[4];
    fused_biases(net, bias);
    const int grid = fused_grid();
    double* part = (double*)ws;
    if (launch_mlp_gmi_fused(net->d_wf, bias, net->sizes[0], net->sizes[4], yq, fmt->dim, tq, fmt->d_labels, fmt->M,
                             n, snr_feature(fmt, sigma2), part, grid, st) != hipSuccess)
        return MDGMI_E_HIP;
    hipLaunchKernelGGL(k_learned_finish, dim3(1), dim3(64), 0, st, part, grid, n, fmt->m, out_row);
    return hipGetLastError() == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

}  // namespace

int learned_gmi_workspace_size(const mdgmi_format* fmt, int64_t n, int32_t n_snr, size_t* bytes) {
    const LearnedBinding* b = fmt->learned;
    if (!b) return MDGMI_E_UNSUPPORTED;
    size_t ex = 0;
    const int rc = mdgmi_gmi_workspace_size(fmt, n, n_snr, b->exact_path, &ex);
    if (rc != MDGMI_OK) return rc;
    *bytes = std::max(ex, learned_ws_bytes(b->net, n));
    return MDGMI_OK;
}

int learned_gmi(const mdgmi_format* fmt, const float* y, const uint32_t* tx_idx, int64_t n, const double* sigma2_host,
                int32_t n_snr, double* out, void* ws, size_t ws_bytes, void* stream) {
    if (!fmt || !y || !tx_idx || !sigma2_host || !out) return MDGMI_E_NULL;
    if (n < 1 || n_snr < 1) return MDGMI_E_SHAPE;
    const LearnedBinding* b = fmt->learned;
    if (!b) return MDGMI_E_UNSUPPORTED;
    double max_s = 0.0;
    bool any_exact = false;
    for (int q = 0; q < n_snr; q++) {
        if (!finite_pos(sigma2_host[q])) return MDGMI_E_SIGMA2;
        if (!routed(b, sigma2_host[q])) {
            any_exact = true;
            max_s = std::max(max_s, s_of(sigma2_host[q]));
        }
    }
    int p = 0;
    if (any_exact) {
        const int rc = resolve_path(fmt, b->exact_path, max_s, &p);
        if (rc != MDGMI_OK) return rc;
    }
    size_t need = 0;
    int rc = learned_gmi_workspace_size(fmt, n, n_snr, &need);
    if (rc != MDGMI_OK) return rc;
    if (!ws || ws_bytes < need) return MDGMI_E_WORKSPACE;
    if ((rc = check_device(fmt)) != MDGMI_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int dim = fmt->dim;
    // maximal runs of SNR points with the same route, in order
    for (int q0 = 0; q0 < n_snr;) {
        const int r = routed(b, sigma2_host[q0]);
        int q1 = q0 + 1;
        while (q1 < n_snr && routed(b, sigma2_host[q1]) == r) q1++;
        if (r) {
            for (int q = q0; q < q1; q++) {
                rc = learned_gmi_one(fmt, b->net, y + (size_t)q * n * dim, tx_idx + (size_t)q * n, n, sigma2_host[q],
                                     ws, ws_bytes, out + (size_t)q * MDGMI_NFIELDS, st);
                if (rc != MDGMI_OK) return rc;
            }
        } else {
            rc = gmi_with_workspace(fmt, y + (size_t)q0 * n * dim, tx_idx + (size_t)q0 * n, n, sigma2_host + q0,
                                    q1 - q0, b->exact_path, out + (size_t)q0 * MDGMI_NFIELDS, ws, ws_bytes, stream);
            if (rc != MDGMI_OK) return rc;
        }
        q0 = q1;
    }
    return MDGMI_OK;
}

int learned_llr_workspace_size(const mdgmi_format* fmt, int64_t n, size_t* bytes) {
    const LearnedBinding* b = fmt->learned;
    if (!b) return MDGMI_E_UNSUPPORTED;
    size_t ex = 0;
    const int rc = mdgmi_llr_workspace_size(fmt, n, b->exact_path, &ex);
    if (rc != MDGMI_OK) return rc;
    const mdgmi_mlp* net = b->net;
    const size_t le = use_fused(net) ? 0 : (size_t)(al(n * net->sizes[0] * 4) + mlp_ws(net, n).total);
    *bytes = std::max(ex, le);
    return MDGMI_OK;
}

int learned_llr(const mdgmi_format* fmt, const float* y, int64_t n, double sigma2, float* llr, void* ws,
                size_t ws_bytes, void* stream) {
    if (!fmt || !y || !llr) return MDGMI_E_NULL;
    if (n < 1) return MDGMI_E_SHAPE;
    if (!finite_pos(sigma2)) return MDGMI_E_SIGMA2;
    const LearnedBinding* b = fmt->learned;
    if (!b) return MDGMI_E_UNSUPPORTED;
    if (!routed(b, sigma2)) return mdgmi_llr(fmt, y, n, sigma2, llr, b->exact_path, ws, ws_bytes, stream);
    int rc = check_device(fmt);
    if (rc != MDGMI_OK) return rc;
    const mdgmi_mlp* net = b->net;
    hipStream_t st = (hipStream_t)stream;
    if (!use_fused(net)) {
        size_t need = 0;
        if ((rc = learned_llr_workspace_size(fmt, n, &need)) != MDGMI_OK) return rc;
        if (!ws || ws_bytes < need) return MDGMI_E_WORKSPACE;
        float* x = (float*)ws;
        char* mws = (char*)ws + al(n * net->sizes[0] * 4);
        const MlpWs w = mlp_ws(net, n);
        if (features(y, n, fmt->dim, nullptr, snr_feature(fmt, sigma2), x, st) != hipSuccess ||
            forward(net, x, n, mws, w, st) != hipSuccess ||
            hipMemcpyAsync(llr, mws + w.logits, sizeof(float) * n * fmt->m, hipMemcpyDeviceToDevice, st) !=
                hipSuccess)
            return MDGMI_E_HIP;
        return MDGMI_OK;
    }
    const float* bias[4];
    fused_biases(net, bias);
    const hipError_t e = launch_mlp_llr_fused(net->d_wf, bias, net->sizes[0], net->sizes[4], y, fmt->dim, n, nullptr,
                                              snr_feature(fmt, sigma2), llr, fused_grid(), st);
    return e == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

void learned_free(mdgmi_format* fmt) {
    delete fmt->learned;
    fmt->learned = nullptr;
}

}  // namespace mdgmi

extern "C" {

int mdgmi_mlp_train_workspace_size(const mdgmi_mlp* net, int64_t n, size_t* bytes) {
    if (!net || !bytes) return MDGMI_E_NULL;
    if (n < 1 || n > (int64_t)1 << 30) return MDGMI_E_SHAPE;
    *bytes = (size_t)(al(n * net->sizes[0] * 4) + mlp_ws(net, n).total);
    return MDGMI_OK;
}

int mdgmi_mlp_train_step(mdgmi_mlp* net, const float* y, const float* snr_db, const float* llr_target, int64_t n,
                         float lr, double* loss, void* ws, size_t ws_bytes, void* stream) {
    if (!net || !y || !snr_db || !llr_target || !loss || !ws) return MDGMI_E_NULL;
    if (n < 1 || n > (int64_t)1 << 30) return MDGMI_E_SHAPE;
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return MDGMI_E_ARG;
    size_t need = 0;
    mdgmi_mlp_train_workspace_size(net, n, &need);
    if (ws_bytes < need) return MDGMI_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    float* x = (float*)ws;
    char* mws = (char*)ws + al(n * net->sizes[0] * 4);
    if (features(y, n, net->sizes[0] - 1, snr_db, 0.0f, x, st) != hipSuccess) return MDGMI_E_HIP;
    int rc = mdgmi_mlp_loss_grad(net, x, llr_target, n, loss, mws, (size_t)mlp_ws(net, n).total, stream);
    if (rc != MDGMI_OK) return rc;
    return mdgmi_mlp_adam_step(net, lr, 0.9f, 0.999f, 1e-8f, stream);
}

int mdgmi_mlp_llr_workspace_size(const mdgmi_mlp* net, int64_t n, size_t* bytes) {
    if (!net || !bytes) return MDGMI_E_NULL;
    if (n < 1 || n > (int64_t)1 << 30) return MDGMI_E_SHAPE;
    *bytes = net->fused && g_fused_waves != 0 ? 0 : (size_t)(al(n * net->sizes[0] * 4) + mlp_ws(net, n).total);
    return MDGMI_OK;
}

int mdgmi_mlp_llr(const mdgmi_mlp* net, const float* y, const float* snr_db, int64_t n, float* llr, void* ws,
                  size_t ws_bytes, void* stream) {
    if (!net || !y || !snr_db || !llr) return MDGMI_E_NULL;
    if (n < 1 || n > (int64_t)1 << 30) return MDGMI_E_SHAPE;
    size_t need = 0;
    mdgmi_mlp_llr_workspace_size(net, n, &need);
    if (need > 0 && (!ws || ws_bytes < need)) return MDGMI_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const int dim = net->sizes[0] - 1, out = net->sizes[net->L];
    if (need == 0) {
        const float* bias[4];
        fused_biases(net, bias);
        return launch_mlp_llr_fused(net->d_wf, bias, net->sizes[0], out, y, dim, n, snr_db, 0.0f, llr, fused_grid(),
                                    st) == hipSuccess
                   ? MDGMI_OK
                   : MDGMI_E_HIP;
    }
    float* x = (float*)ws;
    char* mws = (char*)ws + al(n * net->sizes[0] * 4);
    const MlpWs w = mlp_ws(net, n);
    if (features(y, n, dim, snr_db, 0.0f, x, st) != hipSuccess) return MDGMI_E_HIP;
    if (forward(net, x, n, mws, w, st) != hipSuccess) return MDGMI_E_HIP;
    return hipMemcpyAsync(llr, mws + w.logits, sizeof(float) * n * out, hipMemcpyDeviceToDevice, st) == hipSuccess
               ? MDGMI_OK
               : MDGMI_E_HIP;
}

int mdgmi_learned_calibrate_workspace_size(const mdgmi_format* fmt, const mdgmi_mlp* net, int32_t exact_path,
                                           int64_t n, int32_t n_snr, size_t* bytes) {
    if (!fmt || !net || !bytes) return MDGMI_E_NULL;
    if (n < 1 || n_snr < 1) return MDGMI_E_SHAPE;
    size_t ex = 0;
    const int rc = mdgmi_gmi_workspace_size(fmt, n, n_snr, exact_path, &ex);
    if (rc != MDGMI_OK) return rc;
    *bytes = al(2 * (int64_t)n_snr * MDGMI_NFIELDS * 8) + std::max(ex, learned_ws_bytes(net, n));
    return MDGMI_OK;
}

int mdgmi_learned_calibrate(mdgmi_format* fmt, const mdgmi_mlp* net, int32_t exact_path, double max_loss,
                            const float* y, const uint32_t* tx_idx, int64_t n, const double* sigma2_host,
                            int32_t n_snr, double* result_host, void* ws, size_t ws_bytes, void* stream) {
    if (!fmt || !net || !y || !tx_idx || !sigma2_host || !result_host) return MDGMI_E_NULL;
    if (n < 1 || n_snr < 1) return MDGMI_E_SHAPE;
    if (!(max_loss >= 0.0) || !std::isfinite(max_loss)) return MDGMI_E_ARG;
    if (exact_path != MDGMI_PATH_F32_DIRECT && exact_path != MDGMI_PATH_F32_MFMA_F16SPLIT &&
        exact_path != MDGMI_PATH_F32_MFMA_BF16SPLIT && exact_path != MDGMI_PATH_AUTO)
        return MDGMI_E_ARG;
    int rc = check_net_for(fmt, net);
    if (rc != MDGMI_OK) return rc;
    double max_s = 0.0;
    for (int q = 0; q < n_snr; q++) {
        if (!finite_pos(sigma2_host[q])) return MDGMI_E_SIGMA2;
        max_s = std::max(max_s, s_of(sigma2_host[q]));
    }
    int p = 0;
    if ((rc = resolve_path(fmt, exact_path, max_s, &p)) != MDGMI_OK) return rc;
    size_t need = 0;
    if ((rc = mdgmi_learned_calibrate_workspace_size(fmt, net, exact_path, n, n_snr, &need)) != MDGMI_OK) return rc;
    if (!ws || ws_bytes < need) return MDGMI_E_WORKSPACE;
    if ((rc = check_device(fmt)) != MDGMI_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    double* rows = (double*)ws;  // [2][n_snr][MDGMI_NFIELDS]: exact, learned
    char* rest = (char*)ws + al(2 * (int64_t)n_snr * MDGMI_NFIELDS * 8);
    const size_t rest_bytes = ws_bytes - (size_t)al(2 * (int64_t)n_snr * MDGMI_NFIELDS * 8);
    rc = gmi_with_workspace(fmt, y, tx_idx, n, sigma2_host, n_snr, exact_path, rows, rest, rest_bytes, stream);
    if (rc != MDGMI_OK) return rc;
    double* lrows = rows + (size_t)n_snr * MDGMI_NFIELDS;
    for (int q = 0; q < n_snr; q++) {
        rc = learned_gmi_one(fmt, net, y + (size_t)q * n * fmt->dim, tx_idx + (size_t)q * n, n, sigma2_host[q], rest,
                             rest_bytes, lrows + (size_t)q * MDGMI_NFIELDS, st);
        if (rc != MDGMI_OK) return rc;
    }
    std::vector<double> h((size_t)2 * n_snr * MDGMI_NFIELDS);
    if (hipMemcpyAsync(h.data(), rows, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MDGMI_E_HIP;
    LearnedBinding* b = new LearnedBinding();
    b->net = net;
    b->exact_path = exact_path;
    b->max_loss = max_loss;
    for (int q = 0; q < n_snr; q++) {
        const double ge = h[(size_t)q * MDGMI_NFIELDS + MDGMI_F_GMI];
        const double gl = h[((size_t)n_snr + q) * MDGMI_NFIELDS + MDGMI_F_GMI];
        const double loss = ge - gl;
        // paired loss on the same samples; a non-finite estimate keeps the exact path
        const uint8_t r = std::isfinite(ge) && std::isfinite(gl) && loss <= max_loss ? 1 : 0;
        b->s2.push_back(sigma2_host[q]);
        b->route.push_back(r);
        result_host[4 * q + 0] = ge;
        result_host[4 * q + 1] = gl;
        result_host[4 * q + 2] = loss;
        result_host[4 * q + 3] = r;
    }
    learned_free(fmt);
    fmt->learned = b;
    return MDGMI_OK;
}

}  // extern "C"
