// s-optimised GMI and per-bit GMI of given LLRs (any demapper: exact,
// max-log, learned).
//
// For LLRs lambda_ik and sent bits b_k(i), with v_ik = (2 b_k(i) - 1) lambda_ik,
//     GMI(s) = m - (1/n) sum_i sum_k log2(1 + exp(-s v_ik)),   s >= 0,
// is the GMI of a bit-metric decoder that uses the LLRs scaled by s; the
// s-optimised GMI is its maximum over s. Each term log(1 + e^{-s v}) is
// convex in s, so GMI(s) is concave and the maximum is where the derivative
// of the total cost
//     C'(s)  = -sum v sigma(-s v),     C''(s) = sum v^2 sigma(s v) sigma(-s v)
// vanishes. The search runs on the device: a pass kernel evaluates the cost
// and both derivatives at the current s (FP64 sums, fixed reduction order),
// a one-block update kernel takes a Newton step kept inside the bracket
// [lo, hi] of the sign changes of C' (bisection, or doubling while no upper
// end is known), and the host only enqueues a fixed number of pass/update
// pairs; once the step has converged the remaining kernels return at once.
#include <algorithm>

#include "device_common.h"

namespace mdgmi {

namespace {

constexpr int kSoptThreads = 256;
constexpr int kSoptPart = 6;      // sum C, sum C^2, sum C', sum C'', sum v, non-finite
constexpr int kSoptPasses = 64;
// state: s, lo, hi, done, iterations, best GMI so far
constexpr int kStS = 0, kStLo = 1, kStHi = 2, kStDone = 3, kStIter = 4, kStBest = 5, kStateLen = 8;

__global__ void k_sopt_init(double* __restrict__ state, double* __restrict__ out) {
    if (threadIdx.x == 0) {
        state[kStS] = 1.0;
        state[kStLo] = 0.0;
        state[kStHi] = INFINITY;
        state[kStDone] = 0.0;
        state[kStIter] = 0.0;
        state[kStBest] = -INFINITY;
    }
    if (threadIdx.x < MDGMI_NFIELDS_S) out[threadIdx.x] = NAN;
}

// Cost per bit and its s-derivatives at z = s v, in the precision of the LLRs.
template <typename T>
__device__ __forceinline__ void term(T v, T s, T& c, T& d1, T& d2) {
    const T z = s * v;
    const T e = exp(-fabs(z));                    // e^{-|z|}
    c = (z < T(0) ? -z : T(0)) + log1p(e);        // log(1 + e^{-z})
    const T sneg = z >= T(0) ? e / (T(1) + e) : T(1) / (T(1) + e);   // sigma(-z)
    d1 = -v * sneg;
    d2 = v * v * (e / ((T(1) + e) * (T(1) + e)));
}

template <typename T>
__global__ __launch_bounds__(kSoptThreads) void k_sopt_pass(const T* __restrict__ llr,
                                                             const uint32_t* __restrict__ tx,
                                                             const uint32_t* __restrict__ labels, int M, int64_t n,
                                                             int m, const double* __restrict__ state,
                                                             double* __restrict__ part) {
    if (state[kStDone] != 0.0) return;  // uniform over the grid
    const T s = (T)state[kStS];
    double sc = 0.0, sc2 = 0.0, sd1 = 0.0, sd2 = 0.0, sv = 0.0, bad = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t row = tx[i];
        const bool row_ok = row < (uint32_t)M;
        const uint32_t slot = labels[row_ok ? row : 0u];
        T c = 0, d1 = 0, d2 = 0, vs = 0;
        for (int k = 0; k < m; k++) {
            const T lam = llr[i * m + k];
            const T v = ((slot >> k) & 1u) ? lam : -lam;
            T ck, ak, bk;
            term<T>(v, s, ck, ak, bk);
            c += ck;
            d1 += ak;
            d2 += bk;
            vs += v;
        }
        double cb = (double)c * kLog2e;  // bits
        if (!row_ok) cb = NAN;
        sc += cb;
        sc2 += cb * cb;
        sd1 += (double)d1 * kLog2e;
        sd2 += (double)d2 * kLog2e;
        sv += (double)vs;
        bad += __builtin_isfinite(cb) ? 0.0 : 1.0;
    }
    double v[kSoptPart] = {sc, sc2, sd1, sd2, sv, bad};
    block_reduce_vals<kSoptPart>(v, part + (size_t)blockIdx.x * kSoptPart);
}

// tol: relative step (and bracket) size taken as converged; it follows the
// precision of the LLRs, whose rounding bounds how small a Newton step the
// derivative sums can resolve.
__global__ __launch_bounds__(256) void k_sopt_update(const double* __restrict__ part, int nblocks, int64_t n, int m,
                                                     double tol, double* __restrict__ state,
                                                     double* __restrict__ out) {
    if (state[kStDone] != 0.0) return;
    double v[kSoptPart] = {};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < kSoptPart; k++) v[k] += part[(size_t)b * kSoptPart + k];
    }
    __shared__ double tot[kSoptPart];
    block_reduce_vals<kSoptPart>(v, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double N = (double)n, s = state[kStS];
    const double gmi = m - tot[0] / N;
    const double var = n > 1 ? (tot[1] - tot[0] * tot[0] / N) / (N - 1.0) : 0.0;
    const double se = sqrt(fmax(var, 0.0) / N);
    const int it = (int)state[kStIter];
    if (it == 0) {  // s = 1
        out[MDGMI_S_GMI1] = gmi;
        out[MDGMI_S_SE1] = se;
        out[MDGMI_S_N] = N;
        out[MDGMI_S_NONFINITE] = tot[5];
        if (tot[5] > 0.0) {  // non-finite LLRs or sent rows out of range: estimates stay NaN
            out[MDGMI_S_ITERS] = 1.0;
            state[kStDone] = 1.0;
            return;
        }
        if (!(tot[4] > 0.0)) {
            // C'(0) = -sum v / 2 >= 0: the cost only grows with s, the
            // maximum is GMI(0) = 0 at s = 0
            out[MDGMI_S_S] = 0.0;
            out[MDGMI_S_GMI] = 0.0;
            out[MDGMI_S_SE] = 0.0;
            out[MDGMI_S_NGMI] = 0.0;
            out[MDGMI_S_ITERS] = 1.0;
            state[kStDone] = 1.0;
            return;
        }
    }
    if (gmi > state[kStBest]) {  // keep the best point evaluated
        state[kStBest] = gmi;
        out[MDGMI_S_S] = s;
        out[MDGMI_S_GMI] = gmi;
        out[MDGMI_S_SE] = se;
        out[MDGMI_S_NGMI] = gmi / m;
    }
    out[MDGMI_S_ITERS] = it + 1;
    state[kStIter] = it + 1;
    const double d1 = tot[2], d2 = tot[3];
    if (d1 == 0.0) {
        state[kStDone] = 1.0;
        return;
    }
    double lo = state[kStLo], hi = state[kStHi];
    if (d1 > 0.0)
        hi = s;
    else
        lo = s;
    const double step = d2 > 0.0 ? d1 / d2 : NAN;
    // converged: the Newton step is below the tolerance (tested before the
    // bracket, which a step of rounding size can touch)
    if (fabs(step) <= tol * s) {
        state[kStDone] = 1.0;
        return;
    }
    double sn = s - step;
    if (!(sn > lo && sn < hi)) sn = hi < INFINITY ? 0.5 * (lo + hi) : 2.0 * s;
    state[kStLo] = lo;
    state[kStHi] = hi;
    state[kStS] = sn;
    if (hi < INFINITY && hi - lo <= tol * hi) state[kStDone] = 1.0;
}

// ---- per-bit GMI of given LLRs (s = 1) ---------------------------------
// GMI_k = 1 - mean_i log2(1 + exp(-v_ik)): per-bit FP64 sums of the cost and
// its square, one pass, then a one-block finish in a fixed order.
constexpr int kBitsPart = 2 * MDGMI_MAX_BITS + 1;

template <typename T>
__global__ __launch_bounds__(kSoptThreads) void k_bits_pass(const T* __restrict__ llr,
                                                             const uint32_t* __restrict__ tx,
                                                             const uint32_t* __restrict__ labels, int M, int64_t n,
                                                             int m, double* __restrict__ part) {
    double v[kBitsPart] = {};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t row = tx[i];
        const bool row_ok = row < (uint32_t)M;
        const uint32_t slot = labels[row_ok ? row : 0u];
        bool fin = row_ok;
#pragma unroll
        for (int k = 0; k < MDGMI_MAX_BITS; k++) {
            if (k < m) {
                const T lam = llr[i * m + k];
                const T u = ((slot >> k) & 1u) ? -lam : lam;   // cost = log(1 + e^u)
                double c = (double)((u > T(0) ? u : T(0)) + log1p(exp(-fabs(u)))) * kLog2e;
                if (!row_ok) c = NAN;
                fin = fin && __builtin_isfinite(c);
                v[2 * k] += c;
                v[2 * k + 1] += c * c;
            }
        }
        v[2 * MDGMI_MAX_BITS] += fin ? 0.0 : 1.0;
    }
    block_reduce_vals<kBitsPart>(v, part + (size_t)blockIdx.x * kBitsPart);
}

__global__ __launch_bounds__(256) void k_bits_finish(const double* __restrict__ part, int nblocks, int64_t n, int m,
                                                     double* __restrict__ out) {
    double v[kBitsPart] = {};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < kBitsPart; k++) v[k] += part[(size_t)b * kBitsPart + k];
    }
    __shared__ double tot[kBitsPart];
    block_reduce_vals<kBitsPart>(v, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double N = (double)n;
    for (int k = 0; k < m; k++) {
        const double s1 = tot[2 * k], s2 = tot[2 * k + 1];
        const double var = n > 1 ? (s2 - s1 * s1 / N) / (N - 1.0) : 0.0;
        out[2 * k] = 1.0 - s1 / N;
        out[2 * k + 1] = sqrt(fmax(var, 0.0) / N);
    }
    out[2 * m] = N;
    out[2 * m + 1] = tot[2 * MDGMI_MAX_BITS];
}

int sopt_blocks(int64_t n) {
    const int64_t want = (n + kSoptThreads - 1) / kSoptThreads;
    const int64_t cap = (int64_t)device_cu_count() * 8;
    return (int)std::max<int64_t>(1, std::min(want, cap));
}

}  // namespace

size_t bits_workspace_bytes(int64_t n) { return (size_t)sopt_blocks(n) * kBitsPart * sizeof(double); }

hipError_t launch_bits(const mdgmi_format* f, const void* llr, bool f64, const uint32_t* tx, int64_t n, double* out,
                       void* ws, hipStream_t st) {
    double* part = (double*)ws;
    const int nb = sopt_blocks(n);
    if (f64)
        hipLaunchKernelGGL(k_bits_pass<double>, dim3(nb), dim3(kSoptThreads), 0, st, (const double*)llr, tx,
                           f->d_labels, f->M, n, f->m, part);
    else
        hipLaunchKernelGGL(k_bits_pass<float>, dim3(nb), dim3(kSoptThreads), 0, st, (const float*)llr, tx,
                           f->d_labels, f->M, n, f->m, part);
    hipLaunchKernelGGL(k_bits_finish, dim3(1), dim3(256), 0, st, part, nb, n, f->m, out);
    return hipGetLastError();
}

size_t sopt_workspace_bytes(int64_t n) {
    return (size_t)(kStateLen + (size_t)sopt_blocks(n) * kSoptPart) * sizeof(double);
}

hipError_t launch_sopt(const mdgmi_format* f, const void* llr, bool f64, const uint32_t* tx, int64_t n, double* out,
                       void* ws, hipStream_t st) {
    double* state = (double*)ws;
    double* part = state + kStateLen;
    const int nb = sopt_blocks(n);
    hipLaunchKernelGGL(k_sopt_init, dim3(1), dim3(64), 0, st, state, out);
    for (int it = 0; it < kSoptPasses; it++) {
        if (f64)
            hipLaunchKernelGGL(k_sopt_pass<double>, dim3(nb), dim3(kSoptThreads), 0, st, (const double*)llr, tx,
                               f->d_labels, f->M, n, f->m, state, part);
        else
            hipLaunchKernelGGL(k_sopt_pass<float>, dim3(nb), dim3(kSoptThreads), 0, st, (const float*)llr, tx,
                               f->d_labels, f->M, n, f->m, state, part);
        hipLaunchKernelGGL(k_sopt_update, dim3(1), dim3(256), 0, st, part, nb, n, f->m, f64 ? 1e-12 : 1e-7, state,
                           out);
    }
    return hipGetLastError();
}

}  // namespace mdgmi
