// Deterministic final reduction of the per-block partials, and the seeded
// on-device sample generator.
#include "device_common.h"

namespace mdgmi {

namespace {

// One block per SNR point; every thread sums a fixed strided subset of the
// block partials, then a fixed shuffle tree and a fixed per-wave order.
template <int KIND>
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ part, int blocks_per_snr, int64_t n,
                                                int m, double* __restrict__ out) {
    constexpr bool HD = KIND == kReduceHd;
    constexpr int NP = HD ? kNPartHd : kNPart;
    const int q = blockIdx.x;
    const double* p = part + (size_t)q * blocks_per_snr * NP;
    double v[NP] = {};
    for (int b = threadIdx.x; b < blocks_per_snr; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < NP; k++) v[k] += p[(size_t)b * NP + k];
    }
    __shared__ double tot[NP];
    block_reduce_vals<NP>(v, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double N = (double)n;
        double* o = out + (size_t)q * (HD ? MDGMI_NFIELDS_HD : MDGMI_NFIELDS);
        o[MDGMI_F_GMI] = m - tot[0] / N;
        o[MDGMI_F_MI] = m - tot[2] / N;
        double vg = n > 1 ? (tot[1] - tot[0] * tot[0] / N) / (N - 1.0) : 0.0;
        double vm = n > 1 ? (tot[3] - tot[2] * tot[2] / N) / (N - 1.0) : 0.0;
        o[MDGMI_F_SE_GMI] = sqrt(fmax(vg, 0.0) / N);
        o[MDGMI_F_SE_MI] = sqrt(fmax(vm, 0.0) / N);
        o[MDGMI_F_N] = N;
        o[MDGMI_F_NONFINITE] = tot[4];
        if (KIND == kReduceMl) o[MDGMI_F_MI] = o[MDGMI_F_SE_MI] = NAN;  // no MI from max-log metrics
        if (HD) {
            o[MDGMI_F_BER] = tot[5] / (N * m);
            o[MDGMI_F_SER] = tot[6] / N;
        }
    }
}

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
        const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    }
    return c;
}

__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double& z0, double& z1) {
    const double u1 = __dmul_rn(__dadd_rn((double)wa, 0.5), 2.3283064365386963e-10);
    const double u2 = __dmul_rn(__dadd_rn((double)wb, 0.5), 2.3283064365386963e-10);
    const double r = sqrt(__dmul_rn(-2.0, log(u1)));
    const double ang = __dmul_rn(6.283185307179586, u2);
    z0 = __dmul_rn(r, cos(ang));
    z1 = __dmul_rn(r, sin(ang));
}

struct GenArgs {
    int n_snr;
    double sq[kMaxSnrPerLaunch];  // sqrt(sigma2), correctly rounded on the host
};

template <int DIM, bool F64>
__global__ __launch_bounds__(256) void k_generate(const double* __restrict__ X64, const uint32_t* __restrict__ labels,
                                                  int m, uint64_t seed, int64_t n, int snr_slot0, int q0, GenArgs ga,
                                                  void* __restrict__ yout, uint32_t* __restrict__ txout) {
    const int q = blockIdx.y;
    const int64_t snr = q0 + q;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += stride) {
        const uint32_t c0 = (uint32_t)s, c1 = (uint32_t)((uint64_t)s >> 32), c2 = (uint32_t)(snr_slot0 + snr);
        U4 w = philox10(U4{c0, c1, c2, 0u}, k0, k1);
        const uint32_t row = m > 0 ? (w.x >> (32 - m)) : 0u;
        double z[((DIM + 3) / 4) * 4];
#pragma unroll
        for (int call = 0; call < (DIM + 3) / 4; call++) {
            U4 v = philox10(U4{c0, c1, c2, (uint32_t)(1 + call)}, k0, k1);
            box_muller(v.x, v.y, z[4 * call], z[4 * call + 1]);
            box_muller(v.z, v.w, z[4 * call + 2], z[4 * call + 3]);
        }
        const uint32_t slot = labels[row];
        const double sq = ga.sq[q];
        const size_t base = ((size_t)snr * n + s) * DIM;
#pragma unroll
        for (int d = 0; d < DIM; d++) {
            const double v = __dadd_rn(X64[(size_t)slot * DIM + d], __dmul_rn(sq, z[d]));
            if (F64)
                ((double*)yout)[base + d] = v;
            else
                ((float*)yout)[base + d] = (float)v;
        }
        txout[(size_t)snr * n + s] = row;
    }
}

}  // namespace

hipError_t launch_reduce(const double* part, int n_snr, int blocks_per_snr, int64_t n, int m, double* out,
                         hipStream_t st, int kind) {
    if (kind == kReduceHd)
        hipLaunchKernelGGL(k_reduce<kReduceHd>, dim3(n_snr), dim3(256), 0, st, part, blocks_per_snr, n, m, out);
    else if (kind == kReduceMl)
        hipLaunchKernelGGL(k_reduce<kReduceMl>, dim3(n_snr), dim3(256), 0, st, part, blocks_per_snr, n, m, out);
    else
        hipLaunchKernelGGL(k_reduce<kReduceGmi>, dim3(n_snr), dim3(256), 0, st, part, blocks_per_snr, n, m, out);
    return hipGetLastError();
}

hipError_t launch_generate(const mdgmi_format* f, uint64_t seed, const double* sigma2, int n_snr, int64_t n,
                           int snr_slot0, void* y, uint32_t* tx, bool f64, hipStream_t st) {
    for (int q0 = 0; q0 < n_snr; q0 += kMaxSnrPerLaunch) {
        GenArgs ga;
        ga.n_snr = n_snr - q0 < kMaxSnrPerLaunch ? n_snr - q0 : kMaxSnrPerLaunch;
        for (int q = 0; q < ga.n_snr; q++) ga.sq[q] = std::sqrt(sigma2[q0 + q]);
        int64_t want = (n + 255) / 256;
        int cap = device_cu_count() * 16;
        dim3 grid((unsigned)(want < cap ? want : cap), ga.n_snr), block(256);
#define MDGMI_GEN(D)                                                                                       \
    case D:                                                                                                \
        if (f64)                                                                                           \
            hipLaunchKernelGGL((k_generate<D, true>), grid, block, 0, st, f->d_X64, f->d_labels, f->m, seed, \
                               n, snr_slot0, q0, ga, y, tx);                                               \
        else                                                                                               \
            hipLaunchKernelGGL((k_generate<D, false>), grid, block, 0, st, f->d_X64, f->d_labels, f->m,    \
                               seed, n, snr_slot0, q0, ga, y, tx);                                         \
        break;
        switch (f->dim) {
            MDGMI_GEN(1)
            MDGMI_GEN(2)
            MDGMI_GEN(4)
            MDGMI_GEN(8)
            default:
                return hipErrorInvalidValue;
        }
#undef MDGMI_GEN
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace mdgmi
