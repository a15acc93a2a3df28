// Ragged batch, the kind that runs on the per-sample 4x4-block MFMA shape
// (small_core.h): a persistent grid over its items, each block pulling the
// next item from the kind's counter as the other kinds do (batch.hip). Its
// own file so that the MFMA accumulators stay in ordinary VGPRs (a build
// flag per file) without touching the 32 x 32 kind.
#include <algorithm>

#include "batch.h"
#include "small_core.h"

namespace mdgmi {

namespace {

constexpr int kSmallWaves = kSmallItemAlign / 64;

// A 4x4-shape item: each wave loads the instance's operand registers and
// takes batches of 64 consecutive samples of [s0, s1) (s0 is a multiple of
// kSmallItemAlign); lanes past s1 count nothing.
template <int DIM, int NG>
__device__ __forceinline__ void run_small_item(const BatchInst& D, int64_t s0, int64_t s1, CostAcc& acc) {
    const uint2* img = (const uint2*)D.img;
    small::half4 a[small::Sets<NG>::value][small::Nk4<DIM>::value];
    small::load_image<DIM, NG>(img, 4 * NG, a);
    HdAcc hd;
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t b0 = s0 + 64 * wave; b0 < s1; b0 += 64 * kSmallWaves)
        small::small_sample<DIM, NG, kModeGmi>(a, img, D.y, D.tx, b0 + lane, s1, D.s, D.X32, D.labels, nullptr,
                                               acc, hd);
}

template <int DIM>
__device__ __forceinline__ void run_small_dim(const BatchInst& D, int64_t s0, int64_t s1, CostAcc& acc) {
    switch (D.M) {
        case 4: run_small_item<DIM, 1>(D, s0, s1, acc); break;
        case 8: run_small_item<DIM, 2>(D, s0, s1, acc); break;
        case 16: run_small_item<DIM, 4>(D, s0, s1, acc); break;
        case 32: run_small_item<DIM, 8>(D, s0, s1, acc); break;
        case 64: run_small_item<DIM, 16>(D, s0, s1, acc); break;
        case 128: run_small_item<DIM, 32>(D, s0, s1, acc); break;
        case 256: run_small_item<DIM, 64>(D, s0, s1, acc); break;
        default:
            if constexpr (DIM < 8) run_small_item<DIM, 128>(D, s0, s1, acc);
            break;
    }
}

__global__ __launch_bounds__(kSmallWaves * 64) void k_batch_small(const BatchInst* __restrict__ insts,
                                                                   const BatchItem* __restrict__ items, int i0,
                                                                   int i1, unsigned* __restrict__ counter,
                                                                   double* __restrict__ part) {
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = i0 + (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it >= i1) break;
        const BatchItem I = items[it];
        const BatchInst D = insts[I.inst];
        CostAcc acc;
        if (D.dim == 1)
            run_small_dim<1>(D, I.s0, I.s1, acc);
        else if (D.dim == 2)
            run_small_dim<2>(D, I.s0, I.s1, acc);
        else if (D.dim == 4)
            run_small_dim<4>(D, I.s0, I.s1, acc);
        else
            run_small_dim<8>(D, I.s0, I.s1, acc);
        block_reduce_store(acc, part + (size_t)it * kNPart);
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_batch_small(const BatchInst* insts, const BatchItem* items, int i0, int i1, unsigned* counter,
                              double* part, hipStream_t st) {
    // one resident round: the blocks per CU that the compiled kernel's
    // registers allow (one kernel serves every (dim, M) of the kind, so the
    // largest formats' operand registers set it), times the CUs. Separate
    // kernels per register class ran the 1/100-scale ragged set slower (three
    // launches, each with a partial last round) and the full set no faster.
    static const int per_cu = [] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void*)k_batch_small, kSmallWaves * 64, 0) !=
                hipSuccess ||
            b < 1)
            b = 1;
        return b;
    }();
    const int grid = std::max(1, std::min(i1 - i0, device_cu_count() * per_cu));
    hipLaunchKernelGGL(k_batch_small, dim3(grid), dim3(kSmallWaves * 64), 0, st, insts, items, i0, i1, counter,
                       part);
    return hipGetLastError();
}

}  // namespace mdgmi
