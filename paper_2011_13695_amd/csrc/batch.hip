// Ragged batch: many (format, SNR, sample-count) instances in one persistent
// launch.
//
// The host cuts every instance into items (contiguous sample ranges of about
// kItemPairs sample*points each, aligned to the kernel's sample tiles) and
// lists them instance by instance: MFMA instances, then direct ones, largest
// constellations first within each. One persistent grid per kind pulls items
// from its own atomic counter; for each item a block
// dispatches on the instance's (dim, M) to the very device functions the
// per-SNR kernels run (mfma_core.h / direct_core.h; the 4x4-shape kind in
// batch_small.hip with small_core.h), staging the
// instance's MFMA A image in LDS when it fits and keeping it there while the
// block stays on that instance. Every item writes its own FP64 partials, and
// one block per instance adds its items' partials in item order, so the
// result does not depend on which block ran which item.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "batch.h"
#include "direct_core.h"
#include "mfma_core.h"
#include "small_core.h"

namespace mdgmi {

namespace {

// MFMA items run in blocks of 16 waves (one block per CU holds a 128 KiB
// image in LDS; 4 waves per SIMD), direct items in blocks of 8 waves.
constexpr int kMfmaWaves = 16;
constexpr int kDirectWaves = 8;
constexpr int kLdsCapU4 = 128 * 1024 / 16;  // A images up to 128 KiB are staged in LDS

template <int DIM, int G, bool IN_LDS>
__device__ __forceinline__ void run_mfma_item(const BatchInst& D, const uint4* __restrict__ A, int64_t s0,
                                              int64_t s1, CostAcc& acc) {
    const int wave = threadIdx.x >> 6;
    const int64_t ct0 = s0 >> 5, ct1 = (s1 + 31) >> 5;
    for (int64_t ct = ct0 + wave; ct < ct1; ct += kMfmaWaves)
        mfma::mfma_coltile<DIM, 1, G, false>(A, D.y, D.tx, D.n, ct, D.M, D.m, D.ntiles, D.s, D.X32, D.labels,
                                             nullptr, acc);
}

template <int DIM, int CHB, int G>
__device__ __forceinline__ void run_direct_item(const BatchInst& D, int64_t s0, int64_t s1, CostAcc& acc) {
    for (int64_t i = s0 + threadIdx.x; i < s1; i += blockDim.x)
        direct::direct_sample<DIM, CHB, G, false>((const float*)D.img, D.y, D.tx, i, D.M, D.m, D.s, D.X32,
                                                  D.labels, nullptr, acc);
}

template <int DIM>
__device__ __forceinline__ void run_direct_dim(const BatchInst& D, int64_t s0, int64_t s1, CostAcc& acc) {
    switch (D.dvar) {
        case 0: run_direct_item<DIM, 1, 1>(D, s0, s1, acc); break;
        case 1: run_direct_item<DIM, 2, 1>(D, s0, s1, acc); break;
        case 2: run_direct_item<DIM, 3, 1>(D, s0, s1, acc); break;
        case 3: run_direct_item<DIM, 4, 1>(D, s0, s1, acc); break;
        case 4: run_direct_item<DIM, 4, 2>(D, s0, s1, acc); break;
        default: run_direct_item<DIM, 4, 4>(D, s0, s1, acc); break;
    }
}

// MFMA batch items need M >= 128, i.e. at least 4 tiles: groups of 8 tiles
// from 8 tiles up, else 4.
template <int DIM>
__device__ __forceinline__ void run_mfma_dim(const BatchInst& D, bool in_lds, const uint4* lds, int64_t s0,
                                             int64_t s1, CostAcc& acc) {
    const uint4* g = (const uint4*)D.img;
    if (D.ntiles >= 8) {
        if (in_lds)
            run_mfma_item<DIM, 8, true>(D, lds, s0, s1, acc);
        else
            run_mfma_item<DIM, 8, false>(D, g, s0, s1, acc);
    } else {
        if (in_lds)
            run_mfma_item<DIM, 4, true>(D, lds, s0, s1, acc);
        else
            run_mfma_item<DIM, 4, false>(D, g, s0, s1, acc);
    }
}

// Persistent grid over items [i0, i1) of one kind, pulled through *counter
// (zeroed before the launch). Every wave leaves the loop on the same item
// index, read once per round from LDS.
template <int KIND>
__global__ __launch_bounds__((KIND == kKindMfma ? kMfmaWaves : kDirectWaves) * 64) void k_batch(
    const BatchInst* __restrict__ insts, const BatchItem* __restrict__ items, int i0, int i1,
    unsigned* __restrict__ counter, double* __restrict__ part) {
    extern __shared__ uint4 lds[];
    __shared__ int s_item, s_staged;
    if (threadIdx.x == 0) s_staged = -1;
    for (;;) {
        if (threadIdx.x == 0) s_item = i0 + (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        const int staged = s_staged;
        __syncthreads();
        if (it >= i1) break;
        const BatchItem I = items[it];
        const BatchInst D = insts[I.inst];
        CostAcc acc;
        if (KIND == kKindMfma) {
            const bool in_lds = D.img_u4 <= kLdsCapU4;
            if (in_lds && staged != I.inst) {
                const uint4* g = (const uint4*)D.img;
                for (int k = threadIdx.x; k < D.img_u4; k += blockDim.x) lds[k] = g[k];
                __syncthreads();
                if (threadIdx.x == 0) s_staged = I.inst;
            }
            if (D.dim == 2)
                run_mfma_dim<2>(D, in_lds, lds, I.s0, I.s1, acc);
            else if (D.dim == 4)
                run_mfma_dim<4>(D, in_lds, lds, I.s0, I.s1, acc);
            else
                run_mfma_dim<8>(D, in_lds, lds, I.s0, I.s1, acc);
        } else {
            if (D.dim == 1)
                run_direct_dim<1>(D, I.s0, I.s1, acc);
            else if (D.dim == 2)
                run_direct_dim<2>(D, I.s0, I.s1, acc);
            else if (D.dim == 4)
                run_direct_dim<4>(D, I.s0, I.s1, acc);
            else
                run_direct_dim<8>(D, I.s0, I.s1, acc);
        }
        block_reduce_store(acc, part + (size_t)it * kNPart);
        __syncthreads();
    }
}

// Images of every instance: one thread per (instance, slot).
__global__ void k_batch_images(const BatchImg* __restrict__ imgs, int n_inst, int64_t total_slots,
                               char* __restrict__ base) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total_slots) return;
    int lo = 0, hi = n_inst - 1;  // last instance with slot_off <= g
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (imgs[mid].slot_off <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    const BatchImg I = imgs[lo];
    const int slot = (int)(g - I.slot_off);
    if (I.kind == kKindMfma) {
        uint4* dst = (uint4*)(base + I.img_off);
        if (I.dim == 2)
            mfma::image_slot<2>(I.X64, I.M, I.ntiles, I.s64, slot, dst);
        else if (I.dim == 4)
            mfma::image_slot<4>(I.X64, I.M, I.ntiles, I.s64, slot, dst);
        else
            mfma::image_slot<8>(I.X64, I.M, I.ntiles, I.s64, slot, dst);
    } else if (I.kind == kKindSmall) {
        uint2* dst = (uint2*)(base + I.img_off);
        if (I.dim == 1)
            small::image_slot<1>(I.X64, I.s64, slot, dst + (size_t)slot * small::Nk4<1>::value);
        else if (I.dim == 2)
            small::image_slot<2>(I.X64, I.s64, slot, dst + (size_t)slot * small::Nk4<2>::value);
        else if (I.dim == 4)
            small::image_slot<4>(I.X64, I.s64, slot, dst + (size_t)slot * small::Nk4<4>::value);
        else
            small::image_slot<8>(I.X64, I.s64, slot, dst + (size_t)slot * small::Nk4<8>::value);
    } else {
        const int rec = ((I.dim + 1 + 3) / 4) * 4;
        direct::direct_record(I.X64, I.dim, rec, I.s64, slot, (float*)(base + I.img_off) + (size_t)slot * rec);
    }
}

__global__ void k_zero_counters(unsigned* c) {
    if (blockIdx.x == 0 && threadIdx.x < 3) c[threadIdx.x] = 0u;
}

int direct_variant(int m) { return m <= 1 ? 0 : m == 2 ? 1 : m == 3 ? 2 : m == 4 ? 3 : m == 5 ? 4 : 5; }

size_t al(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

int batch_kind_for(const mdgmi_format* f, double s, int path) {
    // the 32 x 32 shape takes M >= 128 in a batch (one-dimensional formats
    // excepted); the 4x4 shape the formats it serves, where the per-SNR
    // fp16-split path would run them on it
    const bool mfma_ok = f->dim != 1 && f->M >= 128 && mfma_supported(f, s);
    const bool small_ok = small_shape_fits(f) && mfma_supported(f, s) && prefers_small(f);
    if (path == MDGMI_PATH_F32_DIRECT) return kKindDirect;
    if (path == MDGMI_PATH_F32_MFMA_F16SPLIT) return small_ok ? kKindSmall : (mfma_ok ? kKindMfma : -1);
    // AUTO: the tuned choice for this (dim, M) where one exists
    int tuned = tuned_batch_kind(f->dim, f->M);
    if (tuned == kKindDirect) return kKindDirect;
    if (small_ok) return kKindSmall;
    return mfma_ok ? kKindMfma : kKindDirect;
}

int plan_batch(const mdgmi_instance* inst, int n_inst, int path, int64_t item_pairs, BatchPlan& P) {
    P = BatchPlan();
    P.n_inst = n_inst;
    std::vector<int> kind(n_inst);
    for (int q = 0; q < n_inst; q++) {
        const double s = kLog2e / (2.0 * inst[q].sigma2);
        kind[q] = batch_kind_for(inst[q].fmt, s, path);
        if (kind[q] < 0) return MDGMI_E_UNSUPPORTED;
    }
    // images
    P.imgs.resize(n_inst);
    size_t img_bytes = 0;
    int64_t slots = 0;
    for (int q = 0; q < n_inst; q++) {
        const mdgmi_format* f = inst[q].fmt;
        BatchImg& I = P.imgs[q];
        I.X64 = f->d_X64;
        I.s64 = kLog2e / (2.0 * inst[q].sigma2);
        I.dim = f->dim;
        I.M = f->M;
        I.kind = kind[q];
        I.ntiles = (f->M + 31) / 32;
        I.slot_off = slots;
        I.img_off = img_bytes;
        size_t bytes;
        if (kind[q] == kKindMfma) {
            bytes = (size_t)I.ntiles * (f->dim == 8 ? 2 : 1) * 64 * 16;
            slots += (int64_t)I.ntiles * 32;
        } else if (kind[q] == kKindSmall) {
            bytes = (size_t)f->M * ((3 * f->dim + 2 + 3) / 4) * 8;
            slots += f->M;
        } else {
            bytes = (size_t)f->M * (((f->dim + 1 + 3) / 4) * 4) * sizeof(float);
            slots += f->M;
        }
        img_bytes += al(bytes);
    }
    P.total_slots = slots;
    // MFMA instances first, then 4x4-shape ones, then direct ones (each kind
    // has its own kernel); within a kind, decreasing M (then input order) so
    // the cheap ones form the tail
    auto rank = [&](int q) { return kind[q] == kKindMfma ? 0 : (kind[q] == kKindSmall ? 1 : 2); };
    std::vector<int> order(n_inst);
    for (int q = 0; q < n_inst; q++) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (kind[a] != kind[b]) return rank(a) < rank(b);
        return inst[a].fmt->M > inst[b].fmt->M;
    });
    P.insts.resize(n_inst);
    // items are grouped per instance in the order above; (first, end) per
    // caller instance lets the reduction find them
    std::vector<int32_t> first_of(n_inst), count_of(n_inst);
    for (int oi = 0; oi < n_inst; oi++) {
        const int q = order[oi];
        const mdgmi_format* f = inst[q].fmt;
        const int64_t n = inst[q].n;
        const int align = kind[q] == kKindMfma ? 32 * kMfmaWaves
                                               : (kind[q] == kKindSmall ? kSmallItemAlign : 64 * kDirectWaves);
        int64_t per = item_pairs / f->M;
        per = std::max<int64_t>(align, per / align * align);
        first_of[q] = (int32_t)P.items.size();
        for (int64_t s0 = 0; s0 < n; s0 += per) {
            BatchItem it;
            it.inst = q;
            it.pad = 0;
            it.s0 = s0;
            it.s1 = std::min(n, s0 + per);
            P.items.push_back(it);
        }
        count_of[q] = (int32_t)P.items.size() - first_of[q];
    }
    P.n_mfma_items = P.n_small_items = 0;
    for (const BatchItem& it : P.items) {
        if (kind[it.inst] == kKindMfma) P.n_mfma_items++;
        if (kind[it.inst] == kKindSmall) P.n_small_items++;
    }
    P.item_range.resize(2 * (size_t)n_inst);
    for (int q = 0; q < n_inst; q++) {
        P.item_range[2 * q] = first_of[q];
        P.item_range[2 * q + 1] = first_of[q] + count_of[q];
    }
    for (int q = 0; q < n_inst; q++) {
        const mdgmi_format* f = inst[q].fmt;
        BatchInst& D = P.insts[q];
        D.y = (const float*)inst[q].y;
        D.tx = inst[q].tx_idx;
        D.img = nullptr;  // set once the workspace base is known
        D.X32 = f->d_X32;
        D.labels = f->d_labels;
        D.n = inst[q].n;
        D.s = (float)(kLog2e / (2.0 * inst[q].sigma2));
        D.dim = f->dim;
        D.M = f->M;
        D.m = f->m;
        D.ntiles = (f->M + 31) / 32;
        D.kind = kind[q];
        D.dvar = direct_variant(f->m);
        D.img_u4 = kind[q] == kKindMfma ? (int)(D.ntiles * (f->dim == 8 ? 2 : 1) * 64) : 0;
    }
    P.max_lds_u4 = 0;
    for (int q = 0; q < n_inst; q++)
        if (P.insts[q].kind == kKindMfma && P.insts[q].img_u4 <= kLdsCapU4)
            P.max_lds_u4 = std::max(P.max_lds_u4, P.insts[q].img_u4);
    // workspace layout
    size_t o = 0;
    P.off_insts = o;
    o += al(sizeof(BatchInst) * n_inst);
    P.off_imgs = o;
    o += al(sizeof(BatchImg) * n_inst);
    P.off_items = o;
    o += al(sizeof(BatchItem) * P.items.size());
    P.off_range = o;
    o += al(sizeof(int32_t) * P.item_range.size());
    P.off_part = o;
    o += al(sizeof(double) * kNPart * P.items.size());
    P.off_counter = o;
    o += al(3 * sizeof(unsigned));
    P.off_images = o;
    o += img_bytes;
    P.bytes = o;
    return MDGMI_OK;
}

void bind_batch(BatchPlan& P, char* base) {
    P.base = base;
    for (int q = 0; q < P.n_inst; q++) P.insts[q].img = base + P.off_images + P.imgs[q].img_off;
}

hipError_t upload_batch(const BatchPlan& P, hipStream_t st) {
    hipError_t e;
    if ((e = hipMemcpyAsync(P.base + P.off_insts, P.insts.data(), sizeof(BatchInst) * P.insts.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(P.base + P.off_imgs, P.imgs.data(), sizeof(BatchImg) * P.imgs.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(P.base + P.off_items, P.items.data(), sizeof(BatchItem) * P.items.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(P.base + P.off_range, P.item_range.data(), sizeof(int32_t) * P.item_range.size(),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
        return e;
    const int64_t slots = P.total_slots;
    hipLaunchKernelGGL(k_batch_images, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, st,
                       (const BatchImg*)(P.base + P.off_imgs), P.n_inst, slots, P.base + P.off_images);
    return hipGetLastError();
}

// Reduction over item ranges given as (first, end) pairs per instance.
__global__ __launch_bounds__(256) void k_batch_reduce_ranges(const double* __restrict__ part,
                                                             const int32_t* __restrict__ range,
                                                             const BatchInst* __restrict__ insts,
                                                             double* __restrict__ out) {
    const int q = blockIdx.x;
    const int i0 = range[2 * q], i1 = range[2 * q + 1];
    double v[kNPart] = {0, 0, 0, 0, 0};
    for (int b = i0 + threadIdx.x; b < i1; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < kNPart; k++) v[k] += part[(size_t)b * kNPart + k];
    }
    CostAcc a;
    a.sg = v[0];
    a.sg2 = v[1];
    a.sm = v[2];
    a.sm2 = v[3];
    a.bad = v[4];
    __shared__ double tot[kNPart];
    block_reduce_store(a, tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t n = insts[q].n;
        const double N = (double)n;
        const int m = insts[q].m;
        double* o = out + (size_t)q * MDGMI_NFIELDS;
        o[MDGMI_F_GMI] = m - tot[0] / N;
        o[MDGMI_F_MI] = m - tot[2] / N;
        const double vg = n > 1 ? (tot[1] - tot[0] * tot[0] / N) / (N - 1.0) : 0.0;
        const double vm = n > 1 ? (tot[3] - tot[2] * tot[2] / N) / (N - 1.0) : 0.0;
        o[MDGMI_F_SE_GMI] = sqrt(fmax(vg, 0.0) / N);
        o[MDGMI_F_SE_MI] = sqrt(fmax(vm, 0.0) / N);
        o[MDGMI_F_N] = N;
        o[MDGMI_F_NONFINITE] = tot[4];
    }
}

hipError_t prepare_batch_kernel() {
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        err = hipFuncSetAttribute((const void*)k_batch<kKindMfma>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  kLdsCapU4 * 16);
    });
    return err;
}

hipError_t launch_batch(const BatchPlan& P, double* out, hipStream_t st) {
    unsigned* counter = (unsigned*)(P.base + P.off_counter);
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, counter);
    const BatchInst* insts = (const BatchInst*)(P.base + P.off_insts);
    const BatchItem* items = (const BatchItem*)(P.base + P.off_items);
    double* part = (double*)(P.base + P.off_part);
    const int n_items = (int)P.items.size(), n_mfma = P.n_mfma_items;
    if (n_mfma > 0) {
        // one resident round: blocks per CU limited by the largest LDS image
        // and by 16 waves per CU
        const size_t lds = (size_t)P.max_lds_u4 * 16;
        const int by_lds = lds > 0 ? std::max(1, (int)((160 * 1024) / (lds + 2048))) : 1;
        const int per_cu = std::min(by_lds, 1);
        const int grid = std::max(1, std::min(n_mfma, device_cu_count() * per_cu));
        hipLaunchKernelGGL(k_batch<kKindMfma>, dim3(grid), dim3(kMfmaWaves * 64), lds, st, insts, items, 0, n_mfma,
                           counter, part);
    }
    const int n_small = P.n_small_items, d0 = n_mfma + n_small;
    if (n_small > 0) {
        const hipError_t e = launch_batch_small(insts, items, n_mfma, d0, counter + 1, part, st);
        if (e != hipSuccess) return e;
    }
    if (n_items > d0) {
        const int grid = std::max(1, std::min(n_items - d0, device_cu_count() * 2));
        hipLaunchKernelGGL(k_batch<kKindDirect>, dim3(grid), dim3(kDirectWaves * 64), 0, st, insts, items, d0,
                           n_items, counter + 2, part);
    }
    hipLaunchKernelGGL(k_batch_reduce_ranges, dim3(P.n_inst), dim3(256), 0, st, (const double*)(P.base + P.off_part),
                       (const int32_t*)(P.base + P.off_range), (const BatchInst*)(P.base + P.off_insts), out);
    return hipGetLastError();
}

}  // namespace mdgmi

// ---------------------------------------------------------------- C ABI
struct mdgmi_batch {
    mdgmi::BatchPlan P;
    char* dmem = nullptr;
    int device = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double* graph_out = nullptr;
    int64_t pairs = 0;
};

namespace {

int check_instances(const mdgmi_instance* inst, int n_inst) {
    if (!inst) return MDGMI_E_NULL;
    if (n_inst < 1) return MDGMI_E_SHAPE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return MDGMI_E_HIP;
    for (int q = 0; q < n_inst; q++) {
        const mdgmi_instance& I = inst[q];
        if (!I.fmt || !I.y || !I.tx_idx) return MDGMI_E_NULL;
        if (I.n < 1) return MDGMI_E_SHAPE;
        if (!(std::isfinite(I.sigma2) && I.sigma2 > 0.0)) return MDGMI_E_SIGMA2;
        if (I.fmt->device != dev) return MDGMI_E_DEVICE;
    }
    return MDGMI_OK;
}

int check_batch_path(int path) {
    return (path == MDGMI_PATH_F32_DIRECT || path == MDGMI_PATH_F32_MFMA_F16SPLIT || path == MDGMI_PATH_AUTO)
               ? MDGMI_OK
               : (path == MDGMI_PATH_F64 || path == MDGMI_PATH_F32_MFMA_BF16SPLIT ? MDGMI_E_UNSUPPORTED
                                                                                  : MDGMI_E_ARG);
}

}  // namespace

using namespace mdgmi;

extern "C" {

int mdgmi_gmi_batched_workspace_size(const mdgmi_instance* inst, int32_t n_inst, int32_t path, size_t* bytes) {
    if (!bytes) return MDGMI_E_NULL;
    int rc = check_instances(inst, n_inst);
    if (rc != MDGMI_OK) return rc;
    if ((rc = check_batch_path(path)) != MDGMI_OK) return rc;
    BatchPlan P;
    rc = plan_batch(inst, n_inst, path, tuned_item_pairs(), P);
    if (rc != MDGMI_OK) return rc;
    *bytes = P.bytes;
    return MDGMI_OK;
}

int mdgmi_gmi_batched(const mdgmi_instance* inst, int32_t n_inst, int32_t path, double* out, void* ws,
                      size_t ws_bytes, void* stream) {
    if (!out) return MDGMI_E_NULL;
    int rc = check_instances(inst, n_inst);
    if (rc != MDGMI_OK) return rc;
    if ((rc = check_batch_path(path)) != MDGMI_OK) return rc;
    BatchPlan P;
    rc = plan_batch(inst, n_inst, path, tuned_item_pairs(), P);
    if (rc != MDGMI_OK) return rc;
    if (!ws || ws_bytes < P.bytes) return MDGMI_E_WORKSPACE;
    if (prepare_batch_kernel() != hipSuccess) return MDGMI_E_HIP;
    bind_batch(P, (char*)ws);
    hipStream_t st = (hipStream_t)stream;
    if (upload_batch(P, st) != hipSuccess) return MDGMI_E_HIP;
    return launch_batch(P, out, st) == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

int mdgmi_batch_create(const mdgmi_instance* inst, int32_t n_inst, int32_t path, mdgmi_batch** out) {
    if (!out) return MDGMI_E_NULL;
    *out = nullptr;
    int rc = check_instances(inst, n_inst);
    if (rc != MDGMI_OK) return rc;
    if ((rc = check_batch_path(path)) != MDGMI_OK) return rc;
    if (path == MDGMI_PATH_AUTO) {
        for (int q = 0; q < n_inst; q++) {
            const mdgmi_format* f = inst[q].fmt;
            if (tuned_batch_kind(f->dim, f->M) < 0 && (rc = mdgmi_autotune(f->dim, f->M, 0, nullptr)) != MDGMI_OK)
                return rc;
        }
    }
    mdgmi_batch* b = new mdgmi_batch();
    rc = plan_batch(inst, n_inst, path, tuned_item_pairs(), b->P);
    if (rc != MDGMI_OK) {
        delete b;
        return rc;
    }
    for (int q = 0; q < n_inst; q++) b->pairs += inst[q].n * inst[q].fmt->M;
    (void)hipGetDevice(&b->device);
    bool ok = prepare_batch_kernel() == hipSuccess && hipMalloc(&b->dmem, b->P.bytes) == hipSuccess &&
              hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) == hipSuccess;
    if (ok) {
        bind_batch(b->P, b->dmem);
        ok = upload_batch(b->P, b->cap) == hipSuccess && hipStreamSynchronize(b->cap) == hipSuccess;
    }
    if (!ok) {
        mdgmi_batch_destroy(b);
        return MDGMI_E_HIP;
    }
    *out = b;
    return MDGMI_OK;
}

int mdgmi_batch_run(mdgmi_batch* b, double* out, int32_t use_graph, void* stream) {
    if (!b || !out) return MDGMI_E_NULL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return MDGMI_E_HIP;
    if (dev != b->device) return MDGMI_E_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    if (!use_graph) return launch_batch(b->P, out, st) == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
    if (!b->exec || b->graph_out != out) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return MDGMI_E_HIP;
        const hipError_t le = launch_batch(b->P, out, b->cap);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(b->cap, &g);
        if (le != hipSuccess || ce != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return MDGMI_E_HIP;
        }
        b->graph = g;
        if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return MDGMI_E_HIP;
        b->graph_out = out;
    }
    return hipGraphLaunch(b->exec, st) == hipSuccess ? MDGMI_OK : MDGMI_E_HIP;
}

int mdgmi_batch_info(const mdgmi_batch* b, int64_t* n_items, int64_t* pairs) {
    if (!b) return MDGMI_E_NULL;
    if (n_items) *n_items = (int64_t)b->P.items.size();
    if (pairs) *pairs = b->pairs;
    return MDGMI_OK;
}

int mdgmi_batch_destroy(mdgmi_batch* b) {
    if (!b) return MDGMI_E_NULL;
    if (b->cap) (void)hipStreamSynchronize(b->cap);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->dmem) (void)hipFree(b->dmem);
    delete b;
    return MDGMI_OK;
}

}  // extern "C"
