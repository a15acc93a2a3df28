// Ragged persistent batch: host plan and device descriptors.
#pragma once

#include <vector>

#include "internal.h"

namespace mdgmi {

constexpr int kKindDirect = 0;
constexpr int kKindMfma = 1;
constexpr int kKindSmall = 2;   // per-sample 4x4-block MFMA shape (small_core.h)

// One (format, SNR) instance as the persistent kernel sees it.
struct BatchInst {
    const float* y;
    const uint32_t* tx;
    const void* img;          // MFMA A image (uint4), 4x4-shape image (uint2) or direct records (float)
    const float* X32;
    const uint32_t* labels;
    int64_t n;
    float s;                  // log2(e) / (2 sigma2)
    int dim, M, m, ntiles;
    int kind;                 // kKindDirect / kKindMfma / kKindSmall
    int dvar;                 // direct code variant (chunk bits, group size)
    int img_u4;               // MFMA image size in 16-byte units
};

// A contiguous sample range of one instance.
struct BatchItem {
    int32_t inst;
    int32_t pad;
    int64_t s0, s1;
};

// What the image builder needs per instance.
struct BatchImg {
    const double* X64;
    double s64;
    int dim, M, kind, ntiles;
    int64_t slot_off;         // first global slot of this instance
    size_t img_off;           // byte offset of its image in the image region
};

struct BatchPlan {
    int n_inst = 0;
    std::vector<BatchInst> insts;
    std::vector<BatchImg> imgs;
    std::vector<BatchItem> items;
    std::vector<int32_t> item_range;   // (first, end) item per instance
    int64_t total_slots = 0;
    int max_lds_u4 = 0;
    int n_mfma_items = 0;             // items [0, n_mfma_items) are MFMA items,
    int n_small_items = 0;            // the next n_small_items 4x4-shape items, the rest direct
    size_t off_insts = 0, off_imgs = 0, off_items = 0, off_range = 0, off_part = 0, off_counter = 0,
           off_images = 0, bytes = 0;
    char* base = nullptr;
};

constexpr int64_t kItemPairsDefault = int64_t(1) << 22;
constexpr int kSmallItemAlign = 256;  // 4x4-shape items start at multiples of 64 samples x 4 waves

// Persistent grid of the 4x4-shape kind over items [i0, i1) (batch_small.hip).
hipError_t launch_batch_small(const BatchInst* insts, const BatchItem* items, int i0, int i1, unsigned* counter,
                              double* part, hipStream_t st);

int batch_kind_for(const mdgmi_format* f, double s, int path);
int plan_batch(const mdgmi_instance* inst, int n_inst, int path, int64_t item_pairs, BatchPlan& P);
void bind_batch(BatchPlan& P, char* base);
hipError_t upload_batch(const BatchPlan& P, hipStream_t st);
hipError_t prepare_batch_kernel();
hipError_t launch_batch(const BatchPlan& P, double* out, hipStream_t st);

// autotuner table (autotune.hip)
int tuned_batch_kind(int dim, int M);      // kKind* or -1 when untuned
int64_t tuned_item_pairs();

}  // namespace mdgmi
