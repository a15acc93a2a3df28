// Weight layout of the fused MLP inference kernel, shared by the kernel
// that builds it whole and the Adam step that updates it in place.
//
// Layer l's weights W [out][in] become [out tile][K-block][lane][8] bf16
// (32-row output tiles, 16-input K-blocks, 64 lanes of 8 values): lane
// holds row 32 t + (lane & 31) and, in lane half h = lane >> 5, eight of
// the block's sixteen inputs. Layer 0 takes inputs 8h .. 8h + 7 in order;
// later layers take {4h .. 4h + 3, 8 + 4h .. 8 + 4h + 3}, the order in
// which the previous layer's MFMA output lands in a lane's registers, so
// that activations go from accumulator to operand without a shuffle.
// Each layer is scaled by a power of two: 1/4 for layer 0 (the hidden
// accumulators hold x / 4), 4 for the output layer (it reads GELU / 4).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mdgmi {
namespace fused {

// input (within its 16-input block) of slot i of lane half h, layers >= 1
__host__ __device__ inline int perm_in(int h, int i) { return i < 4 ? 4 * h + i : 8 + 4 * h + (i - 4); }

__host__ __device__ inline float layer_scale(int l) { return l == 0 ? 0.25f : l == 3 ? 4.0f : 1.0f; }

// bf16 element offset of W[o][k] of layer l (in inputs) in the layout
__host__ __device__ inline int64_t fused_offset(int l, int o, int k, int in) {
    const int n_kb = (in + 15) / 16, kb = k / 16, r = k % 16;
    int h, slot;
    if (l == 0) {
        h = r / 8;
        slot = r % 8;
    } else if (r < 8) {  // perm_in(h, slot) = 4 h + slot
        h = r / 4;
        slot = r % 4;
    } else {             // perm_in(h, slot) = 8 + 4 h + slot - 4
        h = (r - 8) / 4;
        slot = 4 + (r - 8) % 4;
    }
    const int lane = 32 * h + o % 32;
    return (((int64_t)(o / 32) * n_kb + kb) * 64 + lane) * 8 + slot;
}

}  // namespace fused
}  // namespace mdgmi
