// The fused inference layout's index map (csrc/mlp_layout.h): for every
// layer of the fused shapes, fused_offset must invert the map the layout
// builder walks (tile, K-block, lane, slot) -> (row, input), and land every
// weight in a distinct slot inside the layer's buffer.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "mlp_layout.h"

using mdgmi::fused::fused_offset;
using mdgmi::fused::perm_in;

static int check(int l, int out, int in) {
    const int n_tiles = (out + 31) / 32, n_kb = (in + 15) / 16;
    std::vector<long> owner((size_t)n_tiles * n_kb * 512, -1);
    for (int t = 0; t < n_tiles; t++)
        for (int kb = 0; kb < n_kb; kb++)
            for (int lane = 0; lane < 64; lane++)
                for (int i = 0; i < 8; i++) {
                    const int row = 32 * t + (lane & 31), h = lane >> 5;
                    const int k = 16 * kb + (l > 0 ? perm_in(h, i) : 8 * h + i);
                    if (row < out && k < in) owner[((size_t)(t * n_kb + kb) * 64 + lane) * 8 + i] = (long)row * in + k;
                }
    int bad = 0;
    for (int o = 0; o < out; o++)
        for (int k = 0; k < in; k++) {
            const long off = (long)fused_offset(l, o, k, in);
            if (off < 0 || off >= (long)owner.size() || owner[off] != (long)o * in + k) bad++;
        }
    return bad;
}

int main() {
    const int ins[] = {1, 9, 16}, outs[] = {1, 11, 32};
    int bad = 0;
    for (int in : ins) bad += check(0, 256, in);
    for (int l = 1; l <= 2; l++) bad += check(l, 256, 256);
    for (int out : outs) bad += check(3, out, 256);
    if (bad) {
        std::printf("layout driver: %d weights misplaced\n", bad);
        return 1;
    }
    std::printf("layout driver ok\n");
    return 0;
}
