// 32 x 32 MFMA demapper kernels for 8-D formats, fp16 hi + lo split.
#define MDGMI_MFMA_KERNELS
#include "mfma_kernels.h"

namespace mdgmi {
template hipError_t mfma_run<8, kSplitF16>(const mdgmi_format*, const float*, const uint32_t*, int64_t, const SnrArgs&,
                                        int, float*, double*, uint4*, int, LaunchCfg, MfmaShape, hipStream_t);
}  // namespace mdgmi
