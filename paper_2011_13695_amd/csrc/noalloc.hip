// mdgmi_gmi_static: mdgmi_gmi with its scratch memory (per-block FP64
// partials and the per-SNR operand images) in a static device array instead
// of a caller workspace, for callers that cannot allocate.
#include <mutex>

#include "internal.h"

namespace {

// One copy per device that the library runs on, held until the process
// ends. Host code never uses this name as an address: the device address
// comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[MDGMI_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

// Device address of `scratch` on the current device (nullptr on failure).
void* scratch_ptr(int* status) {
    static std::mutex mu;
    static void* ptr[kMaxDevices] = {nullptr};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *status = MDGMI_E_HIP;
        return nullptr;
    }
    std::lock_guard<std::mutex> g(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            *status = MDGMI_E_HIP;
            return nullptr;
        }
        ptr[dev] = p;
    }
    *status = MDGMI_OK;
    return ptr[dev];
}

}  // namespace

extern "C" int mdgmi_gmi_static(const mdgmi_format* fmt, const void* y, const uint32_t* tx_idx, int64_t n,
                                const double* sigma2_host, int32_t n_snr, int32_t path, double* out, void* stream) {
    if (!fmt || !y || !tx_idx || !sigma2_host || !out) return MDGMI_E_NULL;
    if (n < 1 || n_snr < 1) return MDGMI_E_SHAPE;
    // the plan's exact need for the resolved path is checked against the
    // array size by the shared entry (MDGMI_E_WORKSPACE beyond it)
    int rc = MDGMI_OK;
    void* ws = scratch_ptr(&rc);
    if (rc != MDGMI_OK) return rc;
    return mdgmi::gmi_with_workspace(fmt, y, tx_idx, n, sigma2_host, n_snr, path, out, ws,
                                     (size_t)MDGMI_STATIC_SCRATCH_BYTES, stream);
}
