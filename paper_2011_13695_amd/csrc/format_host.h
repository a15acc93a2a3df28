// Host-side checks and preparation of a point format (no device calls, no
// HIP headers): the label bijection, the label-ordered copies the kernels
// read, norms and energy, and the twin flags of coincident points. Built into
// libmdgmi and, on its own, into the host sanitizer test.
#pragma once

#include <cstdint>
#include <vector>

namespace mdgmi {

// In the hard-decision label copy: the row's point has the same coordinates
// as a point with a lower label (labels themselves are < 2^12).
constexpr uint32_t kTwinBit = 1u << 16;
constexpr uint32_t kLabelMask = kTwinBit - 1u;

struct FormatHost {
    int32_t M = 0, dim = 0, m = 0;
    std::vector<double> X64;          // [M][dim], slot j = the point labelled j
    std::vector<float> X32;           // the same in FP32
    std::vector<float> n32;           // [M] ||x_j||^2 (FP32 of the FP64 sum)
    std::vector<uint32_t> labels_hd;  // [M] caller row -> label, kTwinBit on twins
    double energy = 0.0;              // mean_j ||x_j||^2
    double max_abs = 0.0;             // max_j,d |x_jd|
    double max_norm2 = 0.0;           // max_j ||x_j||^2
};

// Checks the arguments of mdgmi_format_create (returns its status codes:
// MDGMI_E_NULL, MDGMI_E_SHAPE for dim not in {1,2,4,8} or M not a power of
// two in [2, 4096], MDGMI_E_LABELS, MDGMI_E_ARG for a non-finite coordinate)
// and fills out; on an error out is left unspecified.
int prepare_format(const double* X_host, const uint32_t* labels_host, int32_t M, int32_t dim, FormatHost& out);

}  // namespace mdgmi

extern "C" int mdgmi_validate_labels(const uint32_t* labels_host, int32_t M);
