// Host-side checks and preparation of a point format (see format_host.h).
#include "format_host.h"

#include <algorithm>
#include <cmath>

#include "../../include/mdgmi.h"

extern "C" int mdgmi_validate_labels(const uint32_t* labels_host, int32_t M) {
    if (!labels_host) return MDGMI_E_NULL;
    if (M < 1 || M > (1 << MDGMI_MAX_BITS)) return MDGMI_E_SHAPE;
    std::vector<uint8_t> seen((size_t)M, 0);
    for (int32_t j = 0; j < M; j++) {
        const uint32_t l = labels_host[j];
        if (l >= (uint32_t)M || seen[l]) return MDGMI_E_LABELS;
        seen[l] = 1;
    }
    return MDGMI_OK;
}

namespace mdgmi {

int prepare_format(const double* X_host, const uint32_t* labels_host, int32_t M, int32_t dim, FormatHost& f) {
    if (!X_host || !labels_host) return MDGMI_E_NULL;
    if (dim != 1 && dim != 2 && dim != 4 && dim != 8) return MDGMI_E_SHAPE;
    if (M < 2 || M > (1 << MDGMI_MAX_BITS) || (M & (M - 1)) != 0) return MDGMI_E_SHAPE;
    const int rc = mdgmi_validate_labels(labels_host, M);
    if (rc != MDGMI_OK) return rc;
    for (size_t i = 0; i < (size_t)M * dim; i++)
        if (!std::isfinite(X_host[i])) return MDGMI_E_ARG;
    f.M = M;
    f.dim = dim;
    f.m = 0;
    while ((1 << f.m) < M) f.m++;
    f.X64.assign((size_t)M * dim, 0.0);
    f.X32.assign((size_t)M * dim, 0.0f);
    f.n32.assign((size_t)M, 0.0f);
    f.energy = f.max_abs = f.max_norm2 = 0.0;
    for (int32_t r = 0; r < M; r++) {
        const uint32_t slot = labels_host[r];
        double n2 = 0.0;
        for (int d = 0; d < dim; d++) {
            const double x = X_host[(size_t)r * dim + d];
            f.X64[(size_t)slot * dim + d] = x;
            f.X32[(size_t)slot * dim + d] = (float)x;
            n2 += x * x;
            f.max_abs = std::max(f.max_abs, std::fabs(x));
        }
        f.n32[slot] = (float)n2;
        f.max_norm2 = std::max(f.max_norm2, n2);
        f.energy += n2 / M;
    }
    // Rows sharing their coordinates with a lower label: sort rows by
    // (coordinates, label); within a run of equal points all but the first
    // carry kTwinBit.
    f.labels_hd.assign(labels_host, labels_host + M);
    std::vector<uint32_t> order((size_t)M);
    for (int32_t r = 0; r < M; r++) order[r] = (uint32_t)r;
    auto pt = [&](uint32_t r, int d) { return X_host[(size_t)r * dim + d]; };
    auto same = [&](uint32_t a, uint32_t b) {
        for (int d = 0; d < dim; d++)
            if (!(pt(a, d) == pt(b, d))) return false;
        return true;
    };
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        for (int d = 0; d < dim; d++)
            if (pt(a, d) != pt(b, d)) return pt(a, d) < pt(b, d);
        return labels_host[a] < labels_host[b];
    });
    for (int32_t k = 1; k < M; k++)
        if (same(order[k - 1], order[k])) f.labels_hd[order[k]] |= kTwinBit;
    return MDGMI_OK;
}

}  // namespace mdgmi
