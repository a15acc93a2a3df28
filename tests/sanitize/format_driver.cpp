// Host sanitizer driver for the C-ABI's format checks and preparation
// (mdgmi_validate_labels, prepare_format): valid formats of every dimension
// up to M = 4096, coincident points (twin flags), and each rejected input,
// built with -fsanitize=address,undefined. Exit status 0 when every result
// matches the contract.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <limits>
#include <numeric>
#include <random>
#include <vector>

#include "format_host.h"
#include "mdgmi.h"

static int fails = 0;
#define CHECK(c, what)                                  \
    do {                                                \
        if (!(c)) {                                     \
            std::fprintf(stderr, "failed: %s\n", what); \
            fails++;                                    \
        }                                               \
    } while (0)

int main() {
    std::mt19937_64 rng(7);
    std::normal_distribution<double> nd;
    for (int dim : {1, 2, 4, 8}) {
        for (int M : {2, 4, 64, 4096}) {
            std::vector<double> X((size_t)M * dim);
            for (double& v : X) v = nd(rng);
            std::vector<uint32_t> lab((size_t)M);
            std::iota(lab.begin(), lab.end(), 0u);
            std::shuffle(lab.begin(), lab.end(), rng);
            mdgmi::FormatHost f;
            CHECK(mdgmi::prepare_format(X.data(), lab.data(), M, dim, f) == MDGMI_OK, "valid format");
            CHECK((1 << f.m) == M && f.X64.size() == (size_t)M * dim && f.labels_hd.size() == (size_t)M, "sizes");
            double e = 0.0;
            for (int r = 0; r < M; r++) {
                double n2 = 0.0;
                for (int d = 0; d < dim; d++) {
                    n2 += X[(size_t)r * dim + d] * X[(size_t)r * dim + d];
                    CHECK(f.X64[(size_t)lab[r] * dim + d] == X[(size_t)r * dim + d], "label order");
                }
                e += n2;
                CHECK(f.labels_hd[r] == lab[r], "no twins among random points");
            }
            CHECK(std::fabs(f.energy - e / M) <= 1e-12 * (e / M), "energy");
            // coincident points: rows 0, 1 and the last share coordinates;
            // all but the lowest label carry the twin flag
            if (M >= 4) {
                for (int d = 0; d < dim; d++) X[(size_t)1 * dim + d] = X[(size_t)(M - 1) * dim + d] = X[d];
                CHECK(mdgmi::prepare_format(X.data(), lab.data(), M, dim, f) == MDGMI_OK, "twins");
                const uint32_t lo = std::min({lab[0], lab[1], lab[M - 1]});
                for (int r : {0, 1, M - 1})
                    CHECK(((f.labels_hd[r] & mdgmi::kTwinBit) != 0) == (lab[r] != lo) &&
                              (f.labels_hd[r] & mdgmi::kLabelMask) == lab[r],
                          "twin flags");
            }
            // rejected inputs
            std::vector<uint32_t> bad = lab;
            bad[0] = bad[1];
            CHECK(mdgmi_validate_labels(bad.data(), M) == MDGMI_E_LABELS, "duplicate label");
            CHECK(mdgmi::prepare_format(X.data(), bad.data(), M, dim, f) == MDGMI_E_LABELS, "duplicate label");
            bad = lab;
            bad[M - 1] = (uint32_t)M;
            CHECK(mdgmi_validate_labels(bad.data(), M) == MDGMI_E_LABELS, "label out of range");
            std::vector<double> Xn = X;
            Xn[Xn.size() - 1] = std::numeric_limits<double>::quiet_NaN();
            CHECK(mdgmi::prepare_format(Xn.data(), lab.data(), M, dim, f) == MDGMI_E_ARG, "NaN coordinate");
            Xn[Xn.size() - 1] = std::numeric_limits<double>::infinity();
            CHECK(mdgmi::prepare_format(Xn.data(), lab.data(), M, dim, f) == MDGMI_E_ARG, "inf coordinate");
            CHECK(mdgmi::prepare_format(nullptr, lab.data(), M, dim, f) == MDGMI_E_NULL, "null X");
            CHECK(mdgmi::prepare_format(X.data(), nullptr, M, dim, f) == MDGMI_E_NULL, "null labels");
            CHECK(mdgmi::prepare_format(X.data(), lab.data(), M, 3, f) == MDGMI_E_SHAPE, "dim 3");
            if (M > 2) CHECK(mdgmi::prepare_format(X.data(), lab.data(), M - 1, dim, f) == MDGMI_E_SHAPE, "M odd");
        }
    }
    std::vector<uint32_t> big(8192);
    std::iota(big.begin(), big.end(), 0u);
    CHECK(mdgmi_validate_labels(big.data(), 8192) == MDGMI_E_SHAPE, "M above 4096");
    CHECK(mdgmi_validate_labels(big.data(), 0) == MDGMI_E_SHAPE, "M = 0");
    CHECK(mdgmi_validate_labels(nullptr, 4) == MDGMI_E_NULL, "null labels");
    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("format driver ok\n");
    return 0;
}
