// Autotuner: per (dim, M) and per sample-count regime it times the FP32
// direct kernel and every MFMA launch variant on synthetic samples of that
// shape on the current device, and records the fastest. The bulk regime
// (launches of at least kTuneShortSamples samples over their SNR points) is
// timed on at least 2^20 samples, two resident rounds of the widest launch
// shape and more; the short regime on 2^15 samples, a fraction of one round.
// The table steers MDGMI_PATH_AUTO calls, the MFMA launch shape of
// fp16-split calls and the per-instance kind of ragged batches (bulk); it
// can be saved to and loaded from a small JSON file ({"arch": ...,
// "entries": [{"dim", "M", "regime", "samples", "path", "variant",
// "direct_rate", "mfma_rate"}, ...]}).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "batch.h"
#include "internal.h"

namespace mdgmi {

namespace {

std::mutex g_mu;
std::map<std::tuple<int, int, int>, mdgmi_tune_entry> g_table;  // (dim, M, regime)

// Entry of (dim, M) for a launch of `total` samples: its regime's, else
// the other regime's; nullptr when (dim, M) is untuned. Caller holds g_mu.
const mdgmi_tune_entry* find_entry(int dim, int M, int64_t total) {
    const int r = tune_regime(total);
    auto it = g_table.find({dim, M, r});
    if (it == g_table.end()) it = g_table.find({dim, M, 1 - r});
    return it == g_table.end() ? nullptr : &it->second;
}

// Synthetic format for timing only: two shells (radius 1 and 1.6) in `dim`
// dimensions with Box-Muller directions from a fixed xorshift stream, unit
// average energy, label = index.
void synth_format(int dim, int M, std::vector<double>& X, std::vector<uint32_t>& lab) {
    X.assign((size_t)M * dim, 0.0);
    lab.resize(M);
    uint64_t st = 0x9E3779B97F4A7C15ull ^ ((uint64_t)dim << 32) ^ (uint64_t)M;
    auto next = [&]() {
        st ^= st << 13;
        st ^= st >> 7;
        st ^= st << 17;
        return ((st >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    };
    double e = 0.0;
    for (int j = 0; j < M; j++) {
        double nrm = 0.0;
        for (int d = 0; d < dim; d += 2) {
            const double r = std::sqrt(-2.0 * std::log(next())), a = 6.283185307179586 * next();
            X[(size_t)j * dim + d] = r * std::cos(a);
            if (d + 1 < dim) X[(size_t)j * dim + d + 1] = r * std::sin(a);
        }
        for (int d = 0; d < dim; d++) nrm += X[(size_t)j * dim + d] * X[(size_t)j * dim + d];
        const double rad = j < M / 2 ? 1.0 : 1.6;
        for (int d = 0; d < dim; d++) X[(size_t)j * dim + d] *= rad / std::sqrt(nrm);
        e += rad * rad;
        lab[j] = (uint32_t)j;
    }
    const double sc = 1.0 / std::sqrt(e / M);
    for (double& v : X) v *= sc;
}

}  // namespace

int tuned_batch_kind(int dim, int M) {
    std::lock_guard<std::mutex> g(g_mu);
    const mdgmi_tune_entry* e = find_entry(dim, M, INT64_MAX);  // a batch is one bulk launch per kind
    if (!e) return -1;
    return e->path == MDGMI_PATH_F32_MFMA_F16SPLIT ? kKindMfma : kKindDirect;
}

int tuned_path(int dim, int M, int64_t total) {
    std::lock_guard<std::mutex> g(g_mu);
    const mdgmi_tune_entry* e = find_entry(dim, M, total);
    return e ? e->path : -1;
}

int tuned_mfma_variant(int dim, int M, int64_t total) {
    std::lock_guard<std::mutex> g(g_mu);
    const mdgmi_tune_entry* e = find_entry(dim, M, total);
    return e ? e->mfma_variant : -1;
}

int64_t tuned_item_pairs() { return kItemPairsDefault; }

}  // namespace mdgmi

using namespace mdgmi;

extern "C" {

int mdgmi_tune_lookup(int32_t dim, int32_t M, int32_t regime, mdgmi_tune_entry* out) {
    if (!out) return MDGMI_E_NULL;
    if (regime != MDGMI_TUNE_BULK && regime != MDGMI_TUNE_SHORT) return MDGMI_E_ARG;
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_table.find({dim, M, regime});
    if (it == g_table.end()) return MDGMI_E_ARG;
    *out = it->second;
    return MDGMI_OK;
}

int mdgmi_tune_clear(void) {
    std::lock_guard<std::mutex> g(g_mu);
    g_table.clear();
    return MDGMI_OK;
}

int mdgmi_autotune(int32_t dim, int32_t M, int32_t force, mdgmi_tune_entry* out) {
    if (dim != 1 && dim != 2 && dim != 4 && dim != 8) return MDGMI_E_SHAPE;
    if (M < 2 || M > (1 << MDGMI_MAX_BITS) || (M & (M - 1))) return MDGMI_E_SHAPE;
    if (!force) {
        std::lock_guard<std::mutex> g(g_mu);
        auto bulk = g_table.find({dim, M, MDGMI_TUNE_BULK}), shrt = g_table.find({dim, M, MDGMI_TUNE_SHORT});
        if (bulk != g_table.end() && shrt != g_table.end()) {
            if (out) {
                out[0] = bulk->second;
                out[1] = shrt->second;
            }
            return MDGMI_OK;
        }
    }
    std::vector<double> X;
    std::vector<uint32_t> lab;
    synth_format(dim, M, X, lab);
    mdgmi_format* f = nullptr;
    int rc = mdgmi_format_create(X.data(), lab.data(), M, dim, &f);
    if (rc != MDGMI_OK) return rc;
    // bulk: about 2^28 sample*points per timed call and at least 2^20
    // samples (two resident rounds of every launch shape: the widest, the
    // per-sample 4x4 shape, holds about 3.3e5 samples per round on 256 CUs),
    // at most 2^22; short: 2^15 samples
    int64_t n_regime[2];
    n_regime[MDGMI_TUNE_BULK] = std::min<int64_t>(
        int64_t(1) << 22, std::max<int64_t>(int64_t(1) << 20, (int64_t(1) << 28) / M));
    n_regime[MDGMI_TUNE_SHORT] = int64_t(1) << 15;
    const int64_t n = n_regime[MDGMI_TUNE_BULK];
    const double sigma2 = 1.0 / (dim * 10.0);  // 10 dB
    float* y = nullptr;
    uint32_t* tx = nullptr;
    double* o = nullptr;
    void* ws = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    mdgmi_tune_entry best[2]{};
    size_t wsb = 0, t;
    rc = MDGMI_E_HIP;
    const int saved_override = mdgmi_get_tuning();
    do {
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) break;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) break;
        if (hipMalloc(&y, sizeof(float) * n * dim) != hipSuccess) break;
        if (hipMalloc(&tx, sizeof(uint32_t) * n) != hipSuccess) break;
        if (hipMalloc(&o, sizeof(double) * MDGMI_NFIELDS) != hipSuccess) break;
        if (mdgmi_generate(f, 12345, &sigma2, 1, n, 0, y, tx, 0, st) != MDGMI_OK) break;
        // workspace for the largest candidate (the short calls need less)
        if (mdgmi_gmi_workspace_size(f, n, 1, MDGMI_PATH_F32_DIRECT, &wsb) != MDGMI_OK) break;
        for (int v = 0; v < kMfmaVariants; v++) {
            mdgmi_set_tuning(v);
            if (mdgmi_gmi_workspace_size(f, n, 1, MDGMI_PATH_F32_MFMA_F16SPLIT, &t) == MDGMI_OK) wsb = std::max(wsb, t);
        }
        mdgmi_set_tuning(saved_override);
        if (hipMalloc(&ws, wsb) != hipSuccess) break;
        bool ok = true;
        for (int r = 0; r < 2 && ok; r++) {
            const int64_t nr = n_regime[r];
            // best of 3 timed calls after one untimed call; rate in sample*points/s
            auto time_call = [&](int path) -> double {
                if (mdgmi_gmi(f, y, tx, nr, &sigma2, 1, path, o, ws, wsb, st) != MDGMI_OK) return -1.0;
                float best_ms = 1e30f;
                for (int k = 0; k < 3; k++) {
                    (void)hipEventRecord(e0, st);
                    if (mdgmi_gmi(f, y, tx, nr, &sigma2, 1, path, o, ws, wsb, st) != MDGMI_OK) return -1.0;
                    (void)hipEventRecord(e1, st);
                    if (hipEventSynchronize(e1) != hipSuccess) return -1.0;
                    float ms = 0.0f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    best_ms = std::min(best_ms, ms);
                }
                return (double)nr * M / (best_ms * 1e-3);
            };
            mdgmi_tune_entry& b = best[r];
            b.dim = dim;
            b.M = M;
            b.regime = r;
            b.samples = nr;
            b.path = MDGMI_PATH_F32_DIRECT;
            b.mfma_variant = -1;
            b.direct_rate = time_call(MDGMI_PATH_F32_DIRECT);
            ok = b.direct_rate > 0.0;
            b.mfma_rate = 0.0;
            if (ok && (M >= 32 || small_shape_fits(f)) && mfma_supported(f, kLog2e / (2.0 * sigma2))) {
                for (int v = 0; v < kMfmaVariants; v++) {
                    mdgmi_set_tuning(v);
                    const double rate = time_call(MDGMI_PATH_F32_MFMA_F16SPLIT);
                    if (rate > b.mfma_rate) {
                        b.mfma_rate = rate;
                        b.mfma_variant = v;
                    }
                }
                mdgmi_set_tuning(saved_override);
                if (b.mfma_rate > b.direct_rate) b.path = MDGMI_PATH_F32_MFMA_F16SPLIT;
            }
        }
        if (ok) rc = MDGMI_OK;
    } while (0);
    mdgmi_set_tuning(saved_override);
    if (st) (void)hipStreamSynchronize(st);
    if (ws) (void)hipFree(ws);
    if (o) (void)hipFree(o);
    if (tx) (void)hipFree(tx);
    if (y) (void)hipFree(y);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    mdgmi_format_destroy(f);
    if (rc != MDGMI_OK) return rc;
    {
        std::lock_guard<std::mutex> g(g_mu);
        for (int r = 0; r < 2; r++) g_table[{dim, M, r}] = best[r];
    }
    if (out) {
        out[0] = best[0];
        out[1] = best[1];
    }
    return MDGMI_OK;
}

int mdgmi_tune_save(const char* path) {
    if (!path) return MDGMI_E_NULL;
    FILE* fp = std::fopen(path, "w");
    if (!fp) return MDGMI_E_ARG;
    std::lock_guard<std::mutex> g(g_mu);
    std::fprintf(fp, "{\"arch\": \"gfx950\", \"entries\": [\n");
    size_t k = 0;
    for (const auto& kv : g_table) {
        const mdgmi_tune_entry& e = kv.second;
        std::fprintf(fp,
                     "  {\"dim\": %d, \"M\": %d, \"regime\": %d, \"samples\": %lld, \"path\": %d, "
                     "\"variant\": %d, \"direct_rate\": %.6e, \"mfma_rate\": %.6e}%s\n",
                     e.dim, e.M, e.regime, (long long)e.samples, e.path, e.mfma_variant, e.direct_rate, e.mfma_rate,
                     ++k < g_table.size() ? "," : "");
    }
    std::fprintf(fp, "]}\n");
    std::fclose(fp);
    return MDGMI_OK;
}

int mdgmi_tune_load(const char* path) {
    if (!path) return MDGMI_E_NULL;
    FILE* fp = std::fopen(path, "r");
    if (!fp) return MDGMI_E_ARG;
    std::string text;
    char buf[4096];
    size_t r;
    while ((r = std::fread(buf, 1, sizeof(buf), fp)) > 0) text.append(buf, r);
    std::fclose(fp);
    if (text.find("\"gfx950\"") == std::string::npos) return MDGMI_E_ARG;
    int loaded = 0;
    size_t pos = 0;
    while ((pos = text.find("{\"dim\"", pos)) != std::string::npos) {
        mdgmi_tune_entry e{};
        long long samples = 0;
        if (std::sscanf(text.c_str() + pos,
                        "{\"dim\": %d, \"M\": %d, \"regime\": %d, \"samples\": %lld, \"path\": %d, "
                        "\"variant\": %d, \"direct_rate\": %lf, \"mfma_rate\": %lf}",
                        &e.dim, &e.M, &e.regime, &samples, &e.path, &e.mfma_variant, &e.direct_rate,
                        &e.mfma_rate) == 8) {
            e.samples = samples;
            const bool ok = (e.dim == 1 || e.dim == 2 || e.dim == 4 || e.dim == 8) && e.M >= 2 &&
                            e.M <= (1 << MDGMI_MAX_BITS) && (e.M & (e.M - 1)) == 0 &&
                            (e.regime == MDGMI_TUNE_BULK || e.regime == MDGMI_TUNE_SHORT) &&
                            (e.path == MDGMI_PATH_F32_DIRECT || e.path == MDGMI_PATH_F32_MFMA_F16SPLIT) &&
                            e.mfma_variant >= -1 && e.mfma_variant < kMfmaVariants;
            if (ok) {
                std::lock_guard<std::mutex> g(g_mu);
                g_table[{e.dim, e.M, e.regime}] = e;
                loaded++;
            }
        }
        pos += 6;
    }
    return loaded > 0 ? MDGMI_OK : MDGMI_E_ARG;
}

}  // extern "C"
