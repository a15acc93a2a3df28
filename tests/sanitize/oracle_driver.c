/* Host sanitizer driver for the FP64 oracle: every entry point on small
 * formats of each dimension, with edge inputs (far samples, tiny and large
 * sigma2, non-finite samples, rows out of range, n = 0), built with
 * -fsanitize=address,undefined. Exit status 0 when every call returned what
 * its contract says. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_llr(const double*, int64_t, int, const double*, const uint32_t*, int, double, double*);
int oracle_costs(const double*, const uint32_t*, int64_t, int, const double*, const uint32_t*, int, double, double*,
                 double*);
int oracle_gmi(const double*, const uint32_t*, int64_t, int, const double*, const uint32_t*, int, double, double*);
int oracle_llr_maxlog(const double*, int64_t, int, const double*, const uint32_t*, int, double, double*);
int oracle_hd(const double*, const uint32_t*, int64_t, int, const double*, const uint32_t*, int, double, double*);
double oracle_gelu(double);
int64_t oracle_mlp_param_count(const int*, int);
int oracle_mlp_forward(const double*, const int*, int, const double*, int64_t, double*);
double oracle_mlp_loss_grad(const double*, const int*, int, const double*, const double*, int64_t, double*);
void oracle_adam(double*, const double*, double*, double*, int64_t, int64_t, double, double, double, double);
int oracle_gmi_cost_from_llr(const double*, const uint32_t*, int64_t, int, double*);

static uint64_t st = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* xorshift64*, uniform in [0, 1) */
    st ^= st >> 12;
    st ^= st << 25;
    st ^= st >> 27;
    return (double)((st * 0x2545F4914F6CDD1Dull) >> 11) * 0x1p-53;
}
static double nrand(void) { return sqrt(-2.0 * log(1.0 - urand())) * cos(6.283185307179586 * urand()); }

static int fails = 0;
#define CHECK(c, ...)                  \
    do {                               \
        if (!(c)) {                    \
            fprintf(stderr, __VA_ARGS__); \
            fprintf(stderr, "\n");     \
            fails++;                   \
        }                              \
    } while (0)

static void run_format(int dim, int M, double sigma2) {
    const int64_t n = 37;
    int m = 0;
    while ((1 << m) < M) m++;
    double* X = malloc(sizeof(double) * (size_t)M * dim);
    uint32_t* lab = malloc(sizeof(uint32_t) * (size_t)M);
    double* y = malloc(sizeof(double) * (size_t)n * dim);
    uint32_t* tx = malloc(sizeof(uint32_t) * (size_t)n);
    double* llr = malloc(sizeof(double) * (size_t)n * m);
    double* cg = malloc(sizeof(double) * (size_t)n);
    double* cm = malloc(sizeof(double) * (size_t)n);
    double out[6], hd[4];
    for (int j = 0; j < M; j++) {
        lab[j] = (uint32_t)j;
        for (int d = 0; d < dim; d++) X[j * dim + d] = nrand();
    }
    for (int j = M - 1; j > 0; j--) { /* labels: a random permutation */
        int k = (int)(urand() * (j + 1));
        uint32_t t = lab[j];
        lab[j] = lab[k];
        lab[k] = t;
    }
    for (int64_t s = 0; s < n; s++) {
        tx[s] = (uint32_t)(urand() * M);
        for (int d = 0; d < dim; d++) y[s * dim + d] = X[tx[s] * dim + d] + sqrt(sigma2) * nrand();
    }
    for (int d = 0; d < dim; d++) y[3 * dim + d] = 1.0e5; /* far from every point */
    y[4 * dim] = -3.0e3;
    CHECK(oracle_llr(y, n, dim, X, lab, M, sigma2, llr) == 0, "llr dim %d M %d", dim, M);
    for (int64_t i = 0; i < n * m; i++) CHECK(isfinite(llr[i]), "llr finite dim %d M %d", dim, M);
    CHECK(oracle_costs(y, tx, n, dim, X, lab, M, sigma2, cg, cm) == 0, "costs");
    CHECK(oracle_costs(y, tx, n, dim, X, lab, M, sigma2, NULL, cm) == 0, "costs, no GMI");
    CHECK(oracle_gmi(y, tx, n, dim, X, lab, M, sigma2, out) == 0 && out[4] == (double)n && out[5] == 0.0,
          "gmi dim %d M %d", dim, M);
    CHECK(oracle_llr_maxlog(y, n, dim, X, lab, M, sigma2, llr) == 0, "maxlog");
    CHECK(oracle_hd(y, tx, n, dim, X, lab, M, sigma2, hd) == 0 && hd[2] == (double)n, "hd");
    CHECK(oracle_gmi_cost_from_llr(llr, lab, n < M ? n : M, m, cg) == 0, "cost from llr");
    /* non-finite samples are counted, not dropped */
    y[5 * dim] = NAN;
    y[6 * dim] = INFINITY;
    CHECK(oracle_gmi(y, tx, n, dim, X, lab, M, sigma2, out) == 0 && out[5] == 2.0, "gmi nonfinite %g", out[5]);
    CHECK(oracle_hd(y, tx, n, dim, X, lab, M, sigma2, hd) == 0 && hd[3] == 2.0, "hd nonfinite");
    CHECK(oracle_llr(y, n, dim, X, lab, M, sigma2, llr) == 0, "llr nonfinite");
    /* a sent row out of range and an empty batch are refused */
    tx[7] = (uint32_t)M;
    CHECK(oracle_gmi(y, tx, n, dim, X, lab, M, sigma2, out) == -3, "gmi row out of range");
    CHECK(oracle_costs(y, tx, n, dim, X, lab, M, sigma2, cg, cm) == -3, "costs row out of range");
    CHECK(oracle_hd(y, tx, n, dim, X, lab, M, sigma2, hd) == -3, "hd row out of range");
    CHECK(oracle_gmi(y, tx, 0, dim, X, lab, M, sigma2, out) == -2, "gmi n = 0");
    free(X), free(lab), free(y), free(tx), free(llr), free(cg), free(cm);
}

static void run_mlp(void) {
    const int sizes[4] = {9, 16, 24, 11};
    const int L = 3;
    const int64_t n = 5, P = oracle_mlp_param_count(sizes, L);
    double* p = malloc(sizeof(double) * (size_t)P);
    double* g = malloc(sizeof(double) * (size_t)P);
    double* mm = calloc((size_t)P, sizeof(double));
    double* vv = calloc((size_t)P, sizeof(double));
    double x[5 * 9], tgt[5 * 11], logits[5 * 11];
    for (int64_t i = 0; i < P; i++) p[i] = 0.3 * nrand();
    for (int i = 0; i < 5 * 9; i++) x[i] = nrand();
    for (int i = 0; i < 5 * 11; i++) tgt[i] = urand();
    CHECK(oracle_mlp_forward(p, sizes, L, x, n, logits) == 0, "mlp forward");
    const double loss = oracle_mlp_loss_grad(p, sizes, L, x, tgt, n, g);
    CHECK(isfinite(loss) && loss > 0.0, "mlp loss");
    for (int t = 1; t <= 3; t++) oracle_adam(p, g, mm, vv, P, t, 1e-3, 0.9, 0.999, 1e-8);
    CHECK(isfinite(p[0]) && isfinite(p[P - 1]), "adam");
    CHECK(oracle_gelu(-40.0) == -0.0 || fabs(oracle_gelu(-40.0)) < 1e-300, "gelu tail");
    free(p), free(g), free(mm), free(vv);
}

int main(void) {
    const int dims[4] = {1, 2, 4, 8}, Ms[4] = {2, 16, 64, 256};
    const double s2[3] = {1e-6, 0.05, 1e3};
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++)
            for (int c = 0; c < 3; c++) run_format(dims[a], Ms[b], s2[c]);
    run_mlp();
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle driver ok\n");
    return 0;
}
