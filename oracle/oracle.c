/*
 * FP64 CPU oracle for Monte-Carlo GMI / MI estimation with exact per-bit LLRs.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product (the HIP library and its
 * Python binding) may include, link, load or call this file; only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * The paper defines the quantities only by name (glossary entries GMI, MI,
 * LLR, BICM, BMD, AWGN, SNR); the definitions written out here are the
 * standard information-theoretic ones for bit-interleaved coded modulation
 * with bit-metric decoding over the AWGN channel, uniform priors:
 *
 *   channel        y = x_i + z,  z ~ N(0, sigma2 I_N),  i uniform on [0, M)
 *   metric         t_j(y) = ||y - x_j||^2 / (2 sigma2)                 (nats)
 *   LLR of bit k   lambda_k(y) = ln sum_{j: b_k(j)=1} e^{-t_j}
 *                              - ln sum_{j: b_k(j)=0} e^{-t_j}
 *                  (b_k(j) = bit k of labels[j], LSB first; positive means 1)
 *   GMI cost       c_G(y, i) = sum_k log2(1 + exp(-(2 b_k(i) - 1) lambda_k))
 *   MI cost        c_M(y, i) = log2 sum_j exp(-(t_j - t_i))
 *   estimates      GMI = m - mean(c_G),  MI = m - mean(c_M)   (bits / symbol)
 *                  SE  = sqrt(sum (c - mean)^2 / (N (N - 1)))
 *
 * Every class sum is its own max-subtracted log-sum-exp over all M distances,
 * so nothing underflows however far a class lies. No blocking, folding or
 * reordering: each sample is handled on its own, in the order above.
 *
 * The multilayer-perceptron demapper oracle (forward, loss, backward, Adam)
 * follows at the end of the file.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LN2 0.69314718055994530942

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static int log2_exact(int M) {
    int m = 0;
    while ((1 << m) < M) m++;
    return m;
}

/* Sent rows must index X: returns 0 if every tx_idx[s] < M. */
static int rows_in_range(const uint32_t* tx_idx, int64_t n, int M) {
    for (int64_t s = 0; s < n; s++)
        if (tx_idx[s] >= (uint32_t)M) return 0;
    return 1;
}

/* t_j = ||y - x_j||^2 / (2 sigma2) for all j (nats). */
static void metrics(const double* y, const double* X, int M, int dim, double sigma2, double* t) {
    for (int j = 0; j < M; j++) {
        double d = 0.0;
        for (int q = 0; q < dim; q++) {
            double e = y[q] - X[(size_t)j * dim + q];
            d += e * e;
        }
        t[j] = d / (2.0 * sigma2);
    }
}

/* ln sum_{j in class} e^{-t_j}, class = {j : bit k of labels[j] == b};
 * k < 0 selects every point. Max-subtracted. Returns -INFINITY if empty. */
static double class_lse(const double* t, const uint32_t* labels, int M, int k, int b) {
    double mx = -INFINITY;
    for (int j = 0; j < M; j++) {
        if (k >= 0 && (int)((labels[j] >> k) & 1u) != b) continue;
        if (-t[j] > mx) mx = -t[j];
    }
    if (mx == -INFINITY) return mx;
    double s = 0.0;
    for (int j = 0; j < M; j++) {
        if (k >= 0 && (int)((labels[j] >> k) & 1u) != b) continue;
        s += exp(-t[j] - mx);
    }
    return mx + log(s);
}

/* softplus(u) = ln(1 + e^u), stable for every u. */
static double softplus(double u) {
    return (u > 0.0 ? u : 0.0) + log1p(exp(-fabs(u)));
}

/* LLRs for one sample into llr[0..m-1] (nats); t is scratch of size M. */
static void llr_one(const double* y, int dim, const double* X, const uint32_t* labels, int M,
                    double sigma2, double* t, double* llr) {
    int m = log2_exact(M);
    metrics(y, X, M, dim, sigma2, t);
    for (int k = 0; k < m; k++)
        llr[k] = class_lse(t, labels, M, k, 1) - class_lse(t, labels, M, k, 0);
}

/* Per-bit LLRs (nats) of n samples; y is [n][dim], llr is [n][m]. */
int oracle_llr(const double* y, int64_t n, int dim, const double* X, const uint32_t* labels,
               int M, double sigma2, double* llr) {
    int m = log2_exact(M);
    int err = 0;
#pragma omp parallel
    {
        double* t = (double*)malloc(sizeof(double) * (size_t)M);
        if (!t) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t s = 0; s < n; s++)
                llr_one(y + s * dim, dim, X, labels, M, sigma2, t, llr + s * m);
            free(t);
        }
    }
    return err ? -1 : 0;
}

/* Per-sample GMI and MI costs (bits). tx_idx[s] is the row of X sent
 * (returns -3, computing nothing, if some row is not below M). Either output
 * pointer may be NULL. */
int oracle_costs(const double* y, const uint32_t* tx_idx, int64_t n, int dim, const double* X,
                 const uint32_t* labels, int M, double sigma2, double* c_gmi, double* c_mi) {
    if (!rows_in_range(tx_idx, n, M)) return -3;
    int m = log2_exact(M);
    int err = 0;
#pragma omp parallel
    {
        double* t = (double*)malloc(sizeof(double) * (size_t)M);
        double* llr = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
        if (!t || !llr) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t s = 0; s < n; s++) {
                const double* ys = y + s * dim;
                uint32_t i = tx_idx[s];
                llr_one(ys, dim, X, labels, M, sigma2, t, llr);
                if (c_gmi) {
                    double c = 0.0;
                    for (int k = 0; k < m; k++) {
                        int b = (int)((labels[i] >> k) & 1u);
                        c += softplus(-(2.0 * b - 1.0) * llr[k]);
                    }
                    c_gmi[s] = c / LN2;
                }
                if (c_mi) {
                    /* log sum_j e^{-(t_j - t_i)} = t_i + ln sum_j e^{-t_j} */
                    c_mi[s] = (t[i] + class_lse(t, labels, M, -1, 0)) / LN2;
                }
            }
        }
        free(t);
        free(llr);
    }
    return err ? -1 : 0;
}

/* Mean and standard error of n per-sample costs, summed in order in FP64
 * with Kahan compensation. nonfinite counts entries that are NaN or inf. */
static void mean_se(const double* c, int64_t n, double* mean, double* se, int64_t* nonfinite) {
    double s = 0.0, comp = 0.0;
    int64_t bad = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!isfinite(c[i])) bad++;
        double yk = c[i] - comp;
        double tk = s + yk;
        comp = (tk - s) - yk;
        s = tk;
    }
    double mu = s / (double)n;
    double v = 0.0, cv = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double d = c[i] - mu;
        double yk = d * d - cv;
        double tk = v + yk;
        cv = (tk - v) - yk;
        v = tk;
    }
    *mean = mu;
    *se = n > 1 ? sqrt(v / ((double)n * (double)(n - 1))) : 0.0;
    *nonfinite = bad;
}

/* GMI / MI estimate of one SNR point. out[0..5] = {GMI, MI, SE_GMI, SE_MI, N,
 * n_nonfinite} with GMI and MI in bits per N-dimensional symbol. */
int oracle_gmi(const double* y, const uint32_t* tx_idx, int64_t n, int dim, const double* X,
               const uint32_t* labels, int M, double sigma2, double* out) {
    if (n < 1) return -2;
    double* cg = (double*)malloc(sizeof(double) * (size_t)n);
    double* cm = (double*)malloc(sizeof(double) * (size_t)n);
    if (!cg || !cm) {
        free(cg);
        free(cm);
        return -1;
    }
    int rc = oracle_costs(y, tx_idx, n, dim, X, labels, M, sigma2, cg, cm);
    if (rc == 0) {
        int m = log2_exact(M);
        double mg, sg, mm, sm;
        int64_t bg, bm;
        mean_se(cg, n, &mg, &sg, &bg);
        mean_se(cm, n, &mm, &sm, &bm);
        int64_t bad = 0;
        for (int64_t i = 0; i < n; i++)
            if (!isfinite(cg[i]) || !isfinite(cm[i])) bad++;
        out[0] = m - mg;
        out[1] = m - mm;
        out[2] = sg;
        out[3] = sm;
        out[4] = (double)n;
        out[5] = (double)bad;
        (void)bg;
        (void)bm;
    }
    free(cg);
    free(cm);
    return rc;
}

/* ------------------------------------------------------------------------
 * Max-log LLRs (FP64). Each class log-sum-exp is replaced by its largest
 * term, ln sum_{j in C} e^{-t_j} ~ -min_{j in C} t_j (the error lies in
 * [0, ln |C|]):
 *   lambda_k^ML(y) = min_{j: b_k(j)=0} t_j - min_{j: b_k(j)=1} t_j   (nats)
 * i.e. the difference of the squared distances from y to the nearest point
 * of each class, over 2 sigma2.
 * ---------------------------------------------------------------------- */
static double class_min(const double* t, const uint32_t* labels, int M, int k, int b) {
    double mn = INFINITY;
    for (int j = 0; j < M; j++)
        if ((int)((labels[j] >> k) & 1u) == b && t[j] < mn) mn = t[j];
    return mn;
}

int oracle_llr_maxlog(const double* y, int64_t n, int dim, const double* X, const uint32_t* labels,
                      int M, double sigma2, double* llr) {
    int m = log2_exact(M);
    int err = 0;
#pragma omp parallel
    {
        double* t = (double*)malloc(sizeof(double) * (size_t)M);
        if (!t) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t s = 0; s < n; s++) {
                metrics(y + s * dim, X, M, dim, sigma2, t);
                for (int k = 0; k < m; k++)
                    llr[s * m + k] = class_min(t, labels, M, k, 0) - class_min(t, labels, M, k, 1);
            }
            free(t);
        }
    }
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------
 * Hard decisions (FP64). Two decisions per received sample:
 *   bitwise MAP   b_hat_k = 1 if lambda_k > 0, else 0   (the sign of the
 *                 exact LLR: the hard decision of bit-metric decoding)
 *   nearest point j_hat = argmin_j ||y - x_j||^2; among points at the same
 *                 smallest distance the one with the lowest label is decided
 *                 (a fixed rule a receiver can apply: it does not know the
 *                 sent point; ties have probability zero under continuous
 *                 noise except where two labels share one point)
 * Per sample: errs[s] = number of k with b_hat_k != b_k(i) (0..m) and
 * sym[s] = 1 if j_hat != i, i.e. some j has ||y - x_j|| < ||y - x_i||, or
 * ||y - x_j|| = ||y - x_i|| with label(j) < label(i); else 0. The estimates are
 *   BER = sum errs / (n m),  SER = sum sym / n.
 * Non-finite samples count as errors and are reported separately.
 * ---------------------------------------------------------------------- */
static void hd_one(const double* y, int dim, const double* X, const uint32_t* labels, int M, double sigma2,
                   uint32_t row, double* t, int* errs, int* sym) {
    int m = log2_exact(M);
    metrics(y, X, M, dim, sigma2, t);
    int e = 0;
    uint32_t lab = labels[row];
    for (int k = 0; k < m; k++) {
        double lam = class_lse(t, labels, M, k, 1) - class_lse(t, labels, M, k, 0);
        int bhat = lam > 0.0 ? 1 : 0;
        if (!(lam == lam)) bhat = -1; /* NaN: an error for either bit value */
        if (bhat != (int)((lab >> k) & 1u)) e++;
    }
    /* nearest-point decision, ties to the lowest label: wrong iff another
     * point is strictly nearer, or as near with a lower label */
    int wrong = !(t[row] == t[row]);
    for (int j = 0; j < M; j++)
        if (t[j] < t[row] || (t[j] == t[row] && labels[j] < lab)) wrong = 1;
    *errs = e;
    *sym = wrong;
}

/* out[0] = BER, out[1] = SER, out[2] = n, out[3] = non-finite samples. */
int oracle_hd(const double* y, const uint32_t* tx_idx, int64_t n, int dim, const double* X,
              const uint32_t* labels, int M, double sigma2, double* out) {
    if (n < 1) return -2;
    if (!rows_in_range(tx_idx, n, M)) return -3;
    int m = log2_exact(M);
    int64_t bit_err = 0, sym_err = 0, bad = 0;
    int err = 0;
#pragma omp parallel reduction(+ : bit_err, sym_err, bad)
    {
        double* t = (double*)malloc(sizeof(double) * (size_t)M);
        if (!t) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t s = 0; s < n; s++) {
                int e, q;
                const double* ys = y + s * dim;
                int finite = 1;
                for (int d = 0; d < dim; d++)
                    if (!isfinite(ys[d])) finite = 0;
                hd_one(ys, dim, X, labels, M, sigma2, tx_idx[s], t, &e, &q);
                if (!finite) {
                    e = m;
                    q = 1;
                    bad++;
                }
                bit_err += e;
                sym_err += q;
            }
            free(t);
        }
    }
    if (err) return -1;
    out[0] = (double)bit_err / ((double)n * (double)m);
    out[1] = (double)sym_err / (double)n;
    out[2] = (double)n;
    out[3] = (double)bad;
    return 0;
}

/* ------------------------------------------------------------------------
 * MLP demapper oracle (FP64). A fully connected network maps the input
 * features x (the received sample and an SNR feature) to m logits that are
 * read as LLRs in nats:
 *   h_0 = x;  z_l = W_l h_{l-1} + b_l;  h_l = gelu(z_l) for hidden layers,
 *   logits = z_L (no activation on the output layer).
 * W_l is [out][in] row-major; parameters are laid out flat as
 * W_1, b_1, W_2, b_2, ..., W_L, b_L. GELU is the tanh form of Hendrycks &
 * Gimpel (2016). Loss: binary cross-entropy with logits against target
 * probabilities p (softplus(z) - p z per bit), summed over bits and
 * averaged over samples, in nats. Optimiser: Adam (Kingma & Ba, 2015).
 * ---------------------------------------------------------------------- */
#define GELU_C 0.79788456080286535588 /* sqrt(2/pi) */
#define GELU_A 0.044715

double oracle_gelu(double x) {
    return 0.5 * x * (1.0 + tanh(GELU_C * (x + GELU_A * x * x * x)));
}

static double gelu_grad(double x) {
    double u = GELU_C * (x + GELU_A * x * x * x);
    double t = tanh(u);
    double du = GELU_C * (1.0 + 3.0 * GELU_A * x * x);
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * du;
}

int64_t oracle_mlp_param_count(const int* sizes, int L) {
    int64_t p = 0;
    for (int l = 0; l < L; l++) p += (int64_t)sizes[l + 1] * sizes[l] + sizes[l + 1];
    return p;
}

/* Forward of one sample; z and h hold every layer's pre- and post-activation
 * values (layer l at offset off[l]). */
static void mlp_forward_one(const double* params, const int* sizes, int L, const double* x, double* z, double* h,
                            const int64_t* off) {
    const double* prev = x;
    const double* p = params;
    for (int l = 0; l < L; l++) {
        int in = sizes[l], out = sizes[l + 1];
        const double* W = p;
        const double* b = p + (int64_t)out * in;
        p = b + out;
        for (int o = 0; o < out; o++) {
            double s = b[o];
            for (int i = 0; i < in; i++) s += W[(int64_t)o * in + i] * prev[i];
            z[off[l] + o] = s;
            h[off[l] + o] = (l < L - 1) ? oracle_gelu(s) : s;
        }
        prev = h + off[l];
    }
}

static int64_t* layer_offsets(const int* sizes, int L, int64_t* total) {
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)L);
    int64_t t = 0;
    for (int l = 0; l < L; l++) {
        off[l] = t;
        t += sizes[l + 1];
    }
    *total = t;
    return off;
}

/* logits [n][sizes[L]] of x [n][sizes[0]]. */
int oracle_mlp_forward(const double* params, const int* sizes, int L, const double* x, int64_t n, double* logits) {
    int64_t tot;
    int64_t* off = layer_offsets(sizes, L, &tot);
    int err = 0;
#pragma omp parallel
    {
        double* z = (double*)malloc(sizeof(double) * (size_t)tot);
        double* h = (double*)malloc(sizeof(double) * (size_t)tot);
        if (!z || !h) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t s = 0; s < n; s++) {
                mlp_forward_one(params, sizes, L, x + s * sizes[0], z, h, off);
                for (int k = 0; k < sizes[L]; k++) logits[s * sizes[L] + k] = h[off[L - 1] + k];
            }
        }
        free(z);
        free(h);
    }
    free(off);
    return err ? -1 : 0;
}

/* Mean BCE-with-logits loss over n samples (summed over outputs) and its
 * gradient with respect to every parameter (grad [P], overwritten). */
double oracle_mlp_loss_grad(const double* params, const int* sizes, int L, const double* x, const double* target,
                            int64_t n, double* grad) {
    int64_t tot;
    int64_t* off = layer_offsets(sizes, L, &tot);
    const int64_t P = oracle_mlp_param_count(sizes, L);
    const int out_dim = sizes[L];
    int maxw = 0;
    for (int l = 0; l <= L; l++)
        if (sizes[l] > maxw) maxw = sizes[l];
    for (int64_t i = 0; i < P; i++) grad[i] = 0.0;
    double loss = 0.0;
    double* z = (double*)malloc(sizeof(double) * (size_t)tot);
    double* h = (double*)malloc(sizeof(double) * (size_t)tot);
    double* d = (double*)malloc(sizeof(double) * (size_t)maxw);   /* dLoss/dz of the current layer */
    double* dn = (double*)malloc(sizeof(double) * (size_t)maxw);
    int64_t* poff = (int64_t*)malloc(sizeof(int64_t) * (size_t)L); /* offset of W_l in params */
    int64_t q = 0;
    for (int l = 0; l < L; l++) {
        poff[l] = q;
        q += (int64_t)sizes[l + 1] * sizes[l] + sizes[l + 1];
    }
    for (int64_t s = 0; s < n; s++) {
        const double* xs = x + s * sizes[0];
        mlp_forward_one(params, sizes, L, xs, z, h, off);
        for (int k = 0; k < out_dim; k++) {
            double zz = z[off[L - 1] + k], p = target[s * out_dim + k];
            loss += softplus(zz) - p * zz;
            d[k] = (1.0 / (1.0 + exp(-zz)) - p) / (double)n;
        }
        for (int l = L - 1; l >= 0; l--) {
            int in = sizes[l], out = sizes[l + 1];
            const double* prev = l > 0 ? h + off[l - 1] : xs;
            double* gW = grad + poff[l];
            double* gb = gW + (int64_t)out * in;
            const double* W = params + poff[l];
            for (int o = 0; o < out; o++) {
                gb[o] += d[o];
                for (int i = 0; i < in; i++) gW[(int64_t)o * in + i] += d[o] * prev[i];
            }
            if (l > 0) {
                for (int i = 0; i < in; i++) {
                    double acc = 0.0;
                    for (int o = 0; o < out; o++) acc += W[(int64_t)o * in + i] * d[o];
                    dn[i] = acc * gelu_grad(z[off[l - 1] + i]);
                }
                for (int i = 0; i < in; i++) d[i] = dn[i];
            }
        }
    }
    free(z);
    free(h);
    free(d);
    free(dn);
    free(poff);
    free(off);
    return loss / (double)n;
}

/* One Adam step (bias-corrected, step number t >= 1) on P parameters. */
void oracle_adam(double* params, const double* grad, double* m, double* v, int64_t P, int64_t t, double lr,
                 double b1, double b2, double eps) {
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < P; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        params[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* GMI cost (bits) of given LLRs llr [n][m] for the sent labels. */
int oracle_gmi_cost_from_llr(const double* llr, const uint32_t* sent_label, int64_t n, int m, double* cost) {
    for (int64_t s = 0; s < n; s++) {
        double c = 0.0;
        for (int k = 0; k < m; k++) {
            int b = (int)((sent_label[s] >> k) & 1u);
            c += softplus(-(2.0 * b - 1.0) * llr[s * m + k]);
        }
        cost[s] = c / LN2;
    }
    return 0;
}
