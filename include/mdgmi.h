/*
 * mdgmi — exact per-bit LLRs and Monte-Carlo GMI / MI of N-dimensional
 * modulation formats over the AWGN channel, on AMD Instinct MI355X (gfx950).
 *
 * What is computed. The paper lists GMI, MI, LLR, BICM/BMD, AWGN and SNR in
 * its glossary and names the 4D/8D polarization-ring-switching and
 * two-amplitude 8PSK formats there; it gives no formula. The library follows
 * the standard definitions for bit-interleaved coded modulation with
 * bit-metric decoding, uniform priors:
 *
 *   y = x_i + z,  z ~ N(0, sigma2 I_N),  t_j(y) = ||y - x_j||^2 / (2 sigma2)
 *   lambda_k(y) = ln sum_{j: b_k(j)=1} e^{-t_j} - ln sum_{j: b_k(j)=0} e^{-t_j}   (nats)
 *   GMI = m - (1/n) sum_s sum_k log2(1 + exp(-(2 b_k(i_s) - 1) lambda_k(y_s)))
 *   MI  = m - (1/n) sum_s log2 sum_j exp(-(t_j(y_s) - t_{i_s}(y_s)))
 *
 * with b_k(j) = bit k (LSB first) of the label of constellation row j and
 * m = log2 M. LLR column k is label bit k; a positive LLR favours bit 1.
 *
 * Conventions shared by every call:
 *  - Array arguments named "device" are device pointers on the device that
 *    was current when the format was created; the caller owns them and keeps
 *    them alive until the stream has passed the call. "host" arrays are read
 *    before the call returns and are not retained.
 *  - Arrays are row-major and contiguous.
 *  - `stream` is a hipStream_t passed as void* (NULL: the default stream).
 *    Launches are asynchronous on that stream; nothing synchronises it.
 *  - Every argument is checked on the host before anything is launched; a
 *    failed check returns a negative mdgmi_status and launches nothing.
 *  - Device memory is allocated only by mdgmi_format_create,
 *    mdgmi_batch_create, mdgmi_stream_create, mdgmi_mlp_create and
 *    mdgmi_autotune (its synthetic samples, freed before it returns);
 *    mdgmi_batch_run instantiates a HIP graph on its first replay for an
 *    output buffer. Every other call takes its scratch memory from the
 *    caller's workspace (mdgmi_gmi_static: from a static device array).
 *  - Calls on distinct (stream, workspace, output) triples may overlap;
 *    calls sharing a workspace must be ordered by the caller.
 */
#ifndef MDGMI_H
#define MDGMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MDGMI_OK = 0,
    MDGMI_E_NULL = -1,        /* a required pointer is NULL */
    MDGMI_E_SHAPE = -2,       /* n < 1, n_snr < 1, dim or M out of range */
    MDGMI_E_LABELS = -3,      /* labels are not a permutation of [0, M) */
    MDGMI_E_SIGMA2 = -4,      /* a sigma2 is not finite and > 0 */
    MDGMI_E_UNSUPPORTED = -5, /* path not available for this dim / M / SNR */
    MDGMI_E_WORKSPACE = -6,   /* workspace NULL or smaller than required */
    MDGMI_E_HIP = -7,         /* a HIP runtime call or launch failed */
    MDGMI_E_DEVICE = -8,      /* current device differs from the format's */
    MDGMI_E_ARG = -9          /* another argument is out of range */
} mdgmi_status;

/* Arithmetic of the demapper. The element type of y / LLR follows the path:
 * double for MDGMI_PATH_F64, float for every other path. */
typedef enum {
    MDGMI_PATH_F64 = 0,              /* FP64 throughout, exact per class          */
    MDGMI_PATH_F32_DIRECT = 1,       /* FP32 distances on the vector ALUs         */
    MDGMI_PATH_F32_MFMA_F16SPLIT = 2,/* distance term on MFMA, fp16 hi+lo split,  */
                                     /* FP32 accumulate; log-sum-exp in FP32;     */
                                     /* needs 2s max|x| and s max||x||^2 < 3e4;   */
                                     /* 32x32 tiles, or for 4 <= M <= 512 (8-D:   */
                                     /* M <= 256) one sample per lane on 4x4 blocks */
    MDGMI_PATH_F32_MFMA_BF16SPLIT = 3,/* distance term on MFMA, bf16 three-part  */
                                     /* split (six products per coordinate,       */
                                     /* ~24 bits), FP32 accumulate: any SNR; one  */
                                     /* launch shape; not in ragged batches       */
    MDGMI_PATH_LEARNED_BF16 = 4,     /* mdgmi_gmi / mdgmi_llr only: the MLP       */
                                     /* demapper attached by                      */
                                     /* mdgmi_learned_calibrate (bf16 MFMA, FP32  */
                                     /* accumulate) at the SNR points calibration */
                                     /* routed to it, the exact fallback path     */
                                     /* everywhere else; float y / LLRs           */
    MDGMI_PATH_AUTO = 5              /* fastest FP32 exact path for the shape:    */
                                     /* the autotuner's choice for (dim, M), else */
                                     /* the fp16 split where its 4x4 shape serves */
                                     /* M or M >= 128, direct otherwise; the bf16 */
                                     /* split where fp16 is out of range (M>=128) */
} mdgmi_path;

/* Fields of one GMI/MI result row (doubles). */
enum {
    MDGMI_F_GMI = 0,       /* GMI estimate, bits per N-dimensional symbol   */
    MDGMI_F_MI = 1,        /* MI estimate, bits per N-dimensional symbol    */
    MDGMI_F_SE_GMI = 2,    /* standard error of the GMI estimate            */
    MDGMI_F_SE_MI = 3,     /* standard error of the MI estimate             */
    MDGMI_F_N = 4,         /* number of samples                              */
    MDGMI_F_NONFINITE = 5, /* samples whose GMI or MI cost is NaN or inf    */
    MDGMI_NFIELDS = 6,
    MDGMI_F_BER = 6,       /* mdgmi_gmi_hd: bit error rate of the bitwise   */
                           /* MAP decisions (the signs of the exact LLRs)   */
    MDGMI_F_SER = 7,       /* mdgmi_gmi_hd: symbol error rate of the        */
                           /* nearest-point decisions                        */
    MDGMI_NFIELDS_HD = 8
};

#define MDGMI_MAX_BITS 12   /* M <= 4096 */

typedef struct mdgmi_format mdgmi_format;

/* Human-readable text of a status code (static storage). */
const char* mdgmi_status_string(int status);

/* Host-side check that labels_host[0..M) is a permutation of [0, M).
 * Returns MDGMI_OK or MDGMI_E_LABELS / MDGMI_E_NULL / MDGMI_E_SHAPE. */
int mdgmi_validate_labels(const uint32_t* labels_host, int32_t M);

/* Stage a constellation on the current device (once per format).
 *   X_host      host [M][dim] double: the points, any scale (the channel model
 *               above applies to them as given; formats are normally scaled
 *               to unit average energy per N-dimensional symbol).
 *   labels_host host [M] uint32: labels_host[j] is the m-bit label of row j.
 *   M           2^m with 1 <= m <= MDGMI_MAX_BITS;  dim in {1, 2, 4, 8} (1: PAM
 *               on one real axis, as in the IM/DD chain of the paper).
 * On success *out receives a handle owning device memory; release it with
 * mdgmi_format_destroy. Synchronous. */
int mdgmi_format_create(const double* X_host, const uint32_t* labels_host, int32_t M, int32_t dim,
                        mdgmi_format** out);
int mdgmi_format_destroy(mdgmi_format* fmt);

/* Seeded channel samples (the Monte-Carlo input), generated on the device.
 * For SNR slot q (0 <= q < n_snr) and sample s (0 <= s < n) it draws, with
 * Philox-4x32-10 (Salmon et al., SC'11) keyed by `seed` and counter
 * (s mod 2^32, s / 2^32, snr_slot0 + q, call):
 *   call 0, word 0    -> transmitted row i = word >> (32 - m)
 *   calls 1..2        -> N(0,1) deviates by Box-Muller from word pairs,
 *                        u = (word + 1/2) 2^-32
 * and writes y[q][s][:] = x_i + sqrt(sigma2_host[q]) * z (computed in FP64,
 * stored as double if y_is_f64 else float) and tx_idx[q][s] = i.
 *   y       device [n_snr][n][dim];   tx_idx  device [n_snr][n] uint32. */
int mdgmi_generate(const mdgmi_format* fmt, uint64_t seed, const double* sigma2_host, int32_t n_snr,
                   int64_t n, int32_t snr_slot0, void* y, uint32_t* tx_idx, int32_t y_is_f64,
                   void* stream);

/* Bytes of workspace mdgmi_llr needs for n samples on `path`. */
int mdgmi_llr_workspace_size(const mdgmi_format* fmt, int64_t n, int32_t path, size_t* bytes);

/* Exact per-bit LLRs of n samples at one noise variance.
 *   y    device [n][dim] (double for MDGMI_PATH_F64, else float)
 *   llr  device [n][m]   (same element type), nats, column k = label bit k
 *   ws   device workspace of at least mdgmi_llr_workspace_size bytes.
 * FP32 paths: within about 1e-3 max(|llr|, 1) nats of the exact values.
 * Classes far from y take a per-class path; where s max||x||^2 > 1000
 * (s = log2(e) / (2 sigma2)) a sample with an LLR near zero is recomputed
 * there too, since the expanded distance form loses absolute accuracy in
 * proportion to s. Non-finite samples give NaN LLRs. */
int mdgmi_llr(const mdgmi_format* fmt, const void* y, int64_t n, double sigma2, void* llr,
              int32_t path, void* ws, size_t ws_bytes, void* stream);

/* Bytes of workspace mdgmi_gmi needs. */
int mdgmi_gmi_workspace_size(const mdgmi_format* fmt, int64_t n, int32_t n_snr, int32_t path,
                             size_t* bytes);

/* GMI and MI estimates for n_snr SNR points of n samples each.
 *   y           device [n_snr][n][dim] (double for MDGMI_PATH_F64, else float)
 *   tx_idx      device [n_snr][n] uint32, the transmitted rows of X
 *   sigma2_host host [n_snr] noise variance per real dimension
 *   out         device [n_snr][MDGMI_NFIELDS] double
 * The FP64 sum over samples is reduced in a fixed order: identical inputs
 * give bit-identical outputs. NaN in y gives NaN estimates for that SNR and
 * is counted in MDGMI_F_NONFINITE. */
int mdgmi_gmi(const mdgmi_format* fmt, const void* y, const uint32_t* tx_idx, int64_t n,
              const double* sigma2_host, int32_t n_snr, int32_t path, double* out, void* ws,
              size_t ws_bytes, void* stream);

/* Hard decisions on the same pass. The paper's figure of merit is the
 * Q-factor estimated from the bit error rate (continuous real-time
 * transmission subsection), compared with HD-FEC thresholds (experimental
 * results subsections of the IM/DD and KK chains). Everything mdgmi_gmi
 * computes, plus per SNR point:
 *   MDGMI_F_BER  fraction of (sample, bit) pairs whose bitwise MAP decision
 *                (bit k = 1 iff lambda_k > 0) differs from the sent bit;
 *   MDGMI_F_SER  fraction of samples whose nearest-point decision is not
 *                the sent point; among points at the same distance the
 *                lowest label is decided (a fixed rule, as a receiver that
 *                does not know the sent point must use). A point that
 *                shares its coordinates with a lower label is therefore
 *                never decided. The FP32 paths decide from rounded
 *                metrics: near-ties between distinct points go either way
 *                within that rounding.
 * A sample with non-finite y counts m bit errors and one symbol error.
 *   out  device [n_snr][MDGMI_NFIELDS_HD] double.
 * Paths as for mdgmi_gmi (the MFMA path runs its 16-wave single-column
 * shape here whatever the tuning). */
int mdgmi_gmi_hd_workspace_size(const mdgmi_format* fmt, int64_t n, int32_t n_snr, int32_t path,
                                size_t* bytes);
int mdgmi_gmi_hd(const mdgmi_format* fmt, const void* y, const uint32_t* tx_idx, int64_t n,
                 const double* sigma2_host, int32_t n_snr, int32_t path, double* out, void* ws,
                 size_t ws_bytes, void* stream);

/* Max-log metrics. Each class log-sum-exp in the LLR is replaced by its
 * largest term (the usual low-complexity demapper; the paper names GMI and
 * LLRs only in its glossary, so this is the standard approximation):
 *   lambda_k^ML(y) = (min_{j: b_k(j)=0} ||y - x_j||^2
 *                     - min_{j: b_k(j)=1} ||y - x_j||^2) / (2 sigma2)  (nats)
 * mdgmi_llr_maxlog: as mdgmi_llr (same layout, paths, workspace size from
 *   mdgmi_llr_workspace_size), max-log LLRs instead of exact ones.
 * mdgmi_gmi_maxlog: as mdgmi_gmi (same workspace size), the GMI of the
 *   max-log LLRs at s = 1 with its standard error; MDGMI_F_MI and
 *   MDGMI_F_SE_MI are NaN (max-log metrics define no MI).
 * A sample whose nearest point is far outside the common exponent window
 * (or whose y is not finite) is evaluated from FP32 distances; non-finite
 * samples give NaN LLRs / are counted in MDGMI_F_NONFINITE. */
int mdgmi_llr_maxlog(const mdgmi_format* fmt, const void* y, int64_t n, double sigma2, void* llr,
                     int32_t path, void* ws, size_t ws_bytes, void* stream);
int mdgmi_gmi_maxlog(const mdgmi_format* fmt, const void* y, const uint32_t* tx_idx, int64_t n,
                     const double* sigma2_host, int32_t n_snr, int32_t path, double* out, void* ws,
                     size_t ws_bytes, void* stream);

/* s-optimised GMI and NGMI of given LLRs (any demapper: exact, max-log or
 * learned). With v_ik = (2 b_k(i) - 1) lambda_ik for the sent bits,
 *   GMI(s) = m - (1/n) sum_i sum_k log2(1 + exp(-s v_ik)),   s >= 0,
 * is the GMI of a bit-metric decoder using the LLRs scaled by s; the
 * s-optimised GMI is max_s GMI(s) (concave in s; found on the device by
 * safeguarded Newton steps, no host synchronisation). NGMI = GMI / m, the
 * normalised GMI for uniform priors (glossary entry NGMI of the paper).
 *   llr      device [n][m] FP32 (llr_is_f64 = 0) or FP64 (1), nats
 *   tx_idx   device [n] uint32 rows of the format that were sent
 *   out      device [MDGMI_NFIELDS_S] double, fields below
 *   ws       device workspace of mdgmi_gmi_sopt_workspace_size bytes
 * A non-finite LLR or a sent row outside [0, M) makes every estimate NaN
 * (counted in MDGMI_S_NONFINITE). LLRs that favour the wrong bit on average
 * give s* = 0 and GMI = 0. */
enum {
    MDGMI_S_GMI1 = 0,      /* GMI at s = 1 (the LLRs as given)            */
    MDGMI_S_SE1 = 1,       /* its standard error                          */
    MDGMI_S_S = 2,         /* s* maximising GMI(s)                         */
    MDGMI_S_GMI = 3,       /* GMI(s*), the s-optimised GMI                 */
    MDGMI_S_SE = 4,        /* standard error of GMI(s*)                    */
    MDGMI_S_NGMI = 5,      /* GMI(s*) / m                                  */
    MDGMI_S_N = 6,         /* number of samples                            */
    MDGMI_S_NONFINITE = 7, /* samples with a non-finite cost               */
    MDGMI_S_ITERS = 8,     /* evaluation passes used                       */
    MDGMI_NFIELDS_S = 9
};
int mdgmi_gmi_sopt_workspace_size(int64_t n, size_t* bytes);
int mdgmi_gmi_sopt(const mdgmi_format* fmt, const void* llr, int32_t llr_is_f64, const uint32_t* tx_idx,
                   int64_t n, double* out, void* ws, size_t ws_bytes, void* stream);

/* Per-bit GMI of given LLRs (the LLRs as given, s = 1): for each label bit k
 *   GMI_k = 1 - (1/n) sum_i log2(1 + exp(-(2 b_k(i) - 1) lambda_ik)),
 * the bit's share of the GMI (sum_k GMI_k = MDGMI_S_GMI1 of mdgmi_gmi_sopt).
 *   llr, tx_idx as for mdgmi_gmi_sopt
 *   out    device [2 m + 2] double: out[2k] = GMI_k, out[2k+1] its standard
 *          error (k < m), out[2m] = n, out[2m+1] = samples with a non-finite
 *          cost (those make the GMI_k NaN)
 *   ws     device workspace of mdgmi_gmi_bits_workspace_size bytes */
int mdgmi_gmi_bits_workspace_size(int64_t n, size_t* bytes);
int mdgmi_gmi_bits(const mdgmi_format* fmt, const void* llr, int32_t llr_is_f64, const uint32_t* tx_idx,
                   int64_t n, double* out, void* ws, size_t ws_bytes, void* stream);

/* ---- streaming monitor ---------------------------------------------------
 * GMI/MI of a receiver's output as it arrives, in fixed-size buffers (the
 * paper's receiver processes its ADC stream in buffers of 2^22 samples on
 * several streams ordered by events; real-time GPU receiver architecture
 * section). Each buffer holds up to buffer_n received samples of one format
 * at one noise level, with the rows that were sent. Buffers are taken in
 * turn by n_lanes HIP streams (default priority), each with its own device
 * buffers; a separate stream accumulates the buffers in push order, so the
 * per-buffer rows and the running totals are bit-identical for any number
 * of lanes, and each buffer's row equals mdgmi_gmi on the same samples.
 *   mdgmi_stream_create  sigma2 > 0 fixed for the stream; buffer_n >= 1;
 *                        1 <= n_lanes <= 8; path as for mdgmi_gmi (resolved
 *                        once); ring >= 1 result rows kept on the device.
 *                        Allocates all device memory (synchronous).
 *   mdgmi_stream_push    one buffer of n <= buffer_n samples: y [n][dim]
 *                        (double on the FP64 path, else float) and tx_idx
 *                        [n] uint32. from_host = 1: host pointers, copied
 *                        asynchronously on the buffer's lane (use pinned
 *                        memory for overlap; keep it unchanged until
 *                        mdgmi_stream_wait(index) returns); from_host = 0:
 *                        device pointers read in place (same lifetime
 *                        rule). *index receives the buffer's sequence number.
 *   mdgmi_stream_wait    block until buffer `index` (and every earlier one)
 *                        is accumulated; index < 0 waits for all.
 *   mdgmi_stream_result  host [MDGMI_NFIELDS] row of buffer `index` (waits);
 *                        MDGMI_E_ARG once the ring has moved past it.
 *   mdgmi_stream_total   host [MDGMI_NFIELDS] over every buffer since create
 *                        or reset (waits for all).
 *   mdgmi_stream_reset   zero the running totals (waits for all).
 * A stream object is used from one host thread at a time. */
typedef struct mdgmi_stream mdgmi_stream;
int mdgmi_stream_create(const mdgmi_format* fmt, double sigma2, int64_t buffer_n, int32_t n_lanes, int32_t path,
                        int32_t ring, mdgmi_stream** out);
int mdgmi_stream_push(mdgmi_stream* s, const void* y, const uint32_t* tx_idx, int64_t n, int32_t from_host,
                      int64_t* index);
int mdgmi_stream_wait(mdgmi_stream* s, int64_t index);
int mdgmi_stream_result(mdgmi_stream* s, int64_t index, double* out_host);
int mdgmi_stream_total(mdgmi_stream* s, double* out_host);
int mdgmi_stream_reset(mdgmi_stream* s);
/* Buffers pushed so far and the resolved path. */
int mdgmi_stream_info(const mdgmi_stream* s, int64_t* pushed, int32_t* path);
int mdgmi_stream_destroy(mdgmi_stream* s);

/* Q-factor in dB of a bit error rate, 20 log10(sqrt(2) erfc^-1(2 ber)) (the
 * Gaussian-noise conversion; the paper states no formula). Host-only, no
 * GPU needed; +inf for ber = 0, -inf for ber = 0.5, NaN outside [0, 0.5]. */
double mdgmi_q_factor_db(double ber);

/* ---- no device allocation -------------------------------------------------
 * For callers that cannot allocate device memory (code being captured into
 * a HIP graph, tight serving loops, hosts that forbid hipMalloc):
 * mdgmi_gmi_static computes exactly what mdgmi_gmi computes (same arguments,
 * paths, launches and results, bit for bit), with its scratch memory (the
 * per-block FP64 partials and the per-SNR operand images) taken from a
 * static device array of MDGMI_STATIC_SCRATCH_BYTES that the library holds
 * on every device it runs on until the process ends. It calls no allocator.
 *  - MDGMI_E_WORKSPACE if the call's plan (the resolved path's partial sums
 *    and operand images, at most mdgmi_gmi_workspace_size(fmt, n, n_snr,
 *    path)) needs more than MDGMI_STATIC_SCRATCH_BYTES; nothing is launched
 *    then. 16 MiB holds the images of up to 32 SNR points (the most one
 *    launch takes) of every format on every path, except 32 points of an
 *    8-D M = 4096 format on the bf16 split (512 KiB each), which holds 31;
 *    the partial sums add 5 doubles per block and SNR point of the call,
 *    so calls with very many SNR points may not fit.
 *  - Every call on one device uses the same array, which keeps the last
 *    call's contents: calls that overlap on a device (other streams or host
 *    threads) race and must be ordered by the caller. No part of the array
 *    needs to start at zero: every launch writes what it later reads.
 *  - The first call on a device looks up the array's device address. */
#define MDGMI_STATIC_SCRATCH_BYTES (16u << 20)
int mdgmi_gmi_static(const mdgmi_format* fmt, const void* y, const uint32_t* tx_idx, int64_t n,
                     const double* sigma2_host, int32_t n_snr, int32_t path, double* out, void* stream);

/* ---- ragged batches ------------------------------------------------------
 * Many (format, SNR, sample count) instances evaluated by one persistent
 * kernel: the samples of every instance are cut into items of about 2^22
 * sample*points, a persistent grid pulls items from an atomic counter and
 * dispatches each to the direct or MFMA code of its (dim, M); per-item FP64
 * partials are reduced per instance in item order (bit-reproducible). */
typedef struct {
    const mdgmi_format* fmt;  /* staged format of this instance (any dim, M)   */
    const float* y;           /* device [n][dim] float                          */
    const uint32_t* tx_idx;   /* device [n], the transmitted rows of the format */
    int64_t n;                /* samples, >= 1                                  */
    double sigma2;            /* noise variance per real dimension, > 0         */
} mdgmi_instance;

/* Bytes of workspace mdgmi_gmi_batched needs (host-side planning only). */
int mdgmi_gmi_batched_workspace_size(const mdgmi_instance* inst_host, int32_t n_inst, int32_t path,
                                     size_t* bytes);

/* One-shot ragged batch. inst_host: host [n_inst]; out: device
 * [n_inst][MDGMI_NFIELDS] double, row q for inst_host[q]. path:
 * MDGMI_PATH_F32_DIRECT, MDGMI_PATH_F32_MFMA_F16SPLIT (every instance needs
 * M >= 128 and dim >= 2 for 32x32 tiles, or a format that the per-sample
 * 4x4 shape serves) or MDGMI_PATH_AUTO (per instance: the autotuner's
 * choice, else the 4x4 shape where it serves M, else MFMA tiles for
 * M >= 128, else direct). The work list is copied into the workspace on
 * `stream`. */
int mdgmi_gmi_batched(const mdgmi_instance* inst_host, int32_t n_inst, int32_t path, double* out, void* ws,
                      size_t ws_bytes, void* stream);

/* A reusable batch plan: work list and per-instance operand images built
 * once (device memory owned by the plan; y / tx_idx of every instance must
 * stay valid while the plan is used). With path AUTO, (dim, M) classes the
 * autotuner has not seen are tuned first. */
typedef struct mdgmi_batch mdgmi_batch;
int mdgmi_batch_create(const mdgmi_instance* inst_host, int32_t n_inst, int32_t path, mdgmi_batch** out);
/* Evaluate the plan into out (device [n_inst][MDGMI_NFIELDS]). use_graph != 0
 * replays a hipGraph of the three launches (counter reset, persistent kernel,
 * reduction), captured on first use for this `out`; else launches directly. */
int mdgmi_batch_run(mdgmi_batch* b, double* out, int32_t use_graph, void* stream);
/* Items in the work list, and total sample*points of the batch. */
int mdgmi_batch_info(const mdgmi_batch* b, int64_t* n_items, int64_t* pairs);
int mdgmi_batch_destroy(mdgmi_batch* b);

/* ---- autotuner --------------------------------------------------------------
 * Times the FP32 direct kernel and every MFMA launch variant on synthetic
 * samples of (dim, M) at 10 dB on the current device and records the
 * fastest, separately for two sample-count regimes of a launch (samples over
 * all its SNR points): bulk (at least MDGMI_TUNE_SHORT_SAMPLES), timed on
 * max(2^20, 2^28 / M) samples, at most 2^22 (at least two resident rounds of
 * every launch shape), and short (fewer), timed on 2^15 samples. The table
 * steers MDGMI_PATH_AUTO, the launch shape of MDGMI_PATH_F32_MFMA_F16SPLIT
 * calls (each call by its own regime, falling back to the other regime's
 * entry) and the per-instance kind of ragged batches (bulk). mdgmi_autotune
 * allocates and frees device memory and synchronises its own stream; it
 * re-times only with force or when an entry is missing. Rates in
 * sample*points/s. */
#define MDGMI_TUNE_SHORT_SAMPLES (1 << 18)
#define MDGMI_TUNE_BULK 0
#define MDGMI_TUNE_SHORT 1
typedef struct {
    int32_t dim, M;
    int32_t regime;        /* MDGMI_TUNE_BULK or MDGMI_TUNE_SHORT                */
    int32_t path;          /* MDGMI_PATH_F32_DIRECT or MDGMI_PATH_F32_MFMA_F16SPLIT */
    int32_t mfma_variant;  /* fastest MFMA launch variant, -1 if none ran     */
    int32_t pad;
    int64_t samples;       /* samples per timed call                          */
    double direct_rate, mfma_rate;
} mdgmi_tune_entry;
/* out: NULL or host [2], receives the bulk then the short entry */
int mdgmi_autotune(int32_t dim, int32_t M, int32_t force, mdgmi_tune_entry* out);
/* MDGMI_E_ARG if (dim, M) is untuned in that regime or regime is invalid */
int mdgmi_tune_lookup(int32_t dim, int32_t M, int32_t regime, mdgmi_tune_entry* out);
int mdgmi_tune_save(const char* path);   /* JSON */
int mdgmi_tune_load(const char* path);
int mdgmi_tune_clear(void);

/* ---- learned demapper (MLP) ----------------------------------------------
 * A fully connected network from features x = [y, (SNR_dB - 9.5) / 4.5] to m
 * logits read as LLRs in nats: z_l = W_l h_(l-1) + b_l, h_l = gelu(z_l) on
 * hidden layers (tanh form of Hendrycks & Gimpel), logits = z_L. FP32 master
 * parameters laid out flat as W_1 b_1 W_2 b_2 ... (W_l row-major [out][in]);
 * bf16 copies feed v_mfma_f32_32x32x16_bf16 GEMMs with FP32 accumulation;
 * activations and back-propagated gradients are bf16. Training minimises the
 * binary cross-entropy with logits against p = sigmoid(lambda_exact), summed
 * over bits and averaged over samples (nats), with Adam on the masters. */
#define MDGMI_MLP_MAX_LAYERS 8
typedef struct mdgmi_mlp mdgmi_mlp;
/* sizes_host[0..n_layers]: widths (input, hidden..., output), each 1..4096.
 * Initialisation: W, b ~ U(-1/sqrt(fan_in), +1/sqrt(fan_in)) from a 64-bit
 * Mersenne twister seeded with `seed` (53-bit uniforms). Allocates. */
int mdgmi_mlp_create(const int32_t* sizes_host, int32_t n_layers, uint64_t seed, mdgmi_mlp** out);
int mdgmi_mlp_destroy(mdgmi_mlp* net);
int mdgmi_mlp_param_count(const mdgmi_mlp* net, int64_t* count);
/* Copy (synchronously) the FP32 masters (which = 0), the last gradient (1) or
 * the Adam moments (2: first, 3: second) to host [count]. */
int mdgmi_mlp_get_params(const mdgmi_mlp* net, float* host, int64_t count, int32_t which);
/* Replace the masters (host [count]) and refresh the bf16 copies; synchronous. */
int mdgmi_mlp_set_params(mdgmi_mlp* net, const float* host, int64_t count);
/* Workspace for forward / loss_grad of n samples (activations, gradients). */
int mdgmi_mlp_workspace_size(const mdgmi_mlp* net, int64_t n, size_t* bytes);
/* Features: x [n][dim + 1] = [y, (snr_db - 9.5) / 4.5] from y [n][dim] (device). */
int mdgmi_mlp_features(const float* y, int64_t n, int32_t dim, double snr_db, float* x, void* stream);
/* logits [n][out] (device float) of x [n][in] (device float). */
int mdgmi_mlp_forward(const mdgmi_mlp* net, const float* x, int64_t n, float* logits, void* ws, size_t ws_bytes,
                      void* stream);
/* Forward + backward: loss (device double, 1 value) and the parameter
 * gradient, kept inside the network for mdgmi_mlp_adam_step.
 * target_llr: device [n][out] exact LLRs (targets p = sigmoid(target)). */
int mdgmi_mlp_loss_grad(mdgmi_mlp* net, const float* x, const float* target_llr, int64_t n, double* loss, void* ws,
                        size_t ws_bytes, void* stream);
/* One bias-corrected Adam step on the masters with the last gradient. */
int mdgmi_mlp_adam_step(mdgmi_mlp* net, float lr, float beta1, float beta2, float eps, void* stream);
/* GMI of the network's logits read as LLRs, per SNR point, for samples y
 * [n_snr][n][dim] (device float) with sent rows tx_idx [n_snr][n] of fmt;
 * snr_db_host [n_snr] feeds the SNR feature. Samples are processed in
 * chunks of `chunk` (at most 1024 chunks per SNR point). out [n_snr][6]:
 * GMI, NaN, SE_GMI, NaN, N, non-finite count. The network must have
 * fmt->dim + 1 inputs and log2(M) outputs. */
int mdgmi_mlp_gmi_workspace_size(const mdgmi_mlp* net, int64_t chunk, size_t* bytes);
int mdgmi_mlp_gmi(const mdgmi_mlp* net, const mdgmi_format* fmt, const float* y, const uint32_t* tx_idx, int64_t n,
                  const double* snr_db_host, int32_t n_snr, int64_t chunk, double* out, void* ws, size_t ws_bytes,
                  void* stream);
/* Inference kernel choice of mdgmi_mlp_gmi for networks of shape
 * [<=16, 256, 256, 256, <=32]: waves = 8 (default) or 4 per block for the
 * fused kernel (activations in registers, weights staged in LDS), 0 for the
 * layer-by-layer GEMM path. Process-wide; returns MDGMI_E_ARG otherwise. */
int mdgmi_mlp_set_fused(int waves);
/* One training step in one call: features [y, (snr_db - 9.5) / 4.5] from
 * y [n][dim] and the per-sample SNR snr_db [n] (device float, dB), then
 * forward, BCE loss and backward as mdgmi_mlp_loss_grad, then an Adam step
 * (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr. The network's
 * input width is dim + 1. loss: device double (mean BCE over samples, nats).
 * ws: mdgmi_mlp_train_workspace_size bytes. */
int mdgmi_mlp_train_workspace_size(const mdgmi_mlp* net, int64_t n, size_t* bytes);
int mdgmi_mlp_train_step(mdgmi_mlp* net, const float* y, const float* snr_db, const float* llr_target, int64_t n,
                         float lr, double* loss, void* ws, size_t ws_bytes, void* stream);
/* The network's logits read as LLRs: llr [n][out] (device float, nats) of
 * y [n][dim] at per-sample SNRs snr_db [n] (device float, dB). Networks of
 * the fused shape [<= 16, 256, 256, 256, <= 32] run the fused kernel and
 * need no workspace (size 0; ws may be NULL), others the layer-by-layer
 * GEMMs in a workspace of mdgmi_mlp_llr_workspace_size bytes. The fused
 * kernel evaluates the GELU gate sigmoid(2 sqrt(2/pi) (x + 0.044715 x^3))
 * as a clamped polynomial in packed fp16 (within 8e-4 of it; exactly 0 / 1
 * for |x| >= 4), the layer-by-layer path in the tanh form itself; both
 * results carry the bf16 rounding of weights and activations. */
int mdgmi_mlp_llr_workspace_size(const mdgmi_mlp* net, int64_t n, size_t* bytes);
int mdgmi_mlp_llr(const mdgmi_mlp* net, const float* y, const float* snr_db, int64_t n, float* llr, void* ws,
                  size_t ws_bytes, void* stream);

/* ---- learned demapper as a path, with per-SNR fallback -------------------
 * mdgmi_learned_calibrate attaches a network with dim + 1 inputs and
 * log2(M) outputs to a format and decides, per noise
 * variance, which demapper MDGMI_PATH_LEARNED_BF16 uses: on the given
 * held-out samples y [n_snr][n][dim] (float) with sent rows tx_idx, the
 * exact GMI on exact_path (an FP32 path or AUTO) and the network's GMI are
 * computed on the same samples; where the paired loss GMI_exact - GMI_learned
 * is at most max_loss (and both are finite) that sigma2 is routed to the
 * network, elsewhere to exact_path. result_host [n_snr][4] receives
 * GMI_exact, GMI_learned, the loss and the route (1 learned, 0 exact).
 * The network's SNR feature is 10 log10(E||x||^2 / (dim sigma2)) dB. Any
 * network shape is served (the fused kernel where it applies, else the
 * layer-by-layer GEMMs).
 * Synchronous (waits for `stream`); replaces an earlier calibration of the
 * format; the network must stay alive while the format uses it.
 * MDGMI_PATH_LEARNED_BF16 in mdgmi_gmi: SNR points routed to the network
 * give its GMI and SE (MI fields NaN: bit metrics only); every other point,
 * including noise variances never calibrated (matched to 1e-12 relative),
 * gives exactly what mdgmi_gmi on exact_path gives. In mdgmi_llr: the
 * network's LLRs or the exact ones, by the same rule. Workspaces: from
 * mdgmi_gmi_workspace_size / mdgmi_llr_workspace_size with this path (after
 * calibration; MDGMI_E_UNSUPPORTED before). */
int mdgmi_learned_calibrate_workspace_size(const mdgmi_format* fmt, const mdgmi_mlp* net, int32_t exact_path,
                                           int64_t n, int32_t n_snr, size_t* bytes);
int mdgmi_learned_calibrate(mdgmi_format* fmt, const mdgmi_mlp* net, int32_t exact_path, double max_loss,
                            const float* y, const uint32_t* tx_idx, int64_t n, const double* sigma2_host,
                            int32_t n_snr, double* result_host, void* ws, size_t ws_bytes, void* stream);

/* Checkpoint: widths, step, masters and both Adam moments (binary). */
int mdgmi_mlp_save(const mdgmi_mlp* net, const char* path);
int mdgmi_mlp_load(mdgmi_mlp* net, const char* path);

/* Measured peaks of the current device, behind the roofline figures (the
 * demapper is bound by the exponential issue rate of the vector ALU, the
 * learned demapper by the vector ALU beside the matrix cores): out_host [9]
 * receives
 *   [0] v_exp_f32 results per second over the whole device,
 *   [1] the core clock during that probe (Hz, s_memtime cycles against the
 *       constant reference clock),
 *   [2] FP32 FMA lane-operations per second, [3] the clock during it,
 *   [4] v_mfma_f32_32x32x16_bf16 flops per second,
 *   [5], [6], [7] the same MFMA flops per second at two waves per SIMD when
 *       each MFMA is followed by 0, 4 and 8 independent FP32 FMAs of its
 *       wave (how much vector work issues while the matrix core runs),
 *   [8] iterations per second of each SIMD when one of its two waves runs
 *       two MFMAs and the other sixteen FP32 FMAs per iteration (whether an
 *       MFMA holds up the vector issue of the other wave too).
 * Probes [0]-[4] run 8 waves per SIMD of independent dependency chains; the
 * call allocates and frees a few bytes of device memory and synchronises
 * the device (a measurement call, not for hot loops). */
int mdgmi_probe_rates(double* out_host);

/* Launch-shape override of the MFMA path for tuning sweeps: variant v in
 * 0..7 selects 32x32 tiles with (sample columns per wave, waves per block) =
 * (1,4), (2,4), (1,8), (2,8), (1,16), (1,12) with the operand image in LDS,
 * and (1,16), (1,8) reading it from L2; v = 8 the per-sample 4x4-block shape
 * (formats with 4 <= M <= 512, 8-D M <= 256; others keep their default);
 * v < 0 restores the built-in choice (the autotuner's, else the 4x4 shape
 * where it serves M, else a default). Process-wide; affects workspace sizes,
 * so set it before sizing workspaces. Always MDGMI_OK. */
int mdgmi_set_tuning(int mfma_variant);
int mdgmi_get_tuning(void);   /* the current override, -1 if none */

#ifdef __cplusplus
}
#endif

#endif /* MDGMI_H */
