/*
 * sft.h — C ABI of an MI355X (gfx950) implementation of sFFT-DT: sparse
 * FFT by downsampling in time and syndrome decoding (Hsieh, Lu, Pei,
 * arXiv 1407.8315), non-iterative (Sec. II-C, III) and iterative (Alg. 1).
 *
 * Problem statement (Alg. 1 and Alg. 2, "Input: x, K; Output: x_hat"): given
 * a length-N signal x whose spectrum x_hat has K significant entries, return
 * those entries as a sparse list of (location, value).
 *
 * DFT convention: forward DFT unnormalised, X[f] = sum_n x[n] e^{-2 pi i f n/N},
 * so a test signal is x = IDFT(x_hat) and the returned values are x_hat[s].
 *
 * The path on the device, per signal (Sec. II and III of the paper):
 *   1. gather x_{d,l}[k'] = x[(d k' + l) mod N] for 2L consecutive shifts l
 *      (general mode: also R random shifts n_j), M = N/d samples each;
 *   2. m_l = d * FFT_M(x_{d,l}) (the syndromes, Eq. (2)-(3));
 *   3. per bin k: activity test, order estimate (rank of the Hankel matrix
 *      of Eq. (5) — or the K-vote of Sec. III-C Step 1 in general mode, or a
 *      learned predictor), locator solve (Eq. (5)), roots matched to the grid
 *      {k + t M} (Alg. 1 grid check), Vandermonde least squares for the
 *      values (Step (iii)), residual judge, fallback over orders;
 *   4. general mode: bins no order explains go through pruning (Sec. III-C
 *      Steps 2-3) and Subspace Pursuit on the random-shift syndromes (Eq. (11));
 *   5. output sorted by location (general mode: the K largest values first).
 * Iterative mode (Alg. 1, exactly K-sparse) replaces 1-3 by a_m = L
 * iterations: iteration l takes the FFTs of shifts 2l and 2l + 1 at
 * d_l = 2^l d_0 (M_l = M_0 / 2^l), folds the earlier shifts' syndromes to that
 * grid, subtracts the frequencies solved so far (SubFreq) and decodes every
 * bin still open or newly non-zero at order a = l + 1 (SynDec); a bin whose
 * solution fails the grid check stays open (the set T) for the next grid.
 *
 * Memory: every pointer argument named *_dev is device memory (hipMalloc or a
 * torch CUDA tensor on the plan's device); everything else is host memory.
 * The caller owns inputs and outputs; a plan owns its workspace, tables and
 * graph until sft_destroy.  Calls are enqueued on the plan's stream and are
 * asynchronous, except that passing a non-NULL sft_stats (or SFT_FLAG_SYNC)
 * synchronises the stream and makes status codes such as SFT_E_CAPACITY
 * observable.  A plan is not thread-safe: use one plan per stream.
 * No call allocates device memory except sft_plan, sft_mlp_create and the
 * first sft_batch call of a plan (graph instantiation); sft_exact_noalloc
 * needs no plan and allocates nothing.
 *
 * Errors: every call returns a status; no exception crosses the ABI;
 * sft_last_error() gives the text of the last failure on the calling thread.
 */
#ifndef SFT_H
#define SFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SFT_ABI_VERSION 3
#define SFT_MAX_RSHIFTS 64

typedef enum sft_status {
    SFT_OK = 0,
    SFT_E_INVALID = 1,      /* NULL pointer, K <= 0, K > N, bad dtype or mode, wrong plan kind */
    SFT_E_UNSUPPORTED = 2,  /* N or M not a power of two, M does not divide N, L outside 1..4, M too large */
    SFT_E_NOMEM = 3,        /* device or host allocation failed */
    SFT_E_DEVICE = 4,       /* HIP runtime error (text in sft_last_error) */
    SFT_E_CAPACITY = 5,     /* an output list was too small; its count holds the required size */
    SFT_E_NONFINITE = 6     /* SFT_FLAG_CHECK_FINITE and a gathered sample is NaN or Inf */
} sft_status;

enum { SFT_C64 = 1, SFT_C128 = 2 };                 /* input element type: complex float / double, interleaved */
/* Sec. II-C (exactly K-sparse, non-iterative) / Sec. III (generally K-sparse) /
 * Alg. 1 (exactly K-sparse, iterative: m = M_0 = N / d_0, l = a_m iterations,
 * M_0 >= 2^(l-1); a plan's signals are all iterative or none) */
enum { SFT_MODE_EXACT = 0, SFT_MODE_GENERAL = 1, SFT_MODE_ITERATIVE = 2 };
enum {
    SFT_FLAG_LEARNED = 1u,       /* order estimate from the attached MLP; rank test as fallback */
    SFT_FLAG_SYNC = 2u,          /* synchronise at the end of each call */
    SFT_FLAG_CHECK_FINITE = 4u,  /* count non-finite gathered samples; report SFT_E_NONFINITE (sync calls) */
    SFT_FLAG_AUTOTUNE = 8u,      /* exact mode: M and L chosen by sft_autotune (m and l must be 0) */
    SFT_FLAG_FFT64 = 16u,        /* complex64 input: FFTs and syndromes in FP64 (set on all signals
                                    of a plan or on none); decisions then no longer depend on FP32
                                    rounding of the syndromes */
    SFT_FLAG_SP_ALL = 32u,       /* general mode, Alg. 2 as printed: every voted bin goes straight
                                    to pruning and Subspace Pursuit (no syndrome decoding first) */
    SFT_FLAG_UNKNOWN_K = 64u     /* exact mode, single signal, K unknown (k is ignored; pass 1):
                                    sft_unknown_k tries M = 1, 2, 4 .. m (m = 0: min(N, 2^22)) */
};

/* Parameters of one signal.  Zero means "default" for m, l, r and every
 * threshold.  Defaults: M = 4K rounded up to a power of two (at most N),
 * L = 4 (the paper's a_m = 4, Sec. II-E), R = 3L (Sec. III-A: r = 3 a_m).
 * Thresholds (complex64 / complex128 input): tau_zero 1e-4 / 1e-9 (activity:
 * E_k > tau_zero^2 mean E), tau_rank 1e-5 / 1e-10 (order = #sigma_i > tau_rank
 * sigma_1), tau_res 1e-4 / 1e-9 and c_res 3 (judge: residual^2 <= tau_res^2 E_k
 * + c_res (2L - a) nu), tau_amp 1e-4 / 1e-9 (drop |p_j| < tau_amp max|p|),
 * delta_grid 0.1 (root within 0.1 grid spacing of a point k + tM), delta_mag
 * 0.05 (| |z| - 1 | bound). */
typedef struct sft_params {
    int64_t n;          /* N: signal length, power of two >= 2 */
    int64_t k;          /* K: sparsity, 1 <= K <= N */
    int64_t m;          /* M = N/d: downsampled length, power of two dividing N; 0 = auto */
    int32_t l;          /* L = a_m: maximum collisions decoded per bin, 1..4; 0 = 4 */
    int32_t r;          /* R: random shifts of the CS step (general mode), 1..64, <= d; 0 = min(3L, d) */
    int32_t in_dtype;   /* SFT_C64 or SFT_C128 */
    int32_t mode;       /* SFT_MODE_EXACT or SFT_MODE_GENERAL */
    uint32_t flags;     /* SFT_FLAG_* */
    uint32_t reserved;  /* must be 0 */
    uint64_t seed;      /* seed of the random shifts n_j (general mode) */
    double tau_zero, tau_rank, tau_res, tau_amp, c_res, delta_grid, delta_mag;
    double target_recovery;  /* SFT_FLAG_AUTOTUNE: expected fraction of the K frequencies
                                recovered, in (0, 1); 0 = 0.999 */
} sft_params;

/* A sparse output list.  loc_dev: int64[capacity] locations in [0, N), sorted
 * ascending; val_dev: complex128 (two doubles) [capacity] values x_hat[loc];
 * count_dev: one int64, set to the number of entries found.  When count >
 * capacity only the `capacity` smallest locations (general mode: of the kept
 * K) are written. */
typedef struct sft_sparse_out {
    int64_t* loc_dev;
    void* val_dev;
    int64_t capacity;
    int64_t* count_dev;
} sft_sparse_out;

/* Totals over the signals of one call (filled only when requested). */
typedef struct sft_stats {
    int64_t active_bins;        /* bins that passed the activity test / got votes (iterative:
                                   bin decodes summed over the iterations) */
    int64_t flagged_bins;       /* bins no order up to L explained (iterative: bins whose
                                   decode failed in the last iteration) */
    int64_t cs_bins;            /* flagged bins recovered by pruning + SP (general mode) */
    int64_t mlp_fallbacks;      /* learned mode: bins where the predicted order was rejected */
    int64_t entries;            /* entries found (sum of counts) */
    int64_t overflowed;         /* signals whose count exceeded the capacity */
    int64_t nonfinite;          /* non-finite gathered samples (SFT_FLAG_CHECK_FINITE) */
    double stage_ms[4];         /* gather+FFT, order estimate/vote, decode, output (HIP events);
                                   iterative: gather+FFT, iteration 0, iterations 1.., output */
    double gather_ms[2];        /* the gather+FFT stage in two parts (HIP events): every line but
                                   general mode's random shifts n_j, then those (0 without them);
                                   -1 in both stage fields when not timed */
} sft_stats;

/* What a plan chose for one signal; the oracle consumes exactly these. */
typedef struct sft_plan_info {
    int64_t n, k, m, d;
    int32_t l, r, in_dtype, mode;
    uint32_t flags;
    int32_t n_signals;          /* signals in the plan */
    int64_t rshifts[SFT_MAX_RSHIFTS];   /* n_0 .. n_{R-1}, distinct, in [0, d), ascending */
    double tau_zero, tau_rank, tau_res, tau_amp, c_res, delta_grid, delta_mag;
    int64_t workspace_bytes;    /* device bytes owned by the plan */
} sft_plan_info;

typedef struct sft_plan_s* sft_plan_t;
typedef struct sft_mlp_s* sft_mlp_t;

/* Create a plan for n_params signals (1: single-signal plan for sft_exact /
 * sft_general; >1: batch plan for sft_batch; signals may differ in every
 * field).  hip_stream: a hipStream_t (NULL = default stream) on the current
 * device.  Validates parameters, chooses M and L where 0 (autotuner for
 * batch plans), draws the random shifts from the seed, allocates the
 * workspace and tables.  Errors: SFT_E_INVALID, SFT_E_UNSUPPORTED, SFT_E_NOMEM,
 * SFT_E_DEVICE; *out is NULL on failure. */
sft_status sft_plan(sft_plan_t* out, const sft_params* params, int64_t n_params, void* hip_stream);

/* Exactly K-sparse recovery of one signal (Sec. II, non-iterative).
 * x_dev: N elements of the plan's in_dtype.  Requires a single-signal plan
 * in SFT_MODE_EXACT.  stats may be NULL (then the call is asynchronous). */
sft_status sft_exact(sft_plan_t plan, const void* x_dev, const sft_sparse_out* out, sft_stats* stats);

/* Iterative sFFT-DT (Alg. 1) for one exactly K-sparse signal: x_dev holds N
 * elements of the plan's in_dtype; requires a single-signal plan in
 * SFT_MODE_ITERATIVE.  Output, stats and stream semantics as sft_exact. */
sft_status sft_iterative(sft_plan_t plan, const void* x_dev, const sft_sparse_out* out, sft_stats* stats);

/* Exactly sparse recovery when K is unknown (Sec. II-G): the plan (single
 * signal, SFT_MODE_EXACT, SFT_FLAG_UNKNOWN_K) holds one workspace per rung
 * M = max(1, N / 2^22), .., 2, 4, .., m (d = N / M from N down).  Rungs run in
 * order, each as sft_exact with stats (so the call is synchronous), until one
 * flags no bin; its list is in out and its M in *m_chosen (the last rung's
 * when every rung flags a bin; stats then show flagged_bins > 0).  Errors as
 * sft_exact; SFT_E_CAPACITY only when the chosen rung's list does not fit. */
sft_status sft_unknown_k(sft_plan_t plan, const void* x_dev, const sft_sparse_out* out, sft_stats* stats,
                         int64_t* m_chosen);

/* Generally K-sparse recovery of one signal (Sec. III): syndrome decoding with
 * the K-vote, pruning + Subspace Pursuit on flagged bins, the K largest kept.
 * Requires a single-signal plan in SFT_MODE_GENERAL. */
sft_status sft_general(sft_plan_t plan, const void* x_dev, const sft_sparse_out* out, sft_stats* stats);

/* All signals of a batch plan in one stream-ordered launch sequence captured
 * in a HIP graph (instantiated on the first call).  x_devs: host array of
 * n_signals device pointers; outs: host array of n_signals output lists.
 * Each signal runs in its own mode. */
sft_status sft_batch(sft_plan_t plan, const void* const* x_devs, const sft_sparse_out* outs, sft_stats* stats);

/* Steps 1-2 alone for a single-signal plan: the syndromes
 * m_l[k] = d * FFT_M(x[(d k' + l) mod N])[k] (Sec. II-A, Eq. (2); Alg. 1 and
 * Alg. 2 Part 1) for the plan's S = 2L (+ R) shifts, written to out_dev as
 * [S][M] interleaved complex (float for SFT_C64 input, double for SFT_C128),
 * shift-major; shift s is l = s for s < 2L and n_{s-2L} after that.  Same
 * stream semantics as sft_exact (asynchronous).  Iterative plans write the
 * FFTs Alg. 1 takes: for l = 0 .. L-1 the shifts 2l and 2l + 1 on the grid of
 * M_0 / 2^l bins, [l][2][M_0 / 2^l] concatenated (2 (2 M_0 - M_0 / 2^(L-1))
 * values). */
sft_status sft_syndromes(sft_plan_t plan, const void* x_dev, void* out_dev);

/* ---------------------------------------------------------------------------
 * Learned order predictor (a project addition).  An MLP maps an active bin to
 * its number of aliased frequencies 0..4, replacing the rank test of the order
 * estimate in SFT_MODE_EXACT plans with L = 4 and SFT_FLAG_LEARNED; the rank
 * test remains the fallback and the residual check the judge, so the output
 * is that of the plain method (paper analogue: the order estimate of Sec.
 * III-C, Pruning Step 1).
 *
 * Features of a bin (32 floats): with mt_l the de-rotated syndromes
 * e^{-i 2 pi k l / N} m_l (l < 8), E = sum |mt_l|^2, rms = sqrt(E / 8) and
 * u_l = mt_l conj(mt_0) / (|mt_0| rms): [Re u_0, Im u_0, ..., Re u_7, Im u_7,
 * |mt_0| / rms, ..., |mt_7| / rms, log(E / mean bin energy), 0 x 7].
 * Network: h1 = gelu(W1 f + b1) (128), h2 = gelu(W2 h1 + b2) (128),
 * logits = W3 h2 + b3 (5); gelu(x) = x Phi(x).  Parameters: FP32 vector
 * [W1 (128 x 32), b1, W2 (128 x 128), b2, W3 (5 x 128), b3], row-major,
 * SFT_MLP_PARAMS values; the device computes with BF16 copies of W1..W3 and
 * FP32 accumulation (MFMA).  Training minimises the mean cross-entropy with
 * Adam (beta 0.9 / 0.999, eps 1e-8) on the FP32 master weights.
 * ------------------------------------------------------------------------- */
#define SFT_MLP_FEATURES 32
#define SFT_MLP_CLASSES 5
#define SFT_MLP_PARAMS 21381

/* New predictor with He-uniform weights drawn from `seed`, zero biases.
 * Calls on it are ordered on hip_stream (NULL = default stream). */
sft_status sft_mlp_create(sft_mlp_t* out, uint64_t seed, void* hip_stream);
void sft_mlp_destroy(sft_mlp_t mlp);
/* Copy the FP32 master parameters out / in (host arrays of n = SFT_MLP_PARAMS;
 * set also resets the Adam state).  Both synchronise the predictor's stream. */
sft_status sft_mlp_get_params(sft_mlp_t mlp, float* host, int64_t n);
sft_status sft_mlp_set_params(sft_mlp_t mlp, const float* host, int64_t n);
/* logits_dev[rows][5] for feat_dev[rows][32] (device, FP32). */
sft_status sft_mlp_forward(sft_mlp_t mlp, const float* feat_dev, int64_t rows, float* logits_dev);
/* Gradient of the mean cross-entropy (labels_dev[rows] in 0..4) with respect
 * to the parameters, into grad_dev[SFT_MLP_PARAMS], and the loss into
 * loss_dev[0]; no update. */
sft_status sft_mlp_grad(sft_mlp_t mlp, const float* feat_dev, const int32_t* labels_dev, int64_t rows,
                        float* grad_dev, float* loss_dev);
/* One Adam step with learning rate lr on the mean cross-entropy of the rows;
 * the loss before the step goes to loss_dev[0] (may be NULL). */
sft_status sft_mlp_train_step(sft_mlp_t mlp, const float* feat_dev, const int32_t* labels_dev, int64_t rows,
                              float lr, float* loss_dev);
const char* sft_mlp_last_error(void);

/* Use `mlp` (or NULL to detach) for the plan's SFT_FLAG_LEARNED signals.  The
 * predictor must outlive the plan's use of it. */
sft_status sft_plan_attach_mlp(sft_plan_t plan, sft_mlp_t mlp);

/* Features of the active bins of x (single-signal SFT_MODE_EXACT plan, L = 4):
 * feat_dev[capacity][32] (FP32), bins_dev[capacity] (bin index k), and the
 * number of active bins into count_dev[0] (entries beyond capacity are not
 * written).  Rows come in no particular order.  Asynchronous. */
sft_status sft_features(sft_plan_t plan, const void* x_dev, float* feat_dev, int64_t* bins_dev, int64_t capacity,
                        int64_t* count_dev);

/* Choice of M and L for an exact-mode signal of length n with k frequencies
 * (host only, no device needed; what SFT_FLAG_AUTOTUNE plans use).
 *
 * Model: a frequency is recovered when its bin holds at most L of the K
 * frequencies (the decoder is exact there, the non-iterative case of Sec. II,
 * with the aliasing probabilities of Theorem 1 and Lemma 2); the number of
 * other frequencies in its bin is hypergeometric (K - 1 drawn from the N - 1
 * other positions, d - 1 of which share the bin).
 * Among L = 1..4 and M = N/d (power of two, 2L <= d, M within the supported
 * range) it returns the pair of least modelled device time whose expected
 * recovery reaches `target` (0 = 0.999), or, when none does, the pair of
 * highest expected recovery.  The time model (gather + FFT per line sample,
 * decoder per active and per aliased bin) carries constants measured on
 * MI355X.  expected_recovery and model_us (nullable) receive the chosen
 * pair's figures.  SFT_E_INVALID for n not a power of two >= 2, k outside
 * 1..n, in_dtype not SFT_C64/SFT_C128 or target outside [0, 1). */
sft_status sft_autotune(int64_t n, int64_t k, int32_t in_dtype, double target, int64_t* m_out, int32_t* l_out,
                        double* expected_recovery, double* model_us);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sft_exact
 * for one signal without a plan.  params as for sft_plan (SFT_MODE_EXACT;
 * SFT_FLAG_FFT64 and SFT_FLAG_AUTOTUNE allowed; LEARNED, SYNC, CHECK_FINITE and
 * UNKNOWN_K refused with SFT_E_UNSUPPORTED); x_dev, out as for sft_exact;
 * hip_stream: a hipStream_t of the current device (NULL = default stream).
 *
 * The workspace is one static device array of about 4.5 MiB that the library
 * holds on every GPU it runs on until the process ends.  Limits: M at most
 * 8192 with FP32 FFTs (complex64 input) or 4096 with FP64 FFTs (complex128
 * input or SFT_FLAG_FFT64), d = N/M at most 2^16; larger problems return
 * SFT_E_UNSUPPORTED with the limit in sft_last_error().  The call issues
 * kernels only (no allocation, free, memset or copy), asynchronously: no
 * stats, and no SFT_E_CAPACITY (count_dev receives the number of entries
 * found; only `capacity` of them are written).  The first call on a device
 * also enqueues the fill of the twiddle and unit-root tables (and so does
 * every call under stream capture until an eager call has).  All calls on a
 * GPU share its array: the caller orders them (one stream, or
 * synchronisation between streams); calls that overlap race.  The output
 * equals sft_exact's for the same parameters and input (same kernels and
 * decisions; the tables are computed on the device, so values may differ in
 * the last bits). */
sft_status sft_exact_noalloc(const sft_params* params, const void* x_dev, const sft_sparse_out* out, void* hip_stream);

/* Parameters the plan chose for signal `index` (0-based). */
sft_status sft_plan_get(sft_plan_t plan, int64_t index, sft_plan_info* info);

/* Release a plan (waits for its stream).  NULL is ignored. */
void sft_destroy(sft_plan_t plan);

const char* sft_status_str(sft_status s);
const char* sft_last_error(void);
int32_t sft_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SFT_H */
