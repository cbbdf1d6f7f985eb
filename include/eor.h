/*
 * eor.h - C ABI of the batched FP64 marginal likelihood of the 21-cm power
 * spectrum for one AMD MI355X (gfx950).
 *
 * The problem (Summary and Statement of need; eq. 1 for the k-bins): data
 * d = T a + e with a dense complex instrument/model matrix T (m x n) over the
 * joint EoR + foreground coefficients, a ~ CN(0, Phi(theta)), e ~ CN(0, N),
 * N = diag(sigma^2). The sky coefficients are marginalised analytically, so
 * only theta, the log10 power per spherical k-bin, is sampled. Per theta:
 *
 *   Phi_jj  = s_b 10^theta_b  if coefficient j lies in k-bin b (eq. 1: every
 *             voxel of a shell shares the bin's power), else a fixed variance
 *   Sigma   = A + Phi^{-1},  A = T^H N^{-1} T,  dbar = T^H N^{-1} d
 *   logL    = -m ln(pi) - sum ln sigma_i^2 - ln det Phi - ln det Sigma
 *             - (d^H N^{-1} d - dbar^H Sigma^{-1} dbar)
 *
 * which equals ln CN(d; 0, N + T Phi T^H) exactly (Woodbury identity and
 * matrix-determinant lemma). Complex Gaussians are circular: E[a a^H] = Phi,
 * E[e e^H] = N, with no factors of 1/2.
 *
 * Conventions of every entry point:
 *  - Complex numbers are complex128, interleaved (re, im) doubles.
 *  - "device" pointers are HIP device memory on the context's device;
 *    "host" pointers are ordinary host memory. The caller owns every buffer it
 *    passes; the library copies what it keeps.
 *  - `stream` is a hipStream_t (NULL = the null stream). Calls are
 *    asynchronous on that stream unless stated; results are valid once the
 *    stream has reached the call.
 *  - Argument errors are found before any launch and returned as a negative
 *    eor_status; eor_last_error() then holds a message (thread-local).
 *    Numerical failures are reported per theta through `info` and never stop
 *    the batch. Nothing throws or aborts across the ABI.
 *  - A context is not thread-safe: use one per host thread.
 *  - Every call on one handle (context, group or surrogate) uses the handle's
 *    device buffers (A, the task counter, the per-theta workspace, the
 *    activations). Calls on one handle may go to different streams: a call
 *    on a stream other than the previous call's first makes its stream wait
 *    for the previous call's work (hipStreamWaitEvent), and a call that
 *    reallocates or rewrites such a buffer first waits on the host until the
 *    previous call's work has finished. The calls of one handle therefore
 *    run one after another whatever their streams; work meant to overlap
 *    needs one handle per stream. A group call also waits for, and is then
 *    waited for by, the last call on each of its contexts.
 */
#ifndef EOR_H
#define EOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eor_ctx eor_ctx;
typedef struct eor_group eor_group;
typedef struct eor_surrogate eor_surrogate;

typedef enum {
    EOR_OK = 0,
    EOR_ERR_ARG = -1,   /* a bad argument; nothing was launched */
    EOR_ERR_OOM = -2,   /* device memory could not be allocated */
    EOR_ERR_HIP = -3,   /* a HIP runtime call failed */
    EOR_ERR_STATE = -4  /* call out of order (e.g. loglike before precompute) */
} eor_status;

typedef enum {
    EOR_PREC_FP64 = 0,    /* A formed in FP64 on FP64 MFMA */
    EOR_PREC_FP32 = 1,    /* W = T/sigma rounded to complex64, FP32 MFMA, FP32
                             accumulation per k-chunk, chunks summed in FP64 */
    EOR_PREC_BF16X3 = 2,  /* W split into three bf16 terms, the six leading
                             cross products on bf16 MFMA with FP32
                             accumulation per k-chunk, chunks summed in FP64 */
    EOR_PREC_BF16X2 = 3   /* the cheaper split: two bf16 terms and the three
                             leading cross products (about 2^-16 relative per
                             product instead of 2^-24), otherwise as BF16X3 */
} eor_precision;

/* Message of the last failed call on this thread ("" if none). */
const char *eor_last_error(void);

/* Version string of the library build. */
const char *eor_version(void);

/*
 * Create a context bound to HIP device `device`. *out receives the handle.
 * Errors: EOR_ERR_ARG (bad device, NULL out), EOR_ERR_HIP.
 */
eor_status eor_create(int device, eor_ctx **out);

/* Free the context and all device memory it owns. NULL is a no-op. Waits for
 * the device to finish the context's work first. */
void eor_destroy(eor_ctx *ctx);

/*
 * Once-per-dataset precompute: A = T^H N^{-1} T (stored in FP64 whatever
 * `prec`), dbar = T^H N^{-1} d, c = d^H N^{-1} d and the constant terms of
 * logL.
 *   m, n       rows and columns of T (1 <= m <= 2^28, 1 <= n <= 65536)
 *   T          device, complex128, row-major m x n with row stride
 *              n <= ldT <= 2^24
 *   noise_var  device [m], sigma_i^2; must be > 0 (not checked on the device)
 *   d          device complex128 [m]
 *   n_k        number of k-bins (>= 0)
 *   bin_of     host int32 [n]: k-bin of each coefficient, or -1 for a
 *              fixed-variance (foreground) coefficient
 *   fixed_var  host double [n]: prior variance where bin_of < 0 (> 0);
 *              other entries are ignored. May be NULL if no bin_of is -1.
 *   bin_scale  host double [n_k]: s_b > 0, or NULL for all ones
 *   prec       precision of the A product (eor_precision)
 * T and d may be freed once the stream has passed this call.
 * Errors: EOR_ERR_ARG, EOR_ERR_OOM, EOR_ERR_HIP.
 */
eor_status eor_precompute(eor_ctx *ctx, int64_t m, int64_t n, const void *T, int64_t ldT,
                          const double *noise_var, const void *d, int32_t n_k,
                          const int32_t *bin_of, const double *fixed_var,
                          const double *bin_scale, eor_precision prec, void *stream);

/*
 * logL for a batch of theta: assemble Sigma(theta), factor it (blocked
 * complex Cholesky), solve for the quadratic form, reduce the
 * log-determinants and combine, for every theta of the batch in one launch.
 *   theta  device double [B x n_k], row-major
 *   logL   device double [B]
 *   info   device int32 [B] or NULL: 0 ok; -1 a non-finite theta or prior
 *          variance; k > 0 the 1-based column whose Cholesky pivot was not
 *          positive and finite (LAPACK xPOTRF convention). logL = -inf
 *          whenever info != 0.
 * B = 0 is a no-op. Per-theta workspace is allocated on first use and kept;
 * the call is then asynchronous.
 * Errors: EOR_ERR_ARG, EOR_ERR_STATE (no precompute), EOR_ERR_OOM, EOR_ERR_HIP.
 */
eor_status eor_loglike_batch(eor_ctx *ctx, int64_t B, const double *theta, double *logL,
                             int32_t *info, void *stream);

/*
 * Same as eor_loglike_batch and also writes, per theta, the terms of logL:
 *   terms  device double [B x 4]: ln det Sigma, dbar^H Sigma^{-1} dbar,
 *          ln det Phi, c = d^H N^{-1} d.
 */
eor_status eor_loglike_terms(eor_ctx *ctx, int64_t B, const double *theta, double *logL,
                             int32_t *info, double *terms, void *stream);

/*
 * Copy the precomputed products out, for checking.
 *   A_out      device complex128 [n x n] row-major, full Hermitian (ldA >= n)
 *   dbar_out   device complex128 [n] or NULL
 *   scalars    host double [2] or NULL: c, K0 = -m ln(pi) - sum ln sigma_i^2
 *              (synchronises the stream when not NULL)
 */
eor_status eor_export_precompute(eor_ctx *ctx, void *A_out, int64_t ldA, void *dbar_out,
                                 double *scalars, void *stream);

/* Problem sizes of a context after eor_precompute: m, n, n_k (any may be NULL). */
eor_status eor_shape(const eor_ctx *ctx, int64_t *m, int64_t *n, int32_t *n_k);

/*
 * Device-memory budget of the per-theta workspace of eor_loglike_batch and
 * eor_loglike_terms ("Running BayesEoR" sizes an analysis by the memory it
 * needs; this bounds what the batched likelihood adds to it). Each theta
 * in flight needs one slot of 16 n_pad^2 / 2 + 16 n_pad bytes, n_pad = n
 * rounded up to 64 (the packed tiles of L and the solve vector): about 136 MB
 * at n = 4096. With a budget, a call keeps at most floor(bytes / slot) theta
 * in flight (fewer workgroups, the same results); a budget below one slot
 * makes the next call return EOR_ERR_OOM before any launch.
 *   bytes  0 = no budget (the default: one slot per resident workgroup, as
 *          many as the device holds)
 * A workspace already allocated beyond the new budget is freed once the
 * context's queued work has finished. Errors: EOR_ERR_ARG (NULL ctx),
 * EOR_ERR_HIP.
 */
eor_status eor_set_workspace_limit(eor_ctx *ctx, size_t bytes);

/*
 * Launch choices of this context's eor_loglike_batch / eor_loglike_terms
 * (execution parameters only; results do not depend on them beyond the
 * summation order of the tile updates, which is the same for all):
 *   stages          k-steps of 4 columns the panel update prefetches (2 or 4)
 *   wg_per_cu       theta in flight per compute unit (1 or 2)
 *   tiles_per_pass  1: workgroups of 4 waves; 2: workgroups of 8 waves,
 *                   which then need wg_per_cu = 1. With 64-wide tiles (see
 *                   eor_set_tile_size) that is 1 or 2 tiles of a column
 *                   updated per pass over its panel, with 32-wide tiles 2 or 4.
 * Default: 4, 1, 2. Errors: EOR_ERR_ARG for any other combination.
 */
eor_status eor_set_tuning(eor_ctx *ctx, int32_t stages, int32_t wg_per_cu, int32_t tiles_per_pass);
eor_status eor_get_tuning(const eor_ctx *ctx, int32_t *stages, int32_t *wg_per_cu, int32_t *tiles_per_pass);

/*
 * Side of the square tiles in which this context's eor_loglike_batch /
 * eor_loglike_terms factor Sigma (the blocked Cholesky that the "Running
 * BayesEoR" footnote puts on the GPU): 64 (default) or 32. Smaller tiles make
 * the serial factorisation of each diagonal tile cheaper and the panel
 * updates less efficient; small n gains, large n loses. A stays in 64-wide
 * storage tiles either way. The results differ between the two sides only by
 * the summation order of the tile updates (far inside the parity tolerance).
 * Errors: EOR_ERR_ARG (NULL ctx or argument, a side other than 32 or 64).
 */
eor_status eor_set_tile_size(eor_ctx *ctx, int32_t ts);
eor_status eor_get_tile_size(const eor_ctx *ctx, int32_t *ts);

/*
 * Groups: many datasets of uneven size (e.g. independent frequency
 * sub-bands, each with its own T, noise, data and bins) evaluated together.
 * One eor_group_loglike call is one persistent launch: a fixed set of
 * resident workgroups takes (instance, theta) tasks, longest first, until all
 * are done, so small and large problems share the GPU without a tail per
 * dataset.
 *
 * eor_group_create: n_inst (1..64) contexts on one device, each precomputed
 * before every eor_group_loglike call. The group keeps pointers to the
 * contexts (they must outlive it) and owns its own workspace.
 * Errors: EOR_ERR_ARG, EOR_ERR_OOM, EOR_ERR_HIP.
 */
eor_status eor_group_create(int32_t n_inst, eor_ctx *const *insts, eor_group **out);

/* Free a group (not its contexts). NULL is a no-op. */
void eor_group_destroy(eor_group *g);

/*
 * logL for every instance: B, theta, logL and info are host arrays of length
 * n_inst; theta[i] is a device double [B[i] x n_k(i)], logL[i] a device
 * double [B[i]], info NULL or info[i] a device int32 [B[i]] (or NULL), with
 * the meaning of eor_loglike_batch. The launch is captured once into a HIP
 * graph and replayed while the sizes and pointers stay the same (see
 * eor_group_set_graph). Synchronises the stream before it starts (the
 * per-call descriptors are staged in pinned memory).
 * Errors: EOR_ERR_ARG, EOR_ERR_STATE (an instance without precompute),
 * EOR_ERR_OOM, EOR_ERR_HIP.
 */
eor_status eor_group_loglike(eor_group *g, const int64_t *B, const double *const *theta,
                             double *const *logL, int32_t *const *info, void *stream);

/* Enable (default) or disable graph capture and replay for this group. */
eor_status eor_group_set_graph(eor_group *g, int32_t enable);

/* Set the group's launch choices (meaning and limits as eor_set_tuning). */
eor_status eor_group_set_tuning(eor_group *g, int32_t stages, int32_t wg_per_cu, int32_t tiles_per_pass);

/*
 * Tile side (32 or 64, as eor_set_tile_size) per size bucket of an instance's
 * n: ts_per_bucket[5] for n <= 512, <= 1024, <= 2048, <= 4096 and larger. One
 * launch mixes instances of either side. Default: 64 for every bucket.
 * Errors: EOR_ERR_ARG (NULL argument, a side other than 32 or 64).
 */
eor_status eor_group_set_tile_sizes(eor_group *g, const int32_t *ts_per_bucket);
eor_status eor_group_tile_sizes(const eor_group *g, int32_t *ts_per_bucket);

/* Current launch choices of the group, and how many times it launched a
 * graph and captured one so far (any output may be NULL). */
eor_status eor_group_tuning(const eor_group *g, int32_t *stages, int32_t *wg_per_cu,
                            int32_t *tiles_per_pass, int64_t *graph_launches,
                            int64_t *graph_captures);

/*
 * Autotuner: times the group on the given batch (same arguments as
 * eor_group_loglike, outputs discarded) for every candidate launch shape
 * (panel prefetch depth 2 or 4 k-steps x {workgroups of 4 waves with 1 or 2
 * theta in flight per CU, of 8 waves with 1}) and keeps the fastest; then, for
 * each size bucket of n the batch holds, times that bucket's instances alone
 * with 64- and 32-wide factorisation tiles and keeps the faster side for the
 * bucket (eor_group_set_tile_sizes). With cache_path (may be NULL), the
 * choices are stored in a JSON file keyed by "<gfx arch>|<size bucket of the
 * largest n: n<=512, n<=1024, n<=2048, n<=4096, n>4096>|<single or group>"
 * (the shape) and "<gfx arch>|<bucket>|tile" (the tile side), and existing
 * entries are used without timing unless force != 0. A lone dataset is tuned
 * as a one-instance group. Synchronises the stream.
 * Errors: as eor_group_loglike; EOR_ERR_ARG if the cache cannot be written.
 */
eor_status eor_autotune(eor_group *g, const int64_t *B, const double *const *theta,
                        const char *cache_path, int32_t force, void *stream);

/*
 * Surrogate of logL(theta): an ensemble of n_members fully connected
 * networks n_in -> hidden -> hidden -> 1 with GELU (exact erf form) after
 * each hidden layer, FP32, trained by the library's own forward, backward
 * and Adam kernels on exact evaluations, and used to gate sampler proposals:
 * an ensemble spread above a threshold falls back to the exact likelihood,
 * and every accepted point is judged by the exact likelihood.
 *
 * Parameters of one member, flat FP32, row-major matrices:
 *   W1 [hidden x n_in], b1 [hidden], W2 [hidden x hidden], b2 [hidden],
 *   W3 [hidden], b3 [1]; members follow one another.
 * Inputs: theta mapped from the prior box [lo, hi] to [-1, 1]. Targets:
 * logL standardised by the training mean and standard deviation. Ensemble
 * mean and spread are reported in logL units; the spread is the population
 * standard deviation (ddof = 0) over the members.
 */
typedef struct {
    int32_t epochs;     /* maximum number of epochs */
    int32_t minibatch;  /* samples per Adam step */
    int32_t patience;   /* epochs without a better validation loss before a member stops improving */
    float lr, beta1, beta2, eps;  /* Adam */
    float val_frac;     /* fraction held out for validation, in [0, 0.9) */
    uint64_t seed;      /* split, bootstrap resamples and epoch order */
} eor_train_cfg;

/*
 * Create an ensemble on HIP device `device` with He-normal weights (one
 * seeded stream per member) and zero biases. lo, hi: host double [n_in],
 * hi > lo, the prior box. Sizes: 1 <= n_in <= 64, 1 <= n_members <= 64,
 * hidden a multiple of 4 in [4, 512] (one workgroup keeps a block of samples'
 * activations of both hidden layers in LDS). Anything else: EOR_ERR_ARG.
 */
eor_status eor_surrogate_create(int device, int32_t n_in, int32_t n_members, int32_t hidden,
                                uint64_t seed, const double *lo, const double *hi,
                                eor_surrogate **out);
void eor_surrogate_destroy(eor_surrogate *s);

/* Parameters per member and number of members (either output may be NULL). */
eor_status eor_surrogate_size(const eor_surrogate *s, int64_t *params_per_member,
                              int32_t *n_members);

/*
 * Copy all parameters out (get: device float [n_members x P]) and/or replace
 * them (set: same layout; also clears the Adam moments and step count).
 */
eor_status eor_surrogate_params(eor_surrogate *s, float *get, const float *set, void *stream);

/* Get (host double [2]) and/or set the target standardisation (mean, std). */
eor_status eor_surrogate_standardisation(eor_surrogate *s, double *get_mean_std,
                                         const double *set_mean_std);

/*
 * Train on N exact evaluations: theta device double [N x n_in], logL device
 * double [N] (finite). Each member trains on its own bootstrap resample of
 * the training split with minibatch Adam; after every epoch the validation
 * loss decides each member's best parameters, which are kept. Stops after
 * cfg->epochs or when no member has improved for cfg->patience epochs.
 * Synchronises the stream.
 */
eor_status eor_surrogate_train(eor_surrogate *s, int64_t N, const double *theta, const double *logL,
                               const eor_train_cfg *cfg, void *stream);

/* Epochs run by the last training and each member's best validation loss
 * (host double [n_members], standardised units); either may be NULL. */
eor_status eor_surrogate_report(const eor_surrogate *s, int32_t *epochs_run, double *val_loss);

/*
 * One training step's pieces, exposed for checking: the mean squared error
 * of every member on its own batch (x: device float [n_members x nb x n_in],
 * already scaled; y: device float [n_members x nb], standardised) and its
 * gradient (loss: device float [n_members]; grad: device float
 * [n_members x P]; either may be NULL), and one Adam update of all
 * parameters from the last computed gradient.
 */
eor_status eor_surrogate_loss_grad(eor_surrogate *s, int64_t nb, const float *x, const float *y,
                                   float *loss, float *grad, void *stream);
eor_status eor_surrogate_adam_step(eor_surrogate *s, const eor_train_cfg *cfg, void *stream);

/*
 * Ensemble prediction for B points (theta device double [B x n_in]): mean
 * and spread (device double [B], either may be NULL) in logL units, and
 * optionally each member's standardised output (members: device float
 * [n_members x B]).
 */
eor_status eor_surrogate_infer(eor_surrogate *s, int64_t B, const double *theta, double *mean,
                               double *spread, float *members, void *stream);

/*
 * As eor_surrogate_infer, plus the gate: decision[b] (device int32 [B]) = 0
 * (reject without an exact call) when spread <= tau and mean < L_min,
 * otherwise 1 (evaluate exactly: the surrogate is unsure, or the point may
 * be accepted and must be judged exactly).
 */
eor_status eor_surrogate_gate(eor_surrogate *s, int64_t B, const double *theta, double L_min,
                              double tau, double *mean, double *spread, float *members,
                              int32_t *decision, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * results as eor_surrogate_gate, with the same arguments, from the same
 * kernels, but the members' outputs of the call are kept in a fixed scratch
 * array inside the library instead of a buffer the surrogate grows, so the
 * call allocates nothing (its first call on a device looks up that device's
 * copy of the array; the surrogate must have been trained, or given its
 * standardisation, before).
 * Limit: B * n_members <= 2^22 (16 MiB of FP32 per device, held until the
 * process ends); a larger B returns EOR_ERR_ARG before any launch.
 * Every call on one GPU uses that GPU's one array: calls that overlap on one
 * GPU (from any surrogate, on any stream) race and must be ordered by the
 * caller. Errors: as eor_surrogate_gate, and EOR_ERR_ARG as above.
 */
eor_status eor_surrogate_gate_noalloc(eor_surrogate *s, int64_t B, const double *theta, double L_min,
                                      double tau, double *mean, double *spread, float *members,
                                      int32_t *decision, void *stream);

/*
 * Stable compaction: the rows s of rows (device double [n x n_cols]) with
 * keep[s] != 0 are copied, in order, to rows_out (may be NULL), their
 * indices to index_out (device int32, may be NULL), and their number to
 * *count_out (device int32).
 */
eor_status eor_compact_rows(int64_t n, int32_t n_cols, const int32_t *keep, const double *rows,
                            double *rows_out, int32_t *index_out, int32_t *count_out, void *stream);

/*
 * Out-of-core likelihood, for Sigma too large for the device (the case of the
 * paper's MAGMA footnote, running BayesEoR with matrices beyond the GPU's
 * memory): the same logL as eor_loglike_batch, with A in host memory and each
 * theta's factor L kept in a pinned host buffer of the library, while the
 * device holds a pass of tile columns (64 x 64 tiles) and a window of
 * earlier columns (blocked Cholesky in passes of tile columns: left-looking
 * across passes, right-looking inside one; FP64 MFMA tile products).
 * Up to four theta are factored at once ("lanes"), each on its own stream
 * with its own share of the device memory and its own pinned host factor.
 *   A        host complex128 [n x ldA] row-major, Hermitian; only the lower
 *            triangle is read (eor_export_precompute writes it)
 *   dbar     host complex128 [n];  c, K0: the scalars eor_export_precompute
 *            returns (K0 = -m ln pi - sum ln sigma^2)
 *   n_k, bin_of [n], fixed_var [n], bin_scale [n_k] (or NULL = 1): host, as
 *            for eor_precompute
 *   theta    host double [B x n_k];  logL host double [B];  info host int32
 *            [B] or NULL (0, -1 for an invalid theta, or the 1-based column of
 *            the first non-positive pivot; logL = -inf then); B = 0 returns
 *            EOR_OK after the argument checks (theta and logL may be NULL)
 *   device_bytes: the device memory the call may use, split evenly between
 *            the lanes; each lane needs one column of tiles twice over (about
 *            2 ceil(n/64) x 64 KiB) plus O(n)
 *   lanes    1..4, or 0: as many (at most 4) as leave every lane room for
 *            2 min(ceil(n/64), 8) full-height tile columns and keep the pinned
 *            host buffers (lanes + 1 copies of the packed lower triangle)
 *            within half of the host's physical memory
 * The schedule (lanes, pass width) follows from n, n_k, device_bytes and
 * lanes (with lanes = 0, also from the host's memory), never from B, so a
 * theta's result does not depend on the batch it is in; a different pass
 * width sums the tile products in a different order, so results for
 * different device_bytes or lanes agree to rounding only (pass lanes > 0 for
 * the same bits on hosts of different memory sizes). Synchronous; allocates its device buffers, a pinned packed
 * copy of A and one pinned host factor per lane in use (ceil(n/64)
 * (ceil(n/64) + 1) / 2 tiles each), and frees them before returning.
 * Errors: EOR_ERR_ARG (sizes, NULL arrays, bin_of out of range, fixed
 * variance not positive, lanes outside 0..4), EOR_ERR_OOM (device_bytes too
 * small for the lanes, allocation), EOR_ERR_HIP.
 */
eor_status eor_loglike_host(int device, int64_t n, const double *A, int64_t ldA, const double *dbar,
                            double c, double K0, int32_t n_k, const int32_t *bin_of,
                            const double *fixed_var, const double *bin_scale, int64_t B,
                            const double *theta, size_t device_bytes, int32_t lanes, double *logL,
                            int32_t *info);

/*
 * The schedule eor_loglike_host follows for these arguments, without running
 * it (host only, no device call): lanes_out, the tile columns per pass
 * (cols_per_pass), the tiles of a lane's window of earlier columns
 * (window_tiles) and the host <-> device bytes per theta (link_bytes: A
 * once, the rows of every earlier tile column below a pass once per pass, and
 * the part of each pass's columns that later passes read, written back once).
 * Any output pointer may be NULL. Errors as eor_loglike_host's
 * for the same arguments (EOR_ERR_ARG, EOR_ERR_OOM).
 */
eor_status eor_loglike_host_plan(int64_t n, int32_t n_k, size_t device_bytes, int32_t lanes,
                                 int32_t *lanes_out, int64_t *cols_per_pass, int64_t *window_tiles,
                                 int64_t *link_bytes);

/*
 * Instrument forward model (the step before the likelihood, from the
 * instrument model of the paper's "Running BayesEoR" section: a primary-beam
 * response and the uv sampling of the data). The paper names the inputs but
 * prints no formula; this is the visibility equation on a pixelised sky
 * with the sky expanded in the model's basis of 2-D Fourier cells (u_k, v_k)
 * times spectral modes Z[f][e]:
 *
 *   T[f n_bl + b][e n_uv + k] = norm Z[f][e] sum_p A[f][p]
 *       exp(-2 pi i nu_f / c (x_b l_p + y_b m_p)) exp(2 pi i (u_k l_p + v_k m_p))
 *
 * c = 299792458 m/s. All arrays are device memory, row-major:
 *   freq [n_freq] Hz; bl [n_bl x 2] baseline (x_b, y_b) in metres;
 *   lm [n_pix x 2] pixel direction cosines; beam [n_freq x n_pix] real
 *   response A; uv [n_uv x 2] model cells in wavelengths; Z [n_freq x n_eta]
 *   complex (interleaved re, im); norm: finite scalar.
 *   T out: complex [n_freq n_bl] rows with leading dimension ldT >= n_eta n_uv
 *   (complex elements); rows are channel-major, columns spectral-mode-major.
 * Asynchronous on `stream`; stream-ordered scratch of n_pix n_uv complex
 * (the sky modes) and c n_freq n_bl n_uv complex (partial sums of the pixel
 * sum over c <= 16 chunks of the pixels, added in chunk order).
 * Errors: EOR_ERR_ARG (sizes < 1, n_freq > 65535, n_bl > 65535 x 32, n_uv > 65535 x 64,
 * n_eta > 2^20, n_pix n_uv > 2^34, n_freq n_bl n_uv > 2^40, more than
 * 2^31 - 1 tiles of 32 baselines x 128 uv cells x pixel chunks, NULL array,
 * ldT too small, norm not finite), EOR_ERR_HIP, EOR_ERR_OOM.
 */
eor_status eor_forward_model(int64_t n_freq, int64_t n_bl, int64_t n_pix, int64_t n_uv, int64_t n_eta,
                             const double *freq, const double *bl, const double *lm, const double *beam,
                             const double *uv, const double *Z, double norm, double *T, int64_t ldT,
                             void *stream);

/*
 * DIAGNOSTIC, not part of the method: a measuring instrument for the
 * benchmark's roofline report, kept in the library so that it runs with the
 * same build and clock behaviour as the likelihood kernels.
 * Measured FP64 matrix peak (for reporting beside the specification peak):
 * back-to-back FP64 16x16x4 MFMAs on independent accumulators, two
 * workgroups of four waves per CU, `iters` rounds of eight per wave, timed on
 * a private stream after a short warm-up. A run of about the length of a
 * likelihood launch shows the clock the part sustains under that load.
 *   tflops  out: FP64 TFLOP/s;  ms  out (may be NULL): the timed run
 * Synchronous; allocates and frees a small output buffer.
 * Errors: EOR_ERR_ARG (iters outside 1..2^32, NULL tflops), EOR_ERR_HIP, EOR_ERR_OOM.
 */
eor_status eor_probe_fp64_mfma(int device, int64_t iters, double *tflops, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* EOR_H */
