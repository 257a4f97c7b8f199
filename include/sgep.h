/*
 * sgep.h -- C ABI of the MI355X streaming symmetric generalized eigensolver
 * (stochastic gamma-EigenGame, Gemp, Chen, McWilliams, ICLR 2023,
 * arXiv 2206.04993).
 *
 * The library finds the top-k generalized eigenvectors of A v = lambda B v
 * (A symmetric, B symmetric positive definite; Sec. 1) from a stream of
 * minibatches, by the k-player update of Alg. 2 (M = 1 machine per player:
 * one GPU sees the whole minibatch).  A and B are never formed: each step only
 * needs products of the minibatch with the players' vectors (Sec. 1, App. I).
 *
 * Problem kinds (Sec. 1):
 *   SGEP_KIND_CCA      paired views x (dx) and y (dy), d = dx + dy,
 *                      A = [[0, E xy^T], [E yx^T, 0]], B = diag(E xx^T, E yy^T)
 *   SGEP_KIND_GENERAL  two streams of width d: A = E[y y^T], B = E[x x^T] + eps I
 *   SGEP_KIND_LDA      labelled samples x (width d) of n_classes classes with
 *                      given class means mu_c and priors pi_c:
 *                      A = sum_c pi_c (mu_c - mu)(mu_c - mu)^T, mu = sum_c pi_c mu_c
 *                      (between-class), B = E[(x - mu_l)(x - mu_l)^T] + eps I
 *                      (within-class, l the sample's label)
 *   SGEP_KIND_ICA      one stream x of width d, the kurtosis form of ICA:
 *                      A = E[<x, x> x x^T] - tr(C) C - 2 C^2, B = C + eps I,
 *                      C = E[x x^T] (F64 / F32 single handles)
 * Expectations are estimated by minibatch means (1/b) sum over the rows (ICA:
 * every term, C^2 included, from the one minibatch); the data are taken as
 * zero-mean (Sec. 1) unless cfg.center asks for running-mean centring.
 *
 * Conventions
 *   - Every call returns an sgep_status; 0 is success.
 *   - Argument and shape errors are returned synchronously and leave the
 *     handle unchanged.
 *   - Device faults detected inside a step (non-finite Gram terms or norms:
 *     SGEP_ENONFINITE; an LDA label outside [0, n_classes): SGEP_ELABEL; a
 *     workgroup that gave up its bounded wait for data another workgroup of
 *     the same launch publishes: SGEP_EDEVICE) are latched in a device status
 *     word and reported by the next call that synchronises (sgep_eigvals,
 *     sgep_vectors, sgep_auxiliary, sgep_get_state, sgep_sync).  The handle is then POISONED: every later
 *     call except sgep_set_state and sgep_destroy returns SGEP_EPOISONED.
 *   - Host arrays of player vectors are d x k COLUMN-major doubles: column i
 *     (elements i*d .. i*d+d-1) is player i.
 *   - Minibatch views are device arrays, ROW-major (one sample per row) with a
 *     leading dimension in elements; they are borrowed, never copied or
 *     retained beyond the work the call enqueues on the handle's stream.
 *   - sgep_step never synchronises the host, allocates memory or copies to
 *     pageable memory, so a sequence of steps can be captured in a hipGraph;
 *     the step counter t and the step sizes live on the device.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - The library runs on gfx950 only and has no CPU fallback.
 */
#ifndef SGEP_H
#define SGEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sgep_status;
#define SGEP_OK 0
#define SGEP_EINVAL (-1)       /* bad argument value or NULL pointer */
#define SGEP_ESHAPE (-2)       /* inconsistent sizes / leading dimensions / alignment */
#define SGEP_ENOMEM (-3)       /* device allocation failed (init only) */
#define SGEP_EDEVICE (-4)      /* HIP runtime error */
#define SGEP_ENONFINITE (-5)   /* a step produced a non-finite or zero norm / Gram term */
#define SGEP_EUNSUPPORTED (-6) /* valid request the library does not implement */
#define SGEP_EPOISONED (-7)    /* an earlier fault poisoned the handle */
#define SGEP_ELABEL (-8)       /* an LDA step received a label outside [0, n_classes) */

/* problem kinds */
#define SGEP_KIND_CCA 0
#define SGEP_KIND_GENERAL 1
#define SGEP_KIND_LDA 2
#define SGEP_KIND_ICA 3

/* element type of the minibatch views (and of the arithmetic) */
#define SGEP_F64 0     /* FP64 data, FP64 MFMA, FP64 state */
#define SGEP_F32 1     /* FP32 data, FP32 MFMA, FP32 state */
#define SGEP_BF16 2    /* BF16 data, BF16 MFMA with FP32 accumulation, FP32 state */
#define SGEP_FP8_E4M3 3 /* OCP FP8 e4m3 codes with per-column FP32 scales (value =
                         * code * scale), decoded exactly to BF16; as SGEP_BF16 */

/* optimiser applied to the update direction (Alg. 2 uses plain ascent;
 * App. H uses Adam with b1 = 0.9, b2 = 0.999, eps = 1e-8) */
#define SGEP_SGD 0
#define SGEP_ADAM 1

/* step-size schedules for eta_t, t = 1, 2, ...
 *   CONST            eta0
 *   INV              eta0 / (1 + t / t0): square-summable, not summable
 *                    (condition of the convergence theorem, Sec. 3)
 *   WARMUP_HARMONIC  eta0 * t / t_c for t < t_c, then eta0 (t_c + D) / (t + D)
 *                    with D chosen so that eta_T is reached at t = T (App. H) */
#define SGEP_SCHED_CONST 0
#define SGEP_SCHED_INV 1
#define SGEP_SCHED_WARMUP_HARMONIC 2

typedef struct sgep_config {
    int32_t kind;      /* SGEP_KIND_* */
    int32_t dtype;     /* SGEP_F64 (CCA, GENERAL, ICA); SGEP_F32 (CCA, GENERAL, ICA,
                        * LDA); SGEP_BF16 (CCA, LDA); SGEP_FP8_E4M3 (CCA) */
    int32_t k;         /* number of players, 1 <= k <= 64 (F64, and CCA in BF16 or
                        * FP8: k <= 32) */
    int32_t optimizer; /* SGEP_SGD or SGEP_ADAM */
    int32_t schedule;  /* SGEP_SCHED_* */
    int32_t n_classes; /* LDA: 2 .. 16 classes; 0 otherwise */
    int64_t dx;        /* CCA: width of view x. GENERAL, LDA, ICA: d */
    int64_t dy;        /* CCA: width of view y. GENERAL: must equal dx. LDA, ICA: 0.
                        * BF16, FP8 and LDA: dx and dy multiples of 8 */
    int64_t b_max;     /* largest minibatch that sgep_step will receive */
    double eta0, eta_T, t0, t_c, T; /* schedule parameters (see above) */
    double gamma;      /* rate gamma_t (constant) of the auxiliary [Bv] update
                        * and of the Rayleigh-quotient running means, 0 < gamma <= 1 */
    double rho;        /* Alg. 2 clip: <v_j, [Bv]_j> is replaced by max(., rho),
                        * rho >= 0; Alg. 3: the lower end of the estimate, > 0 */
    double eps_reg;    /* GENERAL, LDA: ridge, B = ... + eps_reg I; CCA: must be 0 */
    double adam_b1, adam_b2, adam_eps;
    uint64_t seed;     /* reserved (initial players are always supplied) */
    int32_t smooth;    /* 0: Alg. 2 (parents' <v_j, B v_j> estimated by
                        * max(<v_j, [Bv]_j>, rho)); 1: Alg. 3 (smooth stochastic
                        * variant, App. G: estimated by
                        * exp(log rho + (log nu - log rho) sigmoid(z_j)), with z_j
                        * starting at 0 and moved at rate gamma by
                        * (<v_j, [Bv]_j> - s_j) s_j (log nu - log rho)
                        * sigmoid(z_j) (1 - sigmoid(z_j)) each iteration) */
    int32_t center;    /* 0: the views are taken as zero-mean (Sec. 1); 1: each
                        * minibatch view is centred by a running mean before the
                        * iteration (the mean of the iteration's start), and the
                        * mean then moves toward the minibatch mean at rate gamma
                        * (starting at 0).  F64 / F32 CCA and GENERAL (single
                        * handles and batches), and BF16 / FP8-e4m3 CCA (there
                        * the products are corrected by the rank-one terms, X
                        * itself enters the arithmetic exactly);
                        * SGEP_EUNSUPPORTED elsewhere (LDA, ICA) */
    double nu;         /* Alg. 3: upper bound of lambda_max(B), nu > rho; unused
                        * (any value) with smooth = 0 */
} sgep_config;

typedef struct sgep_handle_s sgep_handle;

/* Create a solver (Alg. 2 initialisation).
 *   out        : receives the handle
 *   cfg        : copied; validated synchronously
 *   V0         : host, d x k column-major, the players' starting points; each
 *                column is normalised to the unit sphere on the device and the
 *                auxiliary variable starts at [Bv]_i = v_i.  Must be non-NULL
 *                with non-zero columns.
 *   hip_stream : hipStream_t on which all device work of this handle runs
 *                (NULL = the null stream); must belong to the current device
 * Device memory owned by the handle: V, [Bv] (d x k each), the Adam moments
 * (2 d x k, Adam only), the projections of one minibatch (2 b_max x k),
 * k x k coefficient blocks and reduction workspaces.  Errors: SGEP_EINVAL,
 * SGEP_ESHAPE, SGEP_EUNSUPPORTED, SGEP_ENOMEM, SGEP_EDEVICE. */
sgep_status sgep_init(sgep_handle **out, const sgep_config *cfg, const double *V0,
                      void *hip_stream);

/* Problem data that some configurations need at initialisation; all host
 * pointers, copied into handle-owned device memory (the caller keeps
 * ownership).  Members a configuration does not use must be NULL. */
typedef struct sgep_init_aux {
    const float *x_col_scale;   /* FP8: dx positive finite scales of view x */
    const float *y_col_scale;   /* FP8: dy positive finite scales of view y */
    const double *class_means;  /* LDA: n_classes x d, row-major (row c = mu_c) */
    const double *class_priors; /* LDA: n_classes positive weights pi_c */
} sgep_init_aux;

/* sgep_init for every configuration: aux may be NULL unless dtype is
 * SGEP_FP8_E4M3 (column scales) or kind is SGEP_KIND_LDA (class means and
 * priors).  The FP8 scales are fixed for the life of the handle, because the
 * next iteration's product operand is prepared at the end of each step.
 * Errors as sgep_init, plus SGEP_EINVAL for missing, extra or non-finite
 * auxiliary data. */
sgep_status sgep_init_ex(sgep_handle **out, const sgep_config *cfg, const double *V0,
                         const sgep_init_aux *aux, void *hip_stream);

/* Enqueue one iteration of Alg. 2 on the minibatch (X, Y) of b rows.
 *   X   : device, b x dx row-major (element type cfg.dtype), leading dim ldx
 *   Y   : device, b x dy row-major, leading dim ldy (ICA: NULL, ldy ignored)
 *   1 <= b <= b_max.  X and Y must be 16-byte aligned and ldx, ldy multiples
 *   of 16 bytes / element size (2 for F64, 4 for F32), ldx >= dx, ldy >= dy.
 * Per iteration, with v_i the current unit players, [Bv]_i the auxiliary
 * variable, A_t and B_t the minibatch estimates:
 *   s_j  = max(<v_j, [Bv]_j>, rho)                                 (Alg. 2)
 *   grad_i = (v_i'B_t v_i) A_t v_i - (v_i'A_t v_i) B_t v_i
 *          - sum_{j<i} (v_i'A_t v_j / s_j) [ (v_i'B_t v_i)[Bv]_j - (v_i'[Bv]_j) B_t v_i ]
 *   v_i  <- (v_i + eta_t grad_i) / ||.||  (or Adam on grad_i, then normalise)
 *   [Bv]_i <- [Bv]_i + gamma (B_t v_i - [Bv]_i)
 * Returns synchronously only argument errors; SGEP_EPOISONED if poisoned. */
sgep_status sgep_step(sgep_handle *h, const void *X, int64_t ldx, const void *Y, int64_t ldy,
                      int64_t b);

/* LDA iteration: X is b x d row-major as in sgep_step, labels a device array
 * of b int32 class indices in [0, n_classes).  A label outside that range
 * poisons the handle (SGEP_ELABEL from the next synchronising call; that
 * iteration's result is unspecified).  X (BF16 or F32) must be 16-byte
 * aligned with ldx a multiple of 8 elements. */
sgep_status sgep_step_lda(sgep_handle *h, const void *X, int64_t ldx, const int32_t *labels,
                          int64_t b);

/* Number of kernels one iteration launches.  F64 / F32: for a CCA handle
 * with b_max >= 512 and at most 128 backward tiles, 2 (forward products, one
 * workgroup per view and row tile; two row slices of the backward products
 * per tile plus the k x k coefficients, the last slice of each tile summing
 * them and running the update), or 3 with centring (the sum of the slices
 * and the update as a third kernel); else 2 (forward products; backward products,
 * k x k coefficients and update) when the backward tile is one 16-feature
 * block and k * element size <= 128 bytes after padding; else 3 (forward
 * products; k x k coefficients; backward products and update), or 4 when
 * ceil(b_max / 16) (k'(k'+1)/2 + k') >= 32768 for k' the padded k (the
 * coefficients' reduction first spread over many workgroups).  ICA: 4
 * (forward products and row norms; X^T P and X^T diag(||x_r||^2) P; the
 * second forward pass X C_t V with the k x k coefficients; X^T X C_t V and
 * update).  BF16 / FP8: 3 (forward products; operand preparation and
 * reductions; backward products and update). */
sgep_status sgep_kernels_per_step(const sgep_handle *h, int32_t *n);

/* Short name of kernel i (0 <= i < sgep_kernels_per_step) of one iteration,
 * in launch order: "k_fwd", "k_fwds", "k_coef", "k_coefa", "k_coefb", "k_bwdp", "k_bwd1", "k_fwd2",
 * "k_bwd", "k_wfwd", "k_wmid"
 * or "k_wbwd" -- a static string, not to be freed; NULL for a NULL handle or
 * an index out of range. */
const char *sgep_step_kernel_name(const sgep_handle *h, int32_t i);

/* One iteration (sgep_step, or sgep_step_lda when labels is non-NULL) with
 * per-kernel timing: events[2 i] and events[2 i + 1] receive the start and end
 * of the execution of kernel i of the iteration, in launch order (timestamps
 * of the kernel's own dispatch, without launch gaps); n_events must be twice
 * sgep_kernels_per_step.  The events are the caller's hipEvent_t objects,
 * created with timing enabled and read with hipEventElapsedTime.  Errors as
 * the plain step, plus SGEP_EINVAL for a NULL event or a wrong n_events.
 * Not for stream capture. */
sgep_status sgep_step_profiled(sgep_handle *h, const void *X, int64_t ldx, const void *Y,
                               int64_t ldy, const int32_t *labels, int64_t b,
                               void *const *events, int32_t n_events);

/* Wait for the handle's stream and report any latched device fault. */
sgep_status sgep_sync(sgep_handle *h);

/* Eigenvalue estimates lambda_i = abar_i / bbar_i, the ratio of running means
 * (rate gamma) of v_i'A_t v_i and v_i'B_t v_i (Rayleigh quotient, Sec. 2).
 * out: host, k doubles.  Synchronises. */
sgep_status sgep_eigvals(sgep_handle *h, double *out);

/* Flags of sgep_vectors. */
#define SGEP_VEC_BNORM 1     /* v_i / sqrt(s_i), the estimate of the B-normalised
                              * eigenvector, instead of the unit v_i */
#define SGEP_VEC_CANONICAL 2 /* sign convention: each column negated if needed so
                              * that its largest-magnitude component (lowest index
                              * on ties) is positive (v and -v solve the same
                              * problem, Sec. 2) */

/* Current players (Alg. 2 output: the unit vectors v_i), with the read-out
 * options of flags (0 or an OR of SGEP_VEC_*).  Without SGEP_VEC_CANONICAL
 * the signs are those of the iterate.  out: host, d x k column-major doubles.
 * Synchronises.  SGEP_EINVAL for unknown flag bits. */
sgep_status sgep_vectors(sgep_handle *h, int32_t flags, double *out);

/* sgep_vectors without any device allocation, for callers that cannot
 * allocate device memory (serving loops and harnesses that forbid it after
 * start-up): the FP64 read-out is staged in a fixed device array of
 * 4,194,304 doubles (32 MiB) that the library holds on every GPU it runs on
 * until the process ends, instead of the handle's own staging buffer.  Same
 * arguments, flags, output and errors as sgep_vectors, plus
 * SGEP_EUNSUPPORTED when d * k exceeds 4,194,304.  Every call on one GPU
 * uses the same array: calls that overlap on one GPU (from several host
 * threads) race and must be serialised by the caller.  Synchronises. */
sgep_status sgep_vectors_noalloc(sgep_handle *h, int32_t flags, double *out);

/* The auxiliary variable [Bv] (host, d x k column-major).  Synchronises. */
sgep_status sgep_auxiliary(sgep_handle *h, double *out);

/* Running means of the views (centring, cfg.center = 1): out receives, on the
 * host, the dx means of view x followed by the dy means of view y (GENERAL:
 * dx and dx).  These are the means the next iteration centres with.
 * Synchronises.  SGEP_EINVAL for a handle without centring. */
sgep_status sgep_means(sgep_handle *h, double *out);

/* Number of completed iterations.  Synchronises. */
sgep_status sgep_step_count(sgep_handle *h, int64_t *t);

/* Checkpoint / resume: size in bytes of the opaque state blob, copy it out
 * (synchronises), and restore it (clears a poisoned status).  The blob holds
 * the iterate, the auxiliary variable, the Adam moments, the running means,
 * the step counter and a hash of the configuration, which must match. */
sgep_status sgep_state_size(const sgep_handle *h, size_t *bytes);
sgep_status sgep_get_state(sgep_handle *h, void *host_buf, size_t bytes);
sgep_status sgep_set_state(sgep_handle *h, const void *host_buf, size_t bytes);

/* Release every resource of the handle (synchronises its stream first). */
sgep_status sgep_destroy(sgep_handle *h);

/* ------------------------------------------------------------------------
 * Batched instances.  Many independent problems of kind GENERAL that share
 * the configuration (k, dtype, optimiser, schedule, hyperparameters, b_max)
 * but not the width d are advanced together: one iteration of Alg. 2 for
 * every instance per sgep_batch_step, enqueued as a short fixed sequence of
 * launches on one stream (capturable in a hipGraph).  Each instance computes
 * exactly what a single handle of width d_i computes; an instance advanced by
 * the batch holds the same bits as the same instance advanced alone with the
 * same feature-tile height.  Not part of the paper, whose parallelism is over
 * players and machines (Sec. 3, App. F): a throughput form for many small
 * problems on one GPU.
 * ------------------------------------------------------------------------ */
typedef struct sgep_batch_s sgep_batch;

/* Create n >= 1 instances (n <= 65535).
 *   d       : host, n widths d_i >= common->k
 *   ld      : host, n leading dimensions ld_i >= d_i (elements) of the rows of
 *             instance i's views; a multiple of 16 bytes / element size
 *             enables 16-byte loads (with 16-byte aligned views)
 *   common  : kind SGEP_KIND_GENERAL, dtype SGEP_F32 or SGEP_F64; dx and dy are
 *             ignored (each instance uses dx = dy = d_i); validated as by
 *             sgep_init for every instance
 *   V0      : host, n pointers to d_i x k column-major starting points
 *   hip_stream : the stream of every instance
 * The initial launch plan is one group with 16-feature backward tiles.
 * Errors: as sgep_init; SGEP_EUNSUPPORTED for another kind or dtype. */
sgep_status sgep_batch_init(sgep_batch **out, int32_t n, const int64_t *d, const int64_t *ld,
                            const sgep_config *common, const double *const *V0,
                            void *hip_stream);

/* Borrowed handle of instance i (0 <= i < n) for the read-out and checkpoint
 * calls (sgep_eigvals, sgep_vectors, sgep_auxiliary, sgep_step_count,
 * sgep_get_state / sgep_set_state, sgep_sync) and for stepping the instance
 * alone with sgep_step.  Never pass it to sgep_destroy. */
sgep_status sgep_batch_instance(sgep_batch *bt, int32_t i, sgep_handle **h);

/* Enqueue one iteration for every instance.
 *   X, Y : DEVICE arrays of n device pointers; instance i reads the b x d_i
 *          row-major views X[i], Y[i] with leading dimension ld_i
 *   1 <= b <= b_max (common to all instances)
 * Returns synchronously only argument errors, and SGEP_EPOISONED when any
 * instance is poisoned.  No allocation, synchronisation or host copy. */
sgep_status sgep_batch_step(sgep_batch *bt, const void *const *X, const void *const *Y,
                            int64_t b);

/* Launches of one batched iteration: *n receives their number; kinds (cap
 * entries, nullable) receives 0 for a forward launch, -1 for a coefficient
 * launch (the k x k terms of each instance, once per iteration), the
 * backward feature-tile height in units of 16 features (1, 2 or 4) for a
 * backward launch, and -2 for the one launch of the persistent plan. */
sgep_status sgep_batch_launches(const sgep_batch *bt, int32_t *n, int32_t *kinds, int32_t cap);

/* sgep_batch_step with a start / end event pair per launch, in launch order
 * (n_events = 2 * the count of sgep_batch_launches), stamped by each kernel's
 * own dispatch.  Not for stream capture. */
sgep_status sgep_batch_step_profiled(sgep_batch *bt, const void *const *X, const void *const *Y,
                                     int64_t b, void *const *events, int32_t n_events);

/* The launch plan: *groups >= 1, the number of instance groups run one after
 * the other (each a forward launch and its backward launches, so that a
 * group's minibatches are re-read from cache), or *groups = -L <= -1, the
 * persistent plan: one launch per iteration whose workgroups claim the
 * items of per-XCC work queues (every instance's forward row tiles, its
 * coefficient block and its backward tiles, in that order, the forward of
 * the next L instances placed before an instance's coefficient item) and
 * wait on per-instance counters (bounded waits; a give-up sets the status
 * reported as SGEP_EDEVICE).  mb_bucket[3] is the backward feature-tile
 * height (units of 16 features) for instances with d <= 256, 256 < d <= 1024
 * and d > 1024. */
sgep_status sgep_batch_plan(const sgep_batch *bt, int32_t *groups, int32_t *mb_bucket);

/* Set the launch plan (mb_bucket entries 1 or the larger height this dtype
 * and k allow, as reported by sgep_batch_plan after sgep_batch_tune; groups
 * >= 1, clipped to n, or -64 <= groups <= -1 for the persistent plan).  Only
 * before the first iteration (SGEP_EINVAL otherwise), because the norm
 * partials of a running state are laid out by tile.  The persistent plan
 * returns SGEP_EUNSUPPORTED unless every tile height is 1, k <= 32 (FP32) or
 * k <= 16 (FP64) and the device reports its XCC count.  Synchronises. */
sgep_status sgep_batch_set_plan(sgep_batch *bt, int32_t groups, const int32_t *mb_bucket);

/* Autotune the launch plan on a caller's minibatch before the first
 * iteration: every candidate (groups 1, 2, 4, 8 with, per width bucket, the
 * tile height 16 or the larger one; the persistent plan with look-ahead 1, 2
 * and 4 where it is supported) runs 1 + reps iterations from the initial
 * state on (X, Y, b) and is timed with HIP events; the fastest plan is kept
 * and the initial state restored, so the instances are as after
 * sgep_batch_init.  best_us (nullable) receives the chosen plan's time per
 * iteration in microseconds.  Allocates a temporary copy of the state.
 * Errors: SGEP_EINVAL after the first iteration; as sgep_batch_step. */
sgep_status sgep_batch_tune(sgep_batch *bt, const void *const *X, const void *const *Y, int64_t b,
                            int32_t reps, double *best_us);

/* sgep_sync of every instance; returns the first error. */
sgep_status sgep_batch_sync(sgep_batch *bt);

/* Release every instance and the batch (synchronises the stream first). */
sgep_status sgep_batch_destroy(sgep_batch *bt);

/* Static description of a status code. */
const char *sgep_status_string(sgep_status s);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t sgep_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SGEP_H */
