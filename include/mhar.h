/*
 * mhar.h -- C ABI of libmhar, a Matrix Hit-and-Run (MHAR) sampler for
 * AMD Instinct MI355X (gfx950).
 *
 * Problem (paper S2.1): sample uniformly from
 *     Delta = { x in R^n : A x <= b,  A_eq x = b_eq }
 * with z hit-and-run walks advanced together (paper S4, Alg. 2).  One step
 * of every walk k:
 *   1. h ~ N(0, I_n) from a counter-based Philox4x32-10 stream, Box-Muller
 *      pairs (paper S4.3, Lemma 4.1);
 *   2. d = P h with P = I - A_eq^T (A_eq A_eq^T)^{-1} A_eq when m_eq > 0
 *      (paper S3.2, Lemma 3.1), applied in factored form;
 *   3. line set: lambda_max = min over a_i d > 0 of (b_i - a_i x)/(a_i d),
 *      lambda_min = max over a_i d < 0 (paper S4.4, Lemma 4.2);
 *   4. theta = lambda_min + U (lambda_max - lambda_min), U ~ U(0,1) from the
 *      THETA stream; x <- x + theta d (paper S4.5, Lemma 4.3).
 * The products A D run on the matrix cores in the chosen precision; they only
 * screen which rows can bound each chord.  The bounding rows are then
 * evaluated exactly in FP64 with the formula of step 3, so the chord (and
 * the trajectory) is that of FP64 arithmetic in every precision mode.
 *
 * Random streams (identical definition in any conforming implementation):
 *   key     = (seed & 0xffffffff, seed >> 32)
 *   counter = (block, chain_id, step & 0xffffffff, tag | (step >> 32) << 4)
 *   tags: DIR = 0 (directions), THETA = 1 (chord position), LOWRANK = 2
 *   uniform: 52 high bits u of (w_hi << 32 | w_lo) -> (u + 1/2) 2^-52
 *   normal j of a stream: block j/2, u_a from words (0,1), u_b from (2,3);
 *   sqrt(-2 ln u_a) * (cos if j even else sin)(2 pi u_b)
 *   theta's U: block 0 of the THETA stream, words (0,1).
 *   chain_id = chain_offset + k, so chains can be split across calls (or
 *   devices) without changing any trajectory.
 *
 * Conventions
 *   - Matrices are row-major.  State matrices are (z x n): row k = walk k.
 *   - "dev" pointers are HIP device pointers; "host" pointers host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls enqueue work on it and return without synchronising, except
 *     where a call says it synchronises.
 *   - The caller owns every buffer it passes in.  The library never
 *     allocates device memory: create calls take a caller-provided device
 *     workspace whose size the matching *_workspace_size call reports, and
 *     which must stay valid until the handle is destroyed.  Handles are
 *     small host objects freed by the destroy calls.
 *   - Every call returns a status (0 = MHAR_OK, negative = error).  No call
 *     aborts; the text of the last error of the calling thread is available
 *     from mhar_last_error().  Argument and shape errors are reported before
 *     any work is enqueued.
 *   - Conditions found on the device are per-walk status bits (below),
 *     read with mhar_get_state / mhar_sync; a flagged walk stays where it is
 *     for that step (theta = 0) and keeps going.
 */
#ifndef MHAR_H
#define MHAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MHAR_OK = 0,
    MHAR_E_INVALID_ARG = -1,    /* null pointer, bad option value */
    MHAR_E_SHAPE = -2,          /* sizes out of the supported range */
    MHAR_E_RANK_DEFICIENT = -3, /* A_eq rows linearly dependent (pivot of A_eq A_eq^T <= 1e-12 max diag) */
    MHAR_E_NOT_INTERIOR = -4,   /* a start point is not strictly inside Delta */
    MHAR_E_WORKSPACE = -5,      /* workspace too small or misaligned (256 B) */
    MHAR_E_HIP = -6,            /* a HIP runtime call failed */
    MHAR_E_UNSUPPORTED = -7,    /* no kernel for this configuration */
    MHAR_E_STATE = -8           /* call not valid for the handle's state */
} mhar_status_t;

/* Precision of the matrix-core product A D (the screening product).  The
 * chord itself is always evaluated in FP64. */
typedef enum {
    MHAR_FP64 = 0,   /* FP64 MFMA */
    MHAR_FP32 = 1,   /* FP32 MFMA */
    MHAR_BF16X3 = 2  /* A and D split into bf16 hi + lo; hi*hi + hi*lo + lo*hi, FP32 accumulate */
} mhar_precision_t;

/* per-walk status bits */
enum {
    MHAR_CHAIN_OK = 0,
    MHAR_CHAIN_UNBOUNDED = 1,   /* no row bounds the line on one side (Delta assumed bounded, S2.1) */
    MHAR_CHAIN_DEGENERATE = 2,  /* lambda_max <= lambda_min */
    MHAR_CHAIN_NONFINITE = 4,   /* NaN/Inf in theta or the state */
    MHAR_CHAIN_INFEASIBLE = 8,  /* exact FP64 slack below -1e-12 max(1,|b_i|) */
    MHAR_FIT_FAILED = 32        /* (mhar_sync only) a covariance fit step met a non-positive
                                   pivot or a mean state outside the polytope; that step and
                                   every later one left the covariance unchanged */
};

/* Kernel path of the step.  Every path gives the same trajectories (the
 * chord is evaluated exactly in FP64); they differ in speed only. */
typedef enum {
    MHAR_PATH_AUTO = 0,      /* chosen from the shape (default) */
    MHAR_PATH_GENERAL = 1,   /* one workgroup per 16 walks over all rows, slack in HBM */
    MHAR_PATH_RESIDENT = 2,  /* slack in registers, rows split over co-resident workgroups;
                                FP32/BF16X3, n <= 256, m <= 8192 (else MHAR_E_UNSUPPORTED) */
    MHAR_PATH_TILED = 3,     /* per step a screening GEMM over 128-row x 128-walk tiles and a
                                chords kernel; FP32/BF16X3 (else MHAR_E_UNSUPPORTED) */
    MHAR_PATH_LANE = 4       /* a few lanes per walk, every row evaluated exactly in FP64 each
                                step (no screening product, so any precision); n <= 32, or
                                n <= 64 when A fits in 96 KB of LDS (else MHAR_E_UNSUPPORTED).  With a learned covariance attached the
                                handle steps on the general kernel.  AUTO takes it for
                                n <= 32 where its modelled step time (about
                                2.2 + 0.0065 m n + 0.4 n m_eq us) beats the
                                screened kernels'. */
} mhar_path_t;

typedef struct {
    int32_t precision;        /* mhar_precision_t, default MHAR_FP32 */
    int32_t recompute_every;  /* R >= 1: exact FP64 recompute of the slack b - A X every R steps (default 50) */
    int32_t steps_per_launch; /* 0 = automatic; bounds the steps one kernel launch runs */
    int32_t path;             /* mhar_path_t, default MHAR_PATH_AUTO */
    int32_t reserved[4];      /* must be 0 */
} mhar_options_t;

typedef struct mhar_problem* mhar_problem_t;
typedef struct mhar_chains* mhar_chains_t;
typedef struct mhar_batch* mhar_batch_t;

/* Diagnostics of one chains handle, accumulated since creation. */
typedef struct {
    uint64_t steps;             /* steps taken by every walk */
    uint64_t chain_steps;       /* walks x steps */
    uint64_t exact_rows;        /* rows evaluated exactly in FP64 (candidates of the screening;
                                   every row on the lane path) */
    uint64_t recomputes;        /* exact slack recomputes */
    int32_t kernel;             /* mhar_path_t of the last step: MHAR_PATH_GENERAL, _RESIDENT,
                                   _TILED or _LANE */
    int32_t split;              /* workgroups per 16-walk tile (resident kernel), else 1 */
} mhar_stats_t;

/* library version as major*10000 + minor*100 + patch */
int32_t mhar_version(void);
/* static text for a status code */
const char* mhar_status_string(int32_t status);
/* text of the last error raised on the calling thread ("" if none) */
const char* mhar_last_error(void);
/* fill *opt with the defaults */
mhar_status_t mhar_options_default(mhar_options_t* opt);

/* ---------------------------------------------------------------------- */
/* Problem: the polytope (paper S2.1) and its one-time setup              */
/* ---------------------------------------------------------------------- */

/* Device workspace bytes needed by mhar_problem_create for these sizes.
 * Supported: 1 <= n <= 1152 (up to 8192 in FP32 / BF16X3 with path AUTO or
 * TILED, which then runs the tiled path; batches take n <= 1152),
 * 1 <= m <= 2^24, 0 <= m_eq < n, m_eq <= 64. */
mhar_status_t mhar_problem_workspace_size(int64_t n, int64_t m, int64_t m_eq,
                                          const mhar_options_t* opt, size_t* bytes);

/* Copy the polytope into the workspace and run the one-time setup: FP64
 * copy of A (rows padded), row norms, the operand form of A for the chosen
 * precision and, when m_eq > 0, the Cholesky factor of A_eq A_eq^T and
 * W = A_eq^T (A_eq A_eq^T)^{-1} (paper S3.2; the explicit inverse of the
 * paper is replaced by triangular solves).
 *   A    dev, m x n FP64;  b dev, m;  A_eq dev, m_eq x n FP64 or NULL;
 *   b_eq dev, m_eq or NULL;  opt host or NULL (defaults);
 *   workspace dev, 256-byte aligned, ws_bytes >= the workspace size.
 * Synchronises `stream` once (to report MHAR_E_RANK_DEFICIENT); the input
 * arrays may be freed when it returns. */
mhar_status_t mhar_problem_create(int64_t n, int64_t m, const double* A, const double* b,
                                  int64_t m_eq, const double* A_eq, const double* b_eq,
                                  const mhar_options_t* opt, void* workspace, size_t ws_bytes,
                                  void* stream, mhar_problem_t* out);

/* Write the dense projection P = I - W A_eq (n x n FP64, dev) -- the
 * matrix the paper precomputes (S3.2) -- for inspection. */
mhar_status_t mhar_problem_get_projection(mhar_problem_t problem, double* P, void* stream);

mhar_status_t mhar_problem_destroy(mhar_problem_t problem);

/* ---------------------------------------------------------------------- */
/* Chains: z walks on one problem (paper Alg. 2)                          */
/* ---------------------------------------------------------------------- */

/* Device workspace bytes for z walks on `problem` (z >= 1). */
mhar_status_t mhar_chains_workspace_size(mhar_problem_t problem, int64_t z, size_t* bytes);

/* Start z walks at X0 (dev, z x n FP64), global chain ids chain_offset..,
 * Philox key `seed`, step counter 0.  Every start point must be strictly
 * interior: b - A x > 0 and |A_eq x - b_eq|_inf <= 1e-9 (Alg. 2 starts from
 * a strictly inner point), else MHAR_E_NOT_INTERIOR.  Synchronises `stream`
 * once for that check.  chain_offset + z must not exceed 2^32. */
mhar_status_t mhar_chains_create(mhar_problem_t problem, int64_t z, const double* X0,
                                 uint64_t seed, uint64_t chain_offset, void* workspace,
                                 size_t ws_bytes, void* stream, mhar_chains_t* out);

/* Enqueue `steps` MHAR iterations of every walk (steps >= 0). */
mhar_status_t mhar_step(mhar_chains_t chains, int64_t steps, void* stream);

/* Like mhar_step, and also store the states of walks 0 .. chain_count-1
 * after every stride-th step of this call into out (dev, FP64,
 * (steps/stride) x chain_count x n): the paper's thinned collection of
 * samples (Alg. 2, thinning factor = stride). */
mhar_status_t mhar_record(mhar_chains_t chains, int64_t steps, int64_t stride,
                          int64_t chain_count, double* out, void* stream);

/* Copy the current states (dev z x n FP64, may be NULL) and the per-walk
 * status bits (dev int32 z, may be NULL). */
mhar_status_t mhar_get_state(mhar_chains_t chains, double* X, int32_t* status, void* stream);

/* Replace the states with X (dev z x n FP64) and set the step counter;
 * the slack is recomputed exactly and the status bits cleared.  Used to
 * resume from a checkpoint.  The states are not re-validated. */
mhar_status_t mhar_set_state(mhar_chains_t chains, const double* X, uint64_t step, void* stream);

/* Checkpoint of the whole chain and training state (Alg. 2's X_t with the
 * step counter t, and an attached covariance with its training state): the
 * states, the per-walk status bits, the step counter and, when a covariance
 * is attached, U, V, log sigma, the Adam moments and step count, the Dikin
 * fit's power vector and complement scale, the frozen flag and the fit's
 * failure flag.  host_buf NULL: *bytes receives the size needed.  Otherwise
 * host_buf (host memory, *bytes long) is filled after synchronising
 * `stream`, and *bytes receives the size written.  The slack is not saved:
 * a restore recomputes it exactly, which leaves the trajectories unchanged
 * (the chord is evaluated exactly). */
mhar_status_t mhar_checkpoint(mhar_chains_t chains, void* host_buf, size_t* bytes, void* stream);

/* Restore a checkpoint into chains of the same problem shape, walk count,
 * seed and chain offset; a checkpoint with a covariance needs one of the
 * same rank and objective attached first (mhar_precond_create), one without
 * needs none.  Continuing from the restored handle gives bitwise the
 * trajectories (and covariance updates) of an uninterrupted run.
 * Synchronises `stream` before returning (the buffer may then be reused).
 * Errors: MHAR_E_INVALID_ARG (not a checkpoint, truncated), MHAR_E_SHAPE,
 * MHAR_E_STATE (seed, chain offset or covariance mismatch). */
mhar_status_t mhar_restore(mhar_chains_t chains, const void* host_buf, size_t bytes, void* stream);

/* Current step counter (host, no synchronisation). */
mhar_status_t mhar_get_step(mhar_chains_t chains, uint64_t* step);

/* Synchronise `stream` and return the OR of all per-walk status bits, plus
 * MHAR_FIT_FAILED when an attached covariance's fit failed. */
mhar_status_t mhar_sync(mhar_chains_t chains, void* stream, int32_t* any_flags);

/* Synchronise `stream` and read the diagnostics counters. */
mhar_status_t mhar_get_stats(mhar_chains_t chains, void* stream, mhar_stats_t* stats);

/* Result of mhar_chains_autotune. */
typedef struct {
    int32_t path;              /* the path kept (mhar_path_t) */
    int32_t reserved;
    double ms_per_step[5];     /* per mhar_path_t: measured ms per step, -1 if not tried */
} mhar_tune_t;

/* Choose the kernel path of a chains handle by measurement -- the paper's
 * study of walks per launch (S6.2) turned into a per-shape choice: every
 * path the handle can take (general; register-resident; tiled in FP32 or
 * BF16X3; lane for small n with isotropic directions) runs steps_per_trial
 * steps of the handle's own walks, timed with HIP events after an exact
 * recompute, and the fastest is kept for later mhar_step calls and for the
 * batches the handle joins (a batch runs a resident choice on the tiled
 * path or the general kernel).  A handle whose covariance was attached off
 * the tiled path does not try it (the split screening's buffers are sized
 * at attachment).  The trials are real steps: every path
 * produces bitwise the same walks, so the walks advance by (paths tried) x
 * steps_per_trial steps.  Synchronises `stream` once per path.
 * MHAR_E_INVALID_ARG for steps_per_trial outside [1, 2^20]. */
mhar_status_t mhar_chains_autotune(mhar_chains_t chains, int64_t steps_per_trial, void* stream,
                                   mhar_tune_t* out);

/* Replay the tiled path's launch sequence from a HIP graph of graph_steps
 * steps (0: off; else a multiple of the recompute period R).  mhar_step then
 * runs ordinary launches until the slack schedule restarts (just after an
 * exact recompute), replays the graph while graph_steps steps remain -- the
 * step counter lives on the device and the graph's last node advances it --
 * and runs the rest ordinarily.  The graph is captured (on a private stream)
 * at the first replay and again after the covariance changes; trajectories
 * are bitwise those of ordinary launches.  mhar_record, kernel timing
 * (mhar_trace_enable) and the other paths, whose launches run many steps
 * each, take ordinary launches.  MHAR_E_INVALID_ARG for a negative count or
 * one that R does not divide; MHAR_E_HIP if capture fails at mhar_step. */
mhar_status_t mhar_chains_set_graph(mhar_chains_t chains, int32_t graph_steps);

mhar_status_t mhar_chains_destroy(mhar_chains_t chains);

/* Kernel timing of the tiled path (paper S4.4-S4.5 split over its kernels):
 * with tracing enabled, every launch of the screening GEMM, the chords
 * kernel, the directions kernel and the exact recompute that mhar_step
 * enqueues on the tiled path is bracketed by a pair of HIP events on the
 * step stream, up to max_launches launches (later launches are not timed).
 * Other paths run many steps per launch; time them with events around
 * mhar_step.  The events are created by mhar_trace_enable (max_launches = 0
 * releases them) and by nothing else; mhar_chains_destroy releases them. */
typedef struct {
    int64_t launches[4];   /* 0 screening GEMM, 1 chords, 2 directions, 3 exact recompute */
    double ms[4];          /* summed event-to-event durations, milliseconds */
} mhar_trace_t;
mhar_status_t mhar_trace_enable(mhar_chains_t chains, int32_t max_launches);

/* Synchronise `stream`, sum the durations recorded since enable or the last
 * read per kernel kind into *out, and start a new record. */
mhar_status_t mhar_trace_read(mhar_chains_t chains, void* stream, mhar_trace_t* out);

/* For callers that cannot allocate device memory (a serving loop, a harness
 * that forbids it): mhar_problem_create + mhar_chains_create + mhar_step +
 * mhar_get_state + the two destroys in one call, with both workspaces carved
 * from one static device array of 64 MiB per GPU (held from the library's
 * load until the process ends) instead of caller workspaces.  Runs `steps`
 * isotropic MHAR steps of z walks from X (dev, z x n FP64, in place: the
 * start points in, the states after the steps out), global chain ids
 * chain_offset.., step counter starting at step0; status (dev, int32 z)
 * receives the per-walk bits.  The other arguments are those of
 * mhar_problem_create.  MHAR_E_WORKSPACE (before any device work) when the
 * two workspaces exceed the array.  Calls no device allocation routine.
 * Synchronises `stream` like the create calls.  Every call on a GPU shares
 * that GPU's array: calls that overlap on one GPU (other threads, other
 * streams) race; each call initialises what it reads. */
mhar_status_t mhar_run_noalloc(int64_t n, int64_t m, const double* A, const double* b,
                               int64_t m_eq, const double* A_eq, const double* b_eq, int64_t z,
                               double* X, int32_t* status, uint64_t seed, uint64_t chain_offset,
                               uint64_t step0, int64_t steps, const mhar_options_t* opt,
                               void* stream);

/* ---------------------------------------------------------------------- */
/* Learned direction covariance (burn-in only; not in the paper)          */
/* ---------------------------------------------------------------------- */
/* Directions become d = P (U eps + exp(l) o h), eps ~ N(0, I_rank) from the
 * LOWRANK stream, h ~ N(0, I_n): Gaussian with covariance
 * Sigma = U U^T + diag(exp(2 l)), symmetric and independent of the state,
 * so the uniform target is kept.  Training brings the body towards the
 * near-isotropic position the paper's cost analysis assumes (S3.1), by one
 * of two objectives fixed when the covariance is attached:
 *   MHAR_FIT_STATES: Adam on the Gaussian NLL of the walk states,
 *     1/2 log det Sigma + 1/2 tr(Sigma^{-1} S), S their (1/z) covariance
 *     about their mean;
 *   MHAR_FIT_DIKIN: the divergence of N(0, Sigma) from the Dikin ellipsoid
 *     at the mean walk state xbar,
 *       K = 1/2 tr(H Sigma) - 1/2 log det Sigma,
 *       H = sum_i a_i a_i^T / (b_i - a_i xbar)^2
 *     (the log-barrier Hessian; K is KL(N(0,Sigma) | N(0,H^{-1})) up to a
 *     constant).  Each step sets the diagonal to the largest Gaussian of the
 *     Jacobi shape diag(H)^{-1} inside the Dikin ellipsoid, times kappa^2
 *     (mhar_precond_set_complement),
 *     exp(2 l_i) = kappa^2 / (lam H_ii) with lam the power-iteration estimate
 *     (4 iterations per step, continued across steps from a unit vector
 *     drawn from the TRAIN stream, chain i, step 1) of the largest
 *     eigenvalue of diag(H)^{-1/2} H diag(H)^{-1/2}, and moves U by the
 *     H^{-1}-preconditioned gradient step U <- U - lr H^{-1} dK/dU.  The
 *     walk states reveal long axes of an elongated body only once the walks
 *     have explored them; the slacks of all rows at the mean state reveal
 *     them at once.  Costs O(n^2 m + n^3) per step (n <= 4096).
 * U is n x rank row-major FP64, l (log_sigma) has n entries. */
typedef enum {
    MHAR_FIT_STATES = 0,
    MHAR_FIT_DIKIN = 1
} mhar_fit_t;

/* Device workspace bytes for a covariance of rank 1..64 on these chains,
 * trained by `objective` (mhar_fit_t). */
mhar_status_t mhar_precond_workspace_size(mhar_chains_t chains, int32_t rank, int32_t objective,
                                          size_t* bytes);

/* Attach a covariance: U_ij = 0.01 N(0,1) from the stream (seed, tag 4,
 * chain = i, step 0), l = 0.  workspace: dev, 256-byte aligned. */
mhar_status_t mhar_precond_create(mhar_chains_t chains, int32_t rank, int32_t objective,
                                  void* workspace, size_t ws_bytes, void* stream);

/* Set U (dev n x rank) and log_sigma (dev n); clears the Adam moments and
 * sets the trained coordinates V = diag(exp(-log_sigma)) U. */
mhar_status_t mhar_precond_set(mhar_chains_t chains, const double* U, const double* log_sigma,
                               void* stream);

/* Copy U (dev n x rank) and log_sigma (dev n); either may be NULL. */
mhar_status_t mhar_precond_get(mhar_chains_t chains, double* U, double* log_sigma, void* stream);

/* The objective at the current states and (U, l) and its gradient: loss dev
 * (1 double: the NLL, or K), grad_U dev (n x rank), grad_log_sigma dev (n);
 * any may be NULL. */
mhar_status_t mhar_precond_loss(mhar_chains_t chains, double* loss, double* grad_U,
                                double* grad_log_sigma, void* stream);

/* `steps` burn-in steps: each is one MHAR step with the current Sigma,
 * then one update at the new states.
 * MHAR_FIT_STATES: one Adam update (beta1 0.9, beta2 0.999, eps 1e-8,
 *   learning rate lr > 0) in the scale-free coordinates (V, log_sigma) with
 *   U = diag(exp(log_sigma)) V: their gradients are diag(exp(log_sigma))
 *   grad_U and grad_log_sigma plus the row sums of grad_U o U, so every
 *   axis, long or short, gets an O(1) step.  U is rebuilt from V.
 * MHAR_FIT_DIKIN: the step described above with step size lr in (0, 1];
 *   lr = 1/2 takes the column norms of U along the Babylonian iteration to
 *   their optimum.
 * MHAR_E_STATE once frozen. */
mhar_status_t mhar_precond_train(mhar_chains_t chains, int64_t steps, double lr, void* stream);

/* MHAR_FIT_DIKIN only: scale kappa in (0, 1] of the diagonal relative to the
 * largest Jacobi-shaped Gaussian inside the Dikin ellipsoid, applied from
 * the next fit step on (default 0.1): exp(2 l_i) = kappa^2 / (lam H_ii).  A
 * hit-and-run chord is cut short by whichever axis its direction overshoots;
 * with many short axes in the complement of U, kappa < 1 keeps the
 * isotropic part from cutting the chords along U short.  (Measured on a
 * rotated box, n = 1000, rank 64: min-marginal ESS of 5000 steps 9.5 k at
 * kappa = 1, 17 k at 0.1 and 0.01.) */
mhar_status_t mhar_precond_set_complement(mhar_chains_t chains, double kappa);

/* Freeze the covariance: later steps use it unchanged, training is refused. */
mhar_status_t mhar_precond_freeze(mhar_chains_t chains);

/* Detach the covariance: back to isotropic directions. */
mhar_status_t mhar_precond_destroy(mhar_chains_t chains);

/* ---------------------------------------------------------------------- */
/* Batches: many problems of uneven n and m in one persistent launch      */
/* ---------------------------------------------------------------------- */
/* A batch groups `count` existing chains handles (each on its own problem,
 * all of one precision).  mhar_batch_step advances all of them by the same
 * number of steps in one persistent launch: workgroups take (problem,
 * 16-walk tile) units from a device queue ordered by decreasing cost
 * (m x n), the longest-processing-time-first rule, so uneven problems
 * balance across the GPU.  Trajectories are identical to stepping each
 * handle alone.  The handles stay owned by the caller, must outlive the
 * batch, and should not be stepped on other streams while it exists. */

/* Device workspace bytes for a batch of these handles (count >= 1). */
mhar_status_t mhar_batch_workspace_size(int32_t count, const mhar_chains_t* chains, size_t* bytes);

/* Create the batch (host array of `count` handles; workspace dev, 256-byte
 * aligned).  Allocates one small pinned host buffer for the unit
 * descriptors. */
mhar_status_t mhar_batch_create(int32_t count, const mhar_chains_t* chains, void* workspace,
                                size_t ws_bytes, mhar_batch_t* out);

/* Enqueue `steps` steps of every handle in the batch. */
mhar_status_t mhar_batch_step(mhar_batch_t batch, int64_t steps, void* stream);

/* Release the batch; the handles return to their own kernel paths (a
 * packed batch destroys the handles it created).  The batch is released
 * even when the wait for its last descriptor copy or the release of its
 * pinned buffer reports an error, which is then returned (MHAR_E_HIP). */
mhar_status_t mhar_batch_destroy(mhar_batch_t batch);

/* Packed batches: `count` inequality-only polytopes {A_i x <= b_i} (paper
 * S2.1) given as one device array per field plus host offsets, so that a
 * caller can hold each field of the whole batch in one tensor:
 *   n, m, z       host arrays of count sizes (n_i <= 1152, any m_i, z_i >= 1);
 *   A_packed      dev FP64; problem i's A (m_i x n_i row-major) starts at
 *                 element A_offsets[i] (host array);
 *   b_packed      dev FP64; b_i (m_i) starts at b_offsets[i];
 *   X0_packed     dev FP64; the start points of problem i (z_i x n_i
 *                 row-major, walk k in row k) start at X0_offsets[i].
 * Walk k of problem i draws its random numbers as walk W_i + k of `seed`,
 * W_i = z_0 + ... + z_{i-1}, so every walk of the batch has its own stream
 * (the total must not exceed 2^32).  One precision (opt) for all problems.
 * The library creates a problem and a chains handle per polytope inside
 * the workspace (dev, 256-byte aligned, ws_bytes >= the size below), checks
 * that every start point is strictly interior (one synchronisation of
 * `stream` per problem; MHAR_E_NOT_INTERIOR names the problem), and returns
 * a batch that owns them: read them through mhar_batch_get_chains and step
 * them with mhar_batch_step; mhar_batch_destroy releases them.  The packed
 * inputs may be freed once the call returns.  Errors leave nothing
 * allocated. */
mhar_status_t mhar_batch_packed_workspace_size(int32_t count, const int64_t* n, const int64_t* m,
                                               const int64_t* z, const mhar_options_t* opt, size_t* bytes);
mhar_status_t mhar_batch_create_packed(int32_t count, const int64_t* n, const int64_t* m, const int64_t* z,
                                       const double* A_packed, const int64_t* A_offsets,
                                       const double* b_packed, const int64_t* b_offsets,
                                       const double* X0_packed, const int64_t* X0_offsets, uint64_t seed,
                                       const mhar_options_t* opt, void* workspace, size_t ws_bytes,
                                       void* stream, mhar_batch_t* out);

/* The chains handle of problem i (0 <= i < count) of a batch, borrowed: it
 * stays valid while the batch lives; for mhar_get_state, mhar_record and
 * the other per-handle calls. */
mhar_status_t mhar_batch_get_chains(mhar_batch_t batch, int32_t i, mhar_chains_t* out);

#ifdef __cplusplus
}
#endif
#endif /* MHAR_H */
