/*
 * dsmc.h - C ABI of an MI355X (gfx950) implementation of dSMC, the
 * de-Sequentialized Monte Carlo particle smoother of Corenflos, Chopin and
 * Sarkka (2022).
 *
 * What the library computes (paper, Section 2):
 *   leaves   Algorithm 2: for every time t, N particles X_t^n ~ q_t with
 *            normalised log-weights and log L_t = log mean_n w_t^n; the t = 0
 *            weight is h_0 dP_0/dq_0 (Proposition 2.2).
 *   tree     Algorithm 6 (appendix, parallel combination by array reshaping):
 *            ceil(log2 K) levels; at level l, adjacent blocks of 2^l time
 *            points are merged at boundary c = (2k+1) 2^l, and a block whose
 *            right neighbour is padding is left as it is.
 *   combine  Algorithm 1 at each boundary c: the N x N product-form weights
 *            W_c^{mn} (normalised-weights equation, Section 2.2) with the
 *            stitching weight omega_c of Proposition 2.3, their log-sum
 *            (the normalising-constant increment, equation for L_{a:b}),
 *            N multinomial draws of index pairs (l_n, r_n) (the resampling of
 *            Proposition 2.4), and the gather of the chosen trajectories.
 *   output   equally weighted trajectories approximating Q_{0:K-1} and
 *            log L^N = sum_t log L_t + sum_c Z_c.
 *   conditional  (Section 3.1, Algorithm 4) the same with a given star
 *            trajectory kept in slot 0 throughout: dsmc_smooth_conditional.
 *   lazy     (Section 4.2, Algorithms 7 and 8) the combine's multinomial draw
 *            replaced by Metropolis-Hastings or rejection chains that evaluate
 *            only the pairs they propose: dsmc_plan_desc.resampling.
 *
 * Time points are t = 0..K-1 (the paper's t = 0..T with K = T + 1).
 *
 * Randomness: the library owns it.  Every draw comes from Philox4x64-10
 * (Salmon et al., SC'11) with key (seed, 0x64534D43) and counter
 * (block, t or c, purpose, j).  Purpose 2 = leaf normals, four per block
 * (Box-Muller on the word pairs): for d_x dividing 4 the normals of time t are
 * one flat stream (block q, j = 0: normals 4q..4q+3; coordinate i of particle
 * n is normal n d_x + i), otherwise block (n, t, 2, j) gives normals 4j..4j+3
 * of particle n.  Purpose 3 = the two uniforms (u1, u2) of draw n of the
 * combine at c: block (n, c, 3, 0), words 0 and 1.  Results therefore depend
 * only on (model, N, seed), not on batching or launch order.
 *
 * Multinomial draws are taken in two stages: the left index from the row
 * marginal with u1, then the right index from that row with u2, each by the
 * inverse CDF "first index whose cumulative weight exceeds u * total" on fp64
 * cumulative sums (zero-weight entries are never drawn).
 *
 * Conventions
 *   - Every function returns a dsmc_status (0 = success, < 0 = error) unless
 *     stated otherwise; dsmc_last_error() returns a thread-local message.
 *   - Pointers in dsmc_model_desc are HOST pointers, read during
 *     dsmc_model_create only.  Pointers in dsmc_output are DEVICE pointers
 *     owned by the caller.
 *   - Matrices are row-major, fp64.  Cholesky factors are lower triangular
 *     with positive diagonal.
 *   - dsmc_smooth / dsmc_smooth_conditional / dsmc_smooth_batch validate
 *     their arguments, enqueue all work on the plan's stream and return
 *     without synchronising.  Numerical
 *     conditions found on the device are reported in dsmc_output.status.
 */
#ifndef DSMC_H
#define DSMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dsmc_status {
  DSMC_OK = 0,
  DSMC_EINVAL = -1,       /* invalid argument */
  DSMC_ENOMEM = -2,       /* device or host allocation failed, or plan too small */
  DSMC_EUNSUPPORTED = -3, /* size or option the library does not support */
  DSMC_EAGAIN = -4,       /* dsmc_poll: the job has not finished */
  DSMC_EDEGENERATE = -5,  /* a combine had zero total weight */
  DSMC_ENUMERIC = -6,     /* a weight was NaN */
  DSMC_ECALLBACK = -7,    /* a model callback returned nonzero */
  DSMC_EDEVICE = -8,      /* HIP runtime error */
  DSMC_ECANCELLED = -9,   /* job cancelled, or server shut down, before the job ran */
  DSMC_EDEADLINE = -10    /* serving: the job was still queued at its admission deadline */
} dsmc_status;

/* Bits written to dsmc_output.status by the device (0 = clean run). */
#define DSMC_FLAG_DEGENERATE 1 /* some combine (or leaf) had total weight 0; log_Z = -inf */
#define DSMC_FLAG_NUMERIC 2    /* a NaN weight was met; outputs are undefined */
#define DSMC_FLAG_LAZY_CAP 4   /* a rejection draw hit its proposal cap (DSMC_RESAMPLE_RS) */

/* Largest state dimension and particle count the library accepts. */
#define DSMC_MAX_DX 32
#define DSMC_MAX_N 4096

/* ---------------------------------------------------------------- model */

enum { DSMC_OBS_NONE = -1,           /* no parametric form: h_t is given by the
                                        log_observation callback only, which the
                                        device cannot run (DSMC_EUNSUPPORTED) */
       DSMC_OBS_LINEAR_GAUSSIAN = 0, /* y_t ~ N(H x_t + h, R)                  */
       DSMC_OBS_STOCH_VOL = 1,       /* y_t ~ N(0, exp(x_t)), needs d_x = d_y = 1 */
       DSMC_OBS_BOX = 2 };           /* h_t(x) = 1 if lo_t <= x <= hi_t else 0, with
                                        y_t = (lo_t, hi_t), d_y = 2 d_x: the constrained
                                        random walk of Section 5.3 */

/* Proposal family: GAUSSIAN q_t = N(q_mean[t], q_chol[t] q_chol[t]^T);
 * UNIFORM q_t uniform on the box q_mean[t] +- diag(q_chol[t]) (d_x <= 4; the
 * uniforms are the leaf Philox words, in the places of the normals). */
enum { DSMC_PROPOSAL_GAUSSIAN = 0, DSMC_PROPOSAL_UNIFORM = 1 };

/* Choice of the auxiliary measures nu_t of Definition 2.1 (Section 2.1):
 *   LEAF_OBS      nu_t proportional to h_t q_t: leaf log-weight log h_t (t >= 1),
 *                 log omega_c = log p_c - log q_c (+ a constant estimated by L_t);
 *   BOUNDARY_OBS  nu_t = q_t as in the paper's experiments: leaf weight 1
 *                 (t >= 1), log omega_c = log p_c + log h_c - log q_c.
 * Both target the same smoothing distribution. */
enum { DSMC_WEIGHT_LEAF_OBS = 0, DSMC_WEIGHT_BOUNDARY_OBS = 1 };

/* Host callbacks: the model as the problem statement of the paper's
 * introduction gives it (prior P_0, transition densities p_t, potentials h_t)
 * plus Algorithm 2's proposals q_t.  Each is vectorised over n points, fp64,
 * row-major [n][d_x], and returns 0 on success (nonzero: DSMC_ECALLBACK).
 * Callbacks must be deterministic; the library owns all randomness and hands
 * the proposal its standard variates z.
 *   log_prior        out[i] = log p_0(x_i)
 *   log_transition   out[i] = log p_t(x_i | xp_i), t >= 1
 *   log_observation  out[i] = log h_t(x_i)
 *   proposal         x_out[i] = the draw of q_t made from z_i (standard normals
 *                    for Gaussian proposals, uniforms on [0, 1) for uniform
 *                    ones) and logq_out[i] = log q_t(x_out[i])
 * The GPU cannot call host code, so the kernels evaluate the parametric
 * (device) form of dsmc_model_desc; the callbacks define the model and
 * dsmc_model_check / dsmc_model_create verify that the device form computes
 * the same densities (see dsmc_model_check).  Any callback may be NULL
 * (not checked). */
typedef struct dsmc_model_callbacks {
  void *ctx;
  int (*log_prior)(void *ctx, int n, const double *x, double *out);
  int (*log_transition)(void *ctx, int t, int n, const double *xp, const double *x, double *out);
  int (*log_observation)(void *ctx, int t, int n, const double *x, double *out);
  int (*proposal)(void *ctx, int t, int n, const double *z, double *x_out, double *logq_out);
} dsmc_model_callbacks;

/* The Feynman-Kac model of the paper's introduction: prior P_0, transitions
 * P_t with density p_t, potentials h_t, and the independent proposals q_t of
 * Algorithm 2, given in the parametric (device) form below, read in fp64, and
 * optionally also as host callbacks (dsmc_model_callbacks). */
typedef struct dsmc_model_desc {
  int K;   /* time points t = 0..K-1, K >= 1 */
  int d_x; /* state dimension, 1..DSMC_MAX_DX */
  int d_y; /* observation dimension, >= 1 */
  /* prior P_0 = N(m0, P0 = P0_chol P0_chol^T) */
  const double *m0;      /* [d_x] */
  const double *P0_chol; /* [d_x][d_x] */
  /* transition P_t(x_t | x_{t-1}) = N(F x_{t-1} + f, Q = Q_chol Q_chol^T), t >= 1 */
  const double *F;      /* [d_x][d_x] */
  const double *f;      /* [d_x] */
  const double *Q_chol; /* [d_x][d_x] */
  /* potential h_t(x_t) = density of the observation y_t given x_t */
  int obs_kind;         /* DSMC_OBS_* */
  const double *H;      /* [d_y][d_x] (LINEAR_GAUSSIAN only) */
  const double *h;      /* [d_y]      (LINEAR_GAUSSIAN only) */
  const double *R_chol; /* [d_y][d_y] (LINEAR_GAUSSIAN only) */
  const double *y;      /* [K][d_y] */
  /* proposal q_t = N(q_mean[t], q_chol[t] q_chol[t]^T), independent over t */
  const double *q_mean; /* [K][d_x] */
  const double *q_chol; /* [K][d_x][d_x] */
  int weighting;        /* DSMC_WEIGHT_* */
  int proposal_kind;    /* DSMC_PROPOSAL_* (0 = Gaussian) */
  const dsmc_model_callbacks *callbacks; /* optional host form of the model (NULL = none) */
} dsmc_model_desc;

typedef struct dsmc_model dsmc_model_t;

/* Host-only validation of a description, no device work.  Checks sizes, kinds
 * and parameters (DSMC_EINVAL).  With callbacks it then evaluates the device
 * form against them at 256 check points: 16 time points t spread over 0..K-1,
 * 16 points each, x drawn from q_t (and x' from q_{t-1} for the transition)
 * with variates of a fixed host generator.  Every log density must agree
 * within |d| <= 1e-9 max(1, |callback value|) (both -inf counts as equal),
 * and the proposal's x and log q likewise; otherwise DSMC_EINVAL, with the
 * component, t and the two values in dsmc_last_error.  A callback returning
 * nonzero gives DSMC_ECALLBACK.  Callbacks without a complete device form
 * (obs_kind DSMC_OBS_NONE, or a missing prior, transition or proposal array)
 * give DSMC_EUNSUPPORTED: the kernels have nothing to evaluate. */
int dsmc_model_check(const dsmc_model_desc *desc);

/* dsmc_model_check, then derive inverse Cholesky factors and log normalisers
 * on the host in fp64 and copy the device form to device memory of the
 * current device (synchronously).  Errors: those of dsmc_model_check
 * (DSMC_EINVAL: bad sizes, non-positive Cholesky diagonal, unknown kind,
 * STOCH_VOL with d_x != 1, BOX with d_y != 2 d_x, UNIFORM proposals with
 * d_x > 4, device form disagreeing with the callbacks; DSMC_ECALLBACK;
 * DSMC_EUNSUPPORTED), DSMC_ENOMEM, DSMC_EDEVICE.  Callbacks are not called
 * after this returns.  The model may be shared by many calls. */
int dsmc_model_create(const dsmc_model_desc *desc, dsmc_model_t **out);
void dsmc_model_destroy(dsmc_model_t *model);
int dsmc_model_K(const dsmc_model_t *model);

/* Parallel-in-time Gaussian proposals (Section 4.1, Algorithm 5) for a
 * linear-Gaussian model (obs_kind LINEAR_GAUSSIAN, Gaussian proposals): the
 * Kalman filter and the RTS smoother run on the device as associative scans
 * over the K time points (span O(log K)), in fp64, and the smoothing marginals
 * N(m_t, P_t) replace the model's proposals q_t (q_mean, q_chol and the derived
 * inverse factors and log normalisers).  For a linear-Gaussian model the
 * linearisation of Algorithm 5 is exact, so one pass is its fixed point.
 * Enqueued on `stream` (hipStream_t, NULL = null stream); smoother calls
 * ordered after it on the same stream use the new proposals, so the model
 * must not be in use by other streams meanwhile.  The model keeps a workspace
 * of about K (5 d_x^2 + 3 d_x) 8 bytes, allocated on the first call.
 * Errors: DSMC_EINVAL (null model), DSMC_EUNSUPPORTED (other model kinds,
 * d_y > DSMC_MAX_DX), DSMC_ENOMEM, DSMC_EDEVICE. */
int dsmc_model_gaussian_proposals(dsmc_model_t *model, void *stream);

/* Copy the model's current proposals to host memory (synchronises the device):
 * q_mean [K][d_x], q_chol [K][d_x][d_x].  Errors: DSMC_EINVAL, DSMC_EDEVICE. */
int dsmc_model_read_proposals(const dsmc_model_t *model, double *q_mean, double *q_chol);

/* ----------------------------------------------------------------- plan */

enum { DSMC_FP32 = 0, /* particles and pair weights in fp32, sums and CDFs in fp64 */
       DSMC_FP64 = 1, /* everything in fp64 */
       DSMC_BF16 = 2  /* d_x >= 9 only (padded to 16 or 32): as DSMC_FP32, except that the
                         quadratic form ||u - v||^2 of Algorithm 1's pair weight (whitened
                         boundary coordinates u, v) is formed as ||u||^2 + ||v||^2 - 2 u.v
                         with fp32 norms and the dot products on bf16 matrix cores (fp32
                         accumulation) from split operands: each of 2u and v is a bf16
                         number plus a bf16 remainder and three products are summed, so
                         u.v carries about 16 significant bits; results differ from the
                         fp64 oracle by that rounding and the cancellation of the
                         expanded form.  The sampling kernel recomputes a chunk's weights
                         in the direct form and rescales its search to the stored chunk
                         sum, so every draw stays inside its chunk. */ };

#define DSMC_PLAN_PROFILE 1  /* record HIP events around every kernel launch */
#define DSMC_PLAN_AUTOTUNE 2 /* on first use of each level size (combines per launch), run the
                                level with every pair-row tile shape and keep the fastest;
                                costs several level runs per new size, results do not depend
                                on it */
#define DSMC_PLAN_RESCUE_ALL 8 /* testing aid: every row of every combine takes the paths that
                                  rows leaving the fp32 range take (d_x >= 8: the pair-row
                                  kernel redoes its rows with exact row maxima; the sampling
                                  kernel recomputes every row's chunk sums with its exact
                                  maximum as shift); results stay exact */
#define DSMC_PLAN_GRAPH 4    /* capture the kernels of dsmc_smooth / dsmc_smooth_batch for one
                                batch shape (the list of K) in a hipGraph and replay it while
                                the shape repeats: the first call of a shape runs eagerly, the
                                second captures, later ones replay (ignored with
                                DSMC_PLAN_PROFILE).  Models, seeds and outputs may change
                                between calls; they are read from device memory the call
                                uploads before the graph runs. */

typedef struct dsmc_plan_desc {
  int N;           /* particles per time point, 1..DSMC_MAX_N */
  int d_x;         /* state dimension of the models run with this plan */
  int max_K;       /* largest K of one series */
  int max_total_K; /* largest sum of K over one dsmc_smooth_batch call (0 = max_K) */
  int precision;   /* DSMC_FP32, DSMC_FP64 or DSMC_BF16 */
  int flags;       /* DSMC_PLAN_* */
  void *stream;    /* hipStream_t all work is enqueued on; NULL = null stream */
  int resampling;  /* DSMC_RESAMPLE_*: how each combine draws its N index pairs */
  int lazy_param;  /* DSMC_RESAMPLE_MH: steps B per draw (0 = DSMC_MH_STEPS_DEFAULT);
                      DSMC_RESAMPLE_RS: proposals per draw before giving up
                      (0 = DSMC_RS_CAP_DEFAULT) */
} dsmc_plan_desc;

/* Resampling of a combine.  EXACT: Algorithm 1's multinomial draw from all
 * N x N pair weights (pair-row pass, then two-stage inverse CDF); Z_c and
 * log L^N are computed.  The lazy schemes of Section 4.2 run no pair-row pass
 * and evaluate only the pairs they propose, O(N * steps) work per combine:
 *   MH  Algorithm 7: draw n is a Metropolis-Hastings chain started at (n, n)
 *       with proposals uniform over the N^2 pairs, `lazy_param` steps; it
 *       targets W_c but is biased after finitely many steps.
 *   RS  Algorithm 8: draw n proposes pairs uniformly and accepts with
 *       probability W_c(pair) / W_bar, W_bar = max_m w_m * max_n w'_n * max p_c
 *       (a bound of every pair weight of the combine); exact multinomial draws
 *       with random run time.  A draw still rejecting after `lazy_param`
 *       proposals keeps its last proposal and sets DSMC_FLAG_LAZY_CAP.
 * Proposals 2j and 2j + 1 of draw n at boundary c use Philox block
 * (n, c, 4 (MH) or 5 (RS), j): proposal 2j + h takes I = floor(lo32 N / 2^32)
 * and J = floor(hi32 N / 2^32) from the 32-bit halves of word 2h and its
 * acceptance uniform from word 2h + 1 (53 bits).
 * Lazy plans estimate no increment: logZ_inc, row_lse and log_Z are NaN.
 * Conditional runs keep slot 0 as in EXACT plans.  dsmc_plan rejects a lazy
 * scheme with DSMC_BF16 (DSMC_EUNSUPPORTED), an unknown scheme or a negative
 * lazy_param (DSMC_EINVAL). */
#define DSMC_RESAMPLE_EXACT 0
#define DSMC_RESAMPLE_MH 1
#define DSMC_RESAMPLE_RS 2
#define DSMC_MH_STEPS_DEFAULT 32
#define DSMC_RS_CAP_DEFAULT (1 << 20)

typedef struct dsmc_plan_impl dsmc_plan_t;

/* Allocate the plan's device workspace: about
 * max_total_K * N * ((5 d_x + 2) s + 36) bytes for particles, weights, ancestry
 * and per-combine data, plus at most 2 GiB of per-level chunk sums
 * (2 N * N * s / 32 per combine of a launch), s = sizeof the real type;
 * DSMC_BF16 adds max_total_K * N * (16 D + 16) bytes of bf16 operands (D = d_x padded
 * to 16 or 32).
 * Errors: DSMC_EINVAL, DSMC_EUNSUPPORTED (also DSMC_BF16 with d_x <= 8),
 * DSMC_ENOMEM. */
/* Number of GPUs the library's HIP runtime sees (*count, 0 on error).
 * A process that also uses another copy of the HIP runtime (PyTorch ships
 * its own) must load that copy before this library.  Errors: DSMC_EINVAL
 * (null count), DSMC_EDEVICE (no GPU). */
int dsmc_device_count(int *count);

int dsmc_plan(const dsmc_plan_desc *desc, dsmc_plan_t **out);
void dsmc_plan_destroy(dsmc_plan_t *plan);

/* ---------------------------------------------------------------- output */

/* Caller-owned DEVICE buffers for one series of K time points.  `real` is
 * float for DSMC_FP32 and DSMC_BF16 plans and double for DSMC_FP64 plans. */
typedef struct dsmc_output {
  void *traj;      /* real [d_x][K][N]: trajectory n is traj[.][0..K-1][n] (required) */
  void *logw;      /* real [N]: log-weights of the trajectories; -log N when K >= 2,
                      the normalised leaf weights when K == 1 (optional) */
  double *log_Z;   /* [1]: log L^N (required) */
  int32_t *status; /* [1]: DSMC_FLAG_* bits, 0 on a clean run (required) */
  /* diagnostics, NULL = not written */
  void *leaf_x;      /* real [d_x][K][N]: leaf particles X_t^n */
  void *leaf_logw;   /* real [K][N]: normalised leaf log-weights */
  double *leaf_logL; /* [K]: log L_t */
  int32_t *ancestry; /* [K-1][2][N]: (l_n, r_n) of the combine at boundary c, row c-1 */
  double *logZ_inc;  /* [K-1]: Z_c = log sum_{m,n} exp S_c[m,n], row c-1 */
  double *row_lse;   /* [K-1][N]: r_m = log sum_n exp S_c[m,n], row c-1 */
  int32_t *index;    /* [K][N]: leaf particle index of traj[.][t][n] */
} dsmc_output;

/* ------------------------------------------------------------- smoothing */

/* One smoother run: leaves, the combine tree, output.  model->K <= max_K,
 * model d_x == plan d_x.  Enqueued on the plan's stream; `out` buffers must
 * stay valid until the stream reaches this work.  Calls on one plan must not
 * overlap (they share its workspace).  Errors: DSMC_EINVAL, DSMC_EDEVICE. */
int dsmc_smooth(dsmc_plan_t *plan, const dsmc_model_t *model, uint64_t seed,
                const dsmc_output *out);

/* Conditional dSMC (Section 3.1; Algorithm 4 and the conditional
 * initialisation of Section 3.2), the sampling step of parallel-in-time
 * particle Gibbs.  `star` is a DEVICE buffer, real [d_x][K] (the layout of
 * traj with one particle), owned by the caller and read until the stream
 * reaches this work.  The star trajectory takes slot 0 at every time point;
 * slot n >= 1 holds the proposal draw dsmc_smooth puts there.  Weights, row
 * sums, increments and log L^N cover all N x N pairs, the star's included;
 * every combine draws slots 1..N-1 as dsmc_smooth does and keeps (0, 0) for
 * slot 0, so traj[.][.][0] equals the star and index[.][0] is 0.  A new star
 * for the next Gibbs sweep is any output trajectory picked uniformly.
 * Errors as dsmc_smooth; a null `star` is DSMC_EINVAL. */
int dsmc_smooth_conditional(dsmc_plan_t *plan, const dsmc_model_t *model, uint64_t seed,
                            const void *star, const dsmc_output *out);

/* B conditional runs (e.g. independent particle Gibbs chains) in packed
 * launches, as dsmc_smooth_batch; stars[s] is series s's star trajectory
 * (device, real [d_x][K_s]) or NULL for an unconditional run.  Results equal
 * B separate dsmc_smooth_conditional / dsmc_smooth calls bit for bit. */
int dsmc_smooth_batch_conditional(dsmc_plan_t *plan, int B, const dsmc_model_t *const *models,
                                  const uint64_t *seeds, const void *const *stars,
                                  const dsmc_output *outs);

/* B independent series (each with its own model, K and seed) in packed
 * launches: every level's combines of all series run in the same kernels.
 * The results equal B separate dsmc_smooth calls bit for bit.
 * sum of K <= max_total_K.  Errors as dsmc_smooth. */
int dsmc_smooth_batch(dsmc_plan_t *plan, int B, const dsmc_model_t *const *models,
                      const uint64_t *seeds, const dsmc_output *outs);

/* ------------------------------------------------- allocation-free run */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * dsmc_smooth run without a plan and without any device allocation.  All
 * workspace (particles, weights, per-time tables, per-combine data, chunk sums
 * and the combine tree, which a kernel writes from its closed form) lives in a
 * fixed device array of DSMC_STATIC_SCRATCH_BYTES that the library holds on
 * each GPU it runs on until the process ends; the call makes no hipMalloc,
 * hipFree or host-to-device copy.  Results equal dsmc_smooth with the same
 * model, N, precision and seed bit for bit.
 *   precision  DSMC_FP32 or DSMC_FP64 (else DSMC_EUNSUPPORTED);
 *   out        as dsmc_smooth (caller-owned device buffers);
 *   stream     hipStream_t the work is enqueued on (NULL = null stream).
 * The workspace needs about K N ((d_x + 4 D + 3) s + 24) bytes (s = 4 or 8,
 * D = d_x rounded up to a power of two) plus the chunk sums of at least one
 * combine, 2 N ceil(N / 128) 4 s bytes; a run that does not fit fails with
 * DSMC_EUNSUPPORTED before any device work (the stochastic-volatility run with
 * K = 4096, N = 1024 in fp32 fits).  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams or threads) race and
 * must be serialised by the caller; a call may start once the previous one's
 * work is ordered before it on the stream.  Errors: DSMC_EINVAL,
 * DSMC_EUNSUPPORTED, DSMC_EDEVICE. */
#define DSMC_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
int dsmc_smooth_static(const dsmc_model_t *model, int N, int precision, uint64_t seed,
                       const dsmc_output *out, void *stream);

/* --------------------------------------------------------------- serving */

/* A serving engine runs smoothing jobs submitted at any time, with continuous
 * batching: a scheduler thread admits queued jobs as device memory and slots
 * free up, runs their leaves, and at every step packs the next tree level of
 * every resident job of the same (N, d_x) class into one shared pair-rows and
 * one sampling launch.  A job's results equal those of dsmc_smooth alone with
 * the same model, N and seed, bit for bit. */
typedef struct dsmc_server_desc {
  size_t mem_budget; /* device bytes for all job classes together (0 = 16 GiB) */
  int max_jobs;      /* resident jobs per class (0 = 1024) */
  int max_classes;   /* distinct (N, d_x) classes; each gets mem_budget / max_classes (0 = 4) */
  int precision;     /* DSMC_FP32 or DSMC_FP64 */
  int flags;         /* reserved, 0 */
} dsmc_server_desc;

typedef struct dsmc_server_impl dsmc_server_t;

/* One smoothing job.  The model and the output buffers must stay valid until
 * dsmc_poll reports the job DONE or FAILED. */
typedef struct dsmc_job {
  const dsmc_model_t *model;
  int N;          /* particles, 1..DSMC_MAX_N */
  uint64_t seed;
  dsmc_output out;
  double admit_deadline; /* seconds after submission by which the job must have been
                            admitted (placed on the GPU), else it fails with
                            DSMC_EDEADLINE; 0 = none */
} dsmc_job;

enum { DSMC_JOB_QUEUED = 0, DSMC_JOB_RUNNING = 1, DSMC_JOB_DONE = 2, DSMC_JOB_FAILED = 3 };

/* Start the scheduler thread.  Device pools are allocated per class on first
 * use.  Errors: DSMC_EINVAL, DSMC_ENOMEM, DSMC_EDEVICE. */
int dsmc_server_create(const dsmc_server_desc *desc, dsmc_server_t **out);
/* Stop: queued jobs become FAILED (DSMC_ECANCELLED); jobs already on the GPU
 * are finished; device pools are released. */
void dsmc_server_destroy(dsmc_server_t *server);
/* Queue a job (its descriptor is copied).  Errors (job not created):
 * DSMC_EINVAL (bad arguments), DSMC_EUNSUPPORTED (N or d_x out of range). */
int dsmc_submit(dsmc_server_t *server, const dsmc_job *job, uint64_t *job_id);
/* Cancel a queued job: it becomes FAILED (DSMC_ECANCELLED) and its outputs
 * are not written.  Returns DSMC_OK, DSMC_EAGAIN if the job is already
 * running or finished (it completes normally), DSMC_EINVAL for an unknown id.
 * The cancellation takes effect at the scheduler's next step: poll for the
 * final state. */
int dsmc_cancel(dsmc_server_t *server, uint64_t job_id);
/* State of a job: returns DSMC_OK when DONE (outputs complete on the device),
 * DSMC_EAGAIN while QUEUED or RUNNING, the job's error code when FAILED
 * (DSMC_ENOMEM: it can never fit the class pool; DSMC_ECANCELLED;
 * DSMC_EDEADLINE).  `state`
 * may be NULL.  DSMC_EINVAL for an unknown id. */
int dsmc_poll(dsmc_server_t *server, uint64_t job_id, int *state);
/* Host steady-clock times in seconds of a job's submission, admission and
 * observed completion (0 while not reached). */
int dsmc_job_times(dsmc_server_t *server, uint64_t job_id, double *t_submit, double *t_start,
                   double *t_done);
/* Forget a finished job (DONE or FAILED): its record is freed and its id
 * becomes unknown (DSMC_EINVAL from then on).  A long-running server keeps one
 * record per submitted job until it is released or the server is destroyed.
 * Returns DSMC_OK, DSMC_EAGAIN if the job is still queued or running,
 * DSMC_EINVAL for an unknown id. */
int dsmc_job_release(dsmc_server_t *server, uint64_t job_id);

/* Kernel timings of a plan created with DSMC_PLAN_PROFILE, accumulated over
 * every dsmc_smooth / dsmc_smooth_batch since the previous dsmc_plan_profile
 * call: synchronises the stream, fills per-kernel-class totals (HIP events
 * recorded around each launch on the plan's stream) and restarts the
 * accumulation.  Classes: 0 leaves, 1 pair rows, 2 sampling, 3 output. */
#define DSMC_NUM_KERNEL_CLASSES 4
typedef struct dsmc_profile {
  int launches[DSMC_NUM_KERNEL_CLASSES];
  double ms[DSMC_NUM_KERNEL_CLASSES];
  double pairs; /* algorithmic pair evaluations: (K-1) N^2 summed over series */
  double rescued_rows; /* rows whose sum left the fp32 range and were recomputed with
                          their exact maximum as shift (counted once per combine) */
} dsmc_profile;
int dsmc_plan_profile(dsmc_plan_t *plan, dsmc_profile *out);

/* The combine tree the library runs for a series of K points (Algorithm 6:
 * at level l, adjacent blocks 2k and 2k+1 of the previous level are combined;
 * a trailing block without a right neighbour passes through).  Host only, no
 * device work.  Writes K - 1 combines, ordered by level, as left block
 * [a, c), right block [c, b) and level; cap is the length of the four
 * caller-owned arrays.  Returns the number of combines, or DSMC_EINVAL. */
int dsmc_schedule(int K, int cap, int32_t *a, int32_t *c, int32_t *b, int32_t *level);

/* Message describing the last error on this thread ("" if none). */
const char *dsmc_last_error(void);

/* Failure-injection hook for tests of the error paths (not part of the
 * method): from this call on, the k-th (0-based) device allocation that
 * dsmc_plan makes for its workspace fails as an out-of-memory hipMalloc
 * would.  That dsmc_plan then returns DSMC_ENOMEM with *out = NULL, having
 * freed every allocation it had made.  The hook fires once and then turns
 * itself off; k < 0 turns it off without firing.  Process-wide (one counter
 * for all threads and devices); calls of dsmc_plan that overlap with it on
 * several threads may see the failure at any one of them.  Returns DSMC_OK. */
int dsmc_debug_fail_allocation(int k);

#ifdef __cplusplus
}
#endif

#endif /* DSMC_H */
