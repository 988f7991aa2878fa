/*
 * mlmc.h -- C ABI of the MI355X (gfx950) multilevel Monte Carlo library.
 *
 * What it computes (D. J. Higham, "An Introduction to Multilevel Monte Carlo
 * for Option Valuation"):
 *   E[h(X(T))] for an Ito SDE dX = f(X) dt + g(X) dW (Sec. 2, eq. (eq:sde)),
 *   discretised by Euler--Maruyama (eq. (eq:em)) on levels with step
 *   dt_l = M^-l T (Sec. 5, eq. (eq:mlmc:Dtl)), estimated through the
 *   telescoping sum E[P_L] = E[P_0] + sum_l E[P_l - P_{l-1}]
 *   (eq. (eq:mlmc:ident)) with independent level estimators Yhat_l
 *   (eqs. (eq:mlmc:Yzero), (eq:Yldef)) whose fine and coarse paths share one
 *   Brownian path, the coarse increments being sums of M fine ones.
 *
 * Conventions for every entry point:
 *   - returns an mlmc_status; 0 = success.  Nothing aborts or throws across
 *     the ABI.  On failure a message is available from mlmc_last_error().
 *   - structs and host arrays belong to the caller and are only read or
 *     written during the call.  The context owns every device buffer it
 *     allocates.  Arguments named d_* are caller-owned DEVICE pointers on the
 *     context's device; all others are host pointers.
 *   - a context is not thread-safe: use one per host thread.  Calls are
 *     enqueued on the context's stream (mlmc_set_stream) and synchronise it
 *     before returning results to host memory, except mlmc_run: it returns
 *     once the device has published the final driver state (with kernel
 *     timing off, work of its own that changes nothing may still be queued;
 *     later work on the stream is ordered after it).
 *   - random numbers: Philox4x32-10 keyed by the 64-bit seed; sample s of
 *     level l is a pure function of (seed, l, s), so results do not depend on
 *     the launch configuration except for the order of FP64 atomic additions
 *     (relative differences of order 1e-16).  On GBM levels whose paths are
 *     split across lanes (a choice made from the call's N) an fp32 path is
 *     rounded differently from the one-lane evaluation, by a few units in
 *     the last place.
 */
#ifndef MLMC_H
#define MLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MLMC_OK = 0,
    MLMC_ENOTCONV = 1,    /* warning: L_max reached before the bias test
                             passed; the estimate is still returned          */
    MLMC_EINVAL = -1,     /* invalid argument                                */
    MLMC_ENOMEM = -2,     /* device or host allocation failed                */
    MLMC_EDEVICE = -3,    /* HIP runtime error                               */
    MLMC_ENONFINITE = -4  /* some samples were not finite; they are counted
                             in n_nonfinite and left out of the sums          */
} mlmc_status;

/* Models (eq. (eq:sde)); GBM is the model of Sec. 6. */
typedef enum { MLMC_GBM = 0, MLMC_HESTON = 1 } mlmc_model_kind;
typedef enum { MLMC_EULER = 0, MLMC_MILSTEIN = 1 } mlmc_scheme;
/* Payoffs: European call (Sec. 5), arithmetic Asian and floating-strike
 * lookback (named in Sec. 7.1), digital with the tie rule of Sec. 6. */
typedef enum {
    MLMC_CALL = 0, MLMC_ASIAN = 1, MLMC_LOOKBACK = 2, MLMC_DIGITAL = 3, MLMC_DIGITAL_COND = 4
} mlmc_payoff_kind;

typedef struct {
    int kind;                       /* mlmc_model_kind */
    double S0, r, sigma, T;         /* GBM: dS = r S dt + sigma S dW */
    double kappa, theta, xi, rho, v0;
    /* Heston: dS = r S dt + sqrt(v) S dW1, dv = kappa (theta - v) dt +
     * xi sqrt(v) dW2, corr(dW1, dW2) = rho, v(0) = v0; stepped by
     * full-truncation Euler (sigma unused).                               */
    int scheme;      /* mlmc_scheme.  MLMC_EULER: Euler--Maruyama, eq. (eq:em).
                        MLMC_MILSTEIN (GBM only): the Euler step plus
                        sigma^2 S (dW^2 - dt) / 2 -- the higher strong order
                        scheme of Sec. 3 and the remark after the complexity
                        theorem of Sec. 5 (beta = 2 > gamma = 1).            */
    int antithetic;  /* 1: on levels l >= 1 the fine path has an antithetic
                        twin driven by the same increments in reverse order
                        inside every coarse step (Sec. 7, antithetic
                        variables in the multilevel estimator), and
                        Y = (P_f + P_f^a)/2 - (P_c + P_c^a)/2, where the twin
                        coarse path differs from the coarse path only in the
                        lookback's refined minimum.  Cost per sample
                        2 n_f + n_c.  Not with the standard Monte Carlo
                        comparator, the control variate or the persistent
                        kernel (MLMC_EINVAL).                                 */
} mlmc_model;

typedef struct {
    int kind;                       /* mlmc_payoff_kind */
    double K;                       /* strike (unused by the lookback) */
    double payout;                  /* digital cash amount (1 or 100) */
    /* All payoffs are discounted by exp(-rT):
     *   call     max(S_N - K, 0)
     *   Asian    max(A - K, 0), A the trapezoid average over the path's grid
     *   lookback S_N - min S with a Brownian-bridge minimum on every step
     *   digital  payout if S_N > K, payout/2 if S_N == K, else 0
     *   conditional digital (Sec. 7, conditional Monte Carlo inside the
     *            multilevel estimator): the digital's expectation given every
     *            increment of the sample but the last fine one, computed
     *            exactly from the last step (Gaussian for Euler, a quadratic
     *            in the increment for Milstein); same mean as the digital on
     *            every level, far smaller level variances.  Not with the
     *            control variate.                                          */
} mlmc_payoff;

/* Sums of one level's samples, eq. (eq:Yldef): Y = P_l - P_{l-1}
 * (P_{-1} = 0), Pf = P_l (fine), Pc = P_{l-1} (coarse).
 * cost = N * (M^l + M^(l-1)) path steps (N at l = 0), the paper's cost
 * measure of Sec. 3.                                                        */
typedef struct {
    double sum_y, sum_y2, sum_pf, sum_pf2, sum_pc, sum_pc2;
    double cost;
    uint64_t n, n_nonfinite;
} mlmc_level_result;

typedef struct mlmc_ctx mlmc_ctx;
typedef struct mlmc_cv mlmc_cv;

/* Create a context on HIP device `device` (its own non-blocking stream).
 * MLMC_EDEVICE if the device is absent or not gfx950.                      */
mlmc_status mlmc_ctx_create(int device, mlmc_ctx** out);
/* Frees every device buffer of the context; NULL is accepted. */
mlmc_status mlmc_ctx_destroy(mlmc_ctx* ctx);
/* Use `hip_stream` (a hipStream_t, e.g. torch.cuda.current_stream()
 * .cuda_stream) for all later work; NULL restores the context's own.  Waits
 * for the work already enqueued on the previous stream (the context's
 * buffers are shared by all its launches); MLMC_EDEVICE if that work failed. */
mlmc_status mlmc_set_stream(mlmc_ctx* ctx, void* hip_stream);
/* Last error message of this context ("" if none); valid until the next call. */
const char* mlmc_last_error(const mlmc_ctx* ctx);
/* Fix the level kernel's launch shape: block in {64,128,256,512,1024},
 * paths per thread ppt in {1,2,4}.  block = 0 returns to the tuned/default
 * choice.  Results do not depend on it (see determinism above).  GBM levels
 * whose paths are too few to fill the device run each path on several lanes
 * (a choice made from N alone, whatever the shape).                         */
mlmc_status mlmc_set_launch(mlmc_ctx* ctx, int block, int ppt);

/* Kernel timing with HIP events on the context's stream.  Slots:
 *   0..15  level sampler launches at level l (per-level entry points and
 *          per-level driver iterations), 16 persistent all-levels launches
 *          (the batch graph of mlmc_levels_batch; the sampler kernel of the
 *          device-planned mlmc_run),
 *   17     driver update kernel (with the plan in the device-planned run),
 *   18     control-variate training steps.
 * fine_steps / coarse_steps: path steps those launches computed (a
 * device-planned run charges all of its steps to its first stamped sampler
 * launch: the host does not see the per-iteration batches).              */
#define MLMC_STAT_SLOTS 20
typedef struct {
    uint64_t launches;
    double ms;              /* summed event-measured duration */
    double fine_steps, coarse_steps;
} mlmc_kernel_stat;
/* on != 0: start recording every slot (clears the statistics); 0: stop. */
mlmc_status mlmc_set_timing(mlmc_ctx* ctx, int on);
/* Record only the slots whose bit is set in slot_mask (bit s = slot s; 0
 * stops, a non-zero mask clears the statistics).  Each timed launch carries
 * two events, a few microseconds of queue time, so a caller that wants one
 * kernel's duration without slowing the rest times that slot alone.
 * MLMC_EINVAL for bits at or above MLMC_STAT_SLOTS.                          */
mlmc_status mlmc_set_timing_mask(mlmc_ctx* ctx, uint32_t slot_mask);
/* Time one launch in `stride` of each timed slot (the 1st, (stride+1)-th,
 * ... launch of the slot since the mask was last set; 1, the default, times
 * every launch).  A timed launch costs ~10 us of queue time, so a caller that
 * wants a slot's average duration over a long run without slowing it in
 * proportion samples it.  MLMC_EINVAL for 0.                               */
mlmc_status mlmc_set_timing_stride(mlmc_ctx* ctx, uint32_t stride);
/* paused != 0: stamp no launch until called with 0 (the mask, the stride
 * count and the statistics are kept; no wait for the stream).  A caller
 * stamps whole calls, e.g. every k-th mlmc_run with every launch of it, by
 * pausing around the others.                                               */
mlmc_status mlmc_set_timing_paused(mlmc_ctx* ctx, int paused);
/* Copy MLMC_STAT_SLOTS statistics into out (host array). */
mlmc_status mlmc_kernel_stats(mlmc_ctx* ctx, mlmc_kernel_stat* out);

/* Autotuner: times every block size {64..1024} x samples-per-lane {1,2,4}
 * (fp64: 1) of the level sampler on 2^25 fine path steps (median of five
 * launches) for seven level classes (levels 0..5 each, deeper levels at
 * level 6) and keeps the fastest for this (model kind, scheme,
 * antithetic flag, payoff, precision, M); later launches use it unless
 * mlmc_set_launch fixed a shape.  A launch with fewer samples than 256 lanes
 * per compute unit at the tuned ppt takes ppt 1, and a smaller launch halves
 * ppt, then the block, until it has a block per compute unit and two waves
 * per SIMD.  Results are cached in the JSON file
 * cache_path (or $MLMC_TUNE_CACHE; NULL/"" and no variable: no cache) under
 * a key of GPU architecture, compute-unit count and HIP runtime version, and
 * read back instead of measured when present.                             */
mlmc_status mlmc_autotune(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff, int M,
                          int precision, const char* cache_path);
/* Shape the tuner chose for level l (block = ppt = 0 if none). */
mlmc_status mlmc_tuned_shape(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff,
                             int l, int M, int precision, int* block, int* ppt);

/* Level estimator sums (eqs. (eq:mlmc:Yzero), (eq:Yldef)).
 *   l >= 0, M in {2, 4}, M^l <= 4^8 * 4 (262144 steps), N >= 0 paths
 *   seed: Philox key; path_offset: index of the first sample, so further
 *   calls extend the same sequence of independent samples;
 *   precision: 32 (fp32 paths, fp64 sums) or 64 (fp64 throughout);
 *   cv: learned control variate (NULL for plain MLMC; requires precision 32).
 * Returns MLMC_ENONFINITE (sums still valid) if any Y was not finite.     */
mlmc_status mlmc_level(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff,
                       int l, int M, uint64_t N, uint64_t seed, uint64_t path_offset,
                       int precision, const mlmc_cv* cv, mlmc_level_result* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sums of
 * mlmc_level (same model, payoff, l, M, N, seed, path_offset, precision, no
 * control variate) with no context and no allocation.  Runs on the CURRENT
 * HIP device, enqueued on `hip_stream` (a hipStream_t of that device; NULL =
 * its null stream), and does not wait: the result is written to d_out, a
 * caller-owned DEVICE pointer to one mlmc_level_result, when the stream
 * reaches it.  Non-finite samples are counted in d_out->n_nonfinite (no
 * MLMC_ENONFINITE, the call does not read the result back).
 * Scratch: the partial sums go to one group of 64 records (4 KiB) in a static
 * device array, one per device, held until the process ends; that group
 * serves any N <= 2^40 (MLMC_EINVAL beyond, as for mlmc_level).  Every call
 * on a device uses the same array, cleared by a fill kernel at the start of
 * the call: calls that overlap on one device (other streams, other host
 * threads) race and must be ordered by the caller.  Kernel launches only (no
 * memset or copy nodes), so the call can be captured into a graph.
 * err (may be NULL): a caller buffer of err_len bytes that receives the
 * reason of a failure ("" on success).  MLMC_EINVAL for bad arguments,
 * MLMC_EDEVICE for a HIP error (no current device, launch failure).        */
mlmc_status mlmc_level_noalloc(const mlmc_model* model, const mlmc_payoff* payoff, int l, int M,
                               uint64_t N, uint64_t seed, uint64_t path_offset, int precision,
                               void* hip_stream, mlmc_level_result* d_out, char* err,
                               size_t err_len);

/* Same samples as mlmc_level, per path: d_pf[i] = P_l and d_pc[i] = P_{l-1}
 * of sample path_offset + i, i < N (fp64 device arrays of N entries).
 * For testing; out may be NULL.                                             */
mlmc_status mlmc_level_paths(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff,
                             int l, int M, uint64_t N, uint64_t seed, uint64_t path_offset,
                             int precision, const mlmc_cv* cv, double* d_pf, double* d_pc,
                             mlmc_level_result* out);

/* Raw generator words as the sampler draws them: for paths s = s0 .. s0+npaths-1
 * and blocks j < nblocks, d_out[(s - s0) * nblocks * 4 + 4 j + w] is word w of
 * Philox4x32-10 at counter (j, s mod 2^32, level + 256 (s >> 32), stream) with
 * key (seed mod 2^32, seed >> 32).  d_out: uint32 device array.            */
mlmc_status mlmc_philox_words(mlmc_ctx* ctx, uint64_t seed, int level, uint64_t s0,
                              uint32_t stream, uint32_t nblocks, uint64_t npaths,
                              uint32_t* d_out);

/* Standard normals as the sampler draws them (Box--Muller on word pairs),
 * dim 1: d_out[(s - s0) * nsteps + n] = z_n; dim 2: two factors per step,
 * d_out[(s - s0) * 2 nsteps + 2 n + f].  precision 32 or 64; fp64 output. */
mlmc_status mlmc_normals(mlmc_ctx* ctx, uint64_t seed, int level, uint64_t s0, uint32_t stream,
                         int dim, int nsteps, uint64_t npaths, int precision, double* d_out);

/* Standard Monte Carlo comparator: sums of P_L alone (no coupling) over
 * N samples from an independent stream (Sec. 3's estimator a_M).          */
mlmc_status mlmc_stdmc(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff,
                       int L, int M, uint64_t N, uint64_t seed, uint64_t path_offset,
                       int precision, mlmc_level_result* out);

/* Persistent all-levels form (fp32 paths).  Samples every (payoff, level)
 * of one MLMC iteration -- levels 0..L, npayoffs payoffs on one model -- in
 * ONE launch of a persistent kernel, replayed from a captured HIP graph:
 * a plan kernel cuts the samples into items of about equal cost (deepest
 * level first), resident blocks take them (block b item b, the rest from
 * an atomic counter).
 *   N[k * (L+1) + l]: samples of payoff k at level l (0 allowed);
 *   offsets: same layout, first sample index (NULL = all 0);
 *   out[k * (L+1) + l]: the level sums, identical in law (and, up to fp64
 *   summation order, in value) to mlmc_level with the same arguments.
 * 1 <= npayoffs <= 4, L < 16.                                               */
mlmc_status mlmc_levels_batch(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoffs,
                              int npayoffs, int M, int L, const uint64_t* N,
                              const uint64_t* offsets, uint64_t seed, mlmc_level_result* out);
/* Launch shape of the persistent kernel: block in {64..1024}, ppt in
 * {1,2,4}, blocks_per_cu resident blocks per compute unit; block = 0 returns
 * to the tuned/default shape.                                               */
mlmc_status mlmc_set_persistent_launch(mlmc_ctx* ctx, int block, int ppt, int blocks_per_cu);

/* Autotuner of the persistent form: times mlmc_levels_batch for these
 * payoffs, M and L at N_l = 2^24 M^-l (at least 1) for every block size
 * {128, 256, 512} x samples per lane {1, 2, 4} x resident blocks per compute
 * unit {2, 4, 8} with at most 2048 threads per compute unit (median of three
 * after a capture run) and sets the fastest with mlmc_set_persistent_launch.
 * Results do not depend on the shape (see determinism above).  Cached like
 * mlmc_autotune's (cache_path, else $MLMC_TUNE_CACHE) under the machine key
 * and (model kind, scheme, M, L, npayoffs, every payoff kind); a cached
 * shape is set without measuring.  Arguments as for mlmc_levels_batch;
 * shape (host, 3 ints, may be NULL) receives block, ppt, blocks_per_cu.    */
mlmc_status mlmc_autotune_persistent(mlmc_ctx* ctx, const mlmc_model* model,
                                     const mlmc_payoff* payoffs, int npayoffs, int M, int L,
                                     const char* cache_path, int* shape);

/* ---------------------------------------------------------------- driver
 * Sample counts N_l = ceil(2 eps^-2 sqrt(V_l/C_l) sum_k sqrt(V_k C_k)) for
 * l = 0..L (the optimisation of Sec. 5's "Constructive Upper Bound" remark,
 * with eps a root-mean-square error split evenly between bias^2 and
 * variance), computed on the device in FP64.  V, C, N: host arrays of L+1. */
mlmc_status mlmc_optimal_n(mlmc_ctx* ctx, int L, const double* V, const double* C, double eps,
                           double* N);

typedef struct {
    double eps;          /* target root-mean-square error (absolute units)   */
    int M;               /* refinement factor, 2 or 4                       */
    int L_min, L_max;    /* 1 <= L_min <= L_max <= 12                       */
    uint64_t n_pilot;    /* initial samples on each of levels 0..L_min      */
    uint64_t seed;
    int precision;       /* 32 or 64                                         */
    int persistent;      /* 0: one launch per level and iteration; 1: every
                            iteration is one launch of the persistent
                            all-levels sampler and one of a block that
                            absorbs the batch and plans the next; the host
                            enqueues each iteration before the previous
                            update is read (the device plans every batch),
                            and the one iteration queued past the last
                            prepares the start of a next run of the same
                            problem on this context (which then needs no
                            start kernel); the call returns before that
                            iteration has run                              */
    double alpha, beta;  /* assumed weak and variance rates (<= 0: 1 and 1) */
    const mlmc_cv* cv;   /* NULL: plain MLMC.  Needs precision 32, Euler
                            paths without the twin and a plain payoff; with
                            persistent 1 the tabulated form only
                            (mlmc_cv_set_tabulated; MLMC_EINVAL otherwise). */
    int cv_levels;       /* with cv: apply it on levels l < cv_levels only
                            (0 = every level).  Each level estimator keeps its
                            mean either way, so any split is unbiased; level 0
                            costs one network evaluation per launch, deeper
                            levels one per path step.                          */
} mlmc_run_opts;

#define MLMC_MAX_LEVELS 16

typedef struct {
    double estimate;     /* sum_l Yhat_l */
    double rmse_est;     /* sqrt(sum_l V_l/N_l + bias estimate^2)           */
    double wall_s;       /* wall-clock seconds of the call                   */
    int L, converged, iterations;
    uint64_t N[MLMC_MAX_LEVELS];
    double E[MLMC_MAX_LEVELS], V[MLMC_MAX_LEVELS], C[MLMC_MAX_LEVELS];
    double sum_y[MLMC_MAX_LEVELS], sum_y2[MLMC_MAX_LEVELS];
    double alpha, beta, gamma;   /* fitted rates of |E_l|, V_l, C_l (l >= 1) */
    double cost;                 /* total path steps                         */
    uint64_t n_nonfinite;
} mlmc_run_result;

/* Adaptive MLMC (Sec. 5 and its complexity theorem): starts with n_pilot
 * samples on levels 0..L_min, then repeatedly (i) samples the outstanding
 * dN_l, (ii) on the device, estimates E_l and V_l (for l >= 2 floored by
 * E_{l-1} M^-alpha and V_{l-1} M^-beta), sets N_l by mlmc_optimal_n and
 * schedules a level again when its shortfall exceeds 1% of its count,
 * (iii) when nothing is outstanding, tests the bias
 * max(|E_L|, |E_{L-1}| M^-alpha) / (M^alpha - 1) <= eps / sqrt(2), adding a
 * level (V_{L+1} = V_L M^-beta) if it fails.  Returns MLMC_ENOTCONV if L_max
 * is reached first (result still filled).                                    */
mlmc_status mlmc_run(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff,
                     const mlmc_run_opts* opts, mlmc_run_result* out);

/* Autotuner of the device-planned run (mlmc_run with opts->persistent = 1):
 * times whole runs of this model, payoff and opts (a warm-up, then the
 * median of three, all with opts->seed) for every persistent launch shape
 * of mlmc_autotune_persistent's candidate set and sets the fastest with
 * mlmc_set_persistent_launch.  The runs' batches are the tuned workload, so
 * the shape suits that configuration's launch sizes.  Cached like
 * mlmc_autotune's under the machine key and (model kind, scheme, payoff
 * kind, M, eps, L_min, L_max, precision, n_pilot, alpha, beta); a cached
 * shape is set without measuring.  shape (host, 3 ints, may be NULL)
 * receives block, ppt, blocks_per_cu.  MLMC_EINVAL unless persistent = 1. */
mlmc_status mlmc_autotune_run(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff,
                              const mlmc_run_opts* opts, const char* cache_path, int* shape);

/* ----------------------------------------------- randomised estimator
 * Rhee and Glynn's randomised multilevel estimator (cited in Sec. 7): each
 * of the N samples draws its level L with probability
 * p_l = (1 - q) q^l / (1 - q^(L_cap+1)), l = 0..L_cap, and contributes
 * Z = Y_L / p_L (eqs. (eq:mlmc:Yzero), (eq:Yldef)), so E[Z] = E[P_L_cap]
 * (eq. (eq:mlmc:ident)) without a bias test.  The variance is finite when
 * q > M^-beta and the expected cost when q < M^-1: use it with a scheme of
 * beta > 1 (MLMC_MILSTEIN), e.g. q = M^-1.5.  Level draws: word i mod 4 of
 * the generator block at counter (0, i / 4, 0, stream 7), u = ((x >> 8) +
 * 1/2) 2^-24, L = the first l with u < sum_{k <= l} p_k.  Level l then runs
 * on its samples 0 .. N_l - 1 of the ordinary sampler (stream 0).
 * L_cap <= 15 and within the level limits of M; 0 < q < 1; 1 <= N <= 2^40.
 * Host output; MLMC_ENONFINITE as for mlmc_level.                          */
typedef struct {
    double estimate;     /* (1/N) sum_l S1_l / p_l                          */
    double variance;     /* per-sample variance of Z                        */
    double rmse_est;     /* sqrt(variance / N)                              */
    double cost;         /* path steps                                      */
    double wall_s;
    int L_cap;
    uint64_t N[MLMC_MAX_LEVELS];       /* samples that drew each level     */
    double p[MLMC_MAX_LEVELS];
    double sum_y[MLMC_MAX_LEVELS], sum_y2[MLMC_MAX_LEVELS];
    uint64_t n_nonfinite;
} mlmc_rg_result;

mlmc_status mlmc_rhee_glynn(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff,
                            int M, int L_cap, double q, uint64_t N, uint64_t seed, int precision,
                            mlmc_rg_result* out);

/* ------------------------------------------------------- control variate
 * Learned martingale control variate (Sec. 5, "Exploiting Structure": a
 * control variate with known mean).  Each payoff P of a level sample is
 * replaced by P - sum_n phi(t_n, X_n) dW1_n on its own grid (fine path:
 * fine steps and increments; coarse path: coarse steps and summed
 * increments), phi evaluated at the left point, so the sum has mean exactly
 * zero and every level keeps its expectation.  phi is an MLP
 * in_dim -> 64 -> 64 -> 1 with tanh, inputs (t/T, ln(S/S0)/(sref sqrt T)
 * [, (v - theta)/theta]) and output scale sref S0 (sref = sigma for GBM,
 * sqrt(theta) for Heston); for Heston it multiplies dW1 only.  Parameters
 * are fp32 (layout W1[64][in_dim], b1[64], W2[64][64], b2[64], w3[64], b3);
 * the 64x64 layer runs on bf16 matrix cores with fp32 accumulation.
 * A network belongs to the context it was created on.                    */
/* in_dim 2 (GBM) or 3 (Heston), hidden 64; Xavier-uniform weights from
 * Philox stream 6 keyed by init_seed (word i % 4 of block i / 4 for
 * parameter i), zero biases.                                              */
mlmc_status mlmc_cv_create(mlmc_ctx* ctx, int in_dim, int hidden, uint64_t init_seed,
                           mlmc_cv** out);
mlmc_status mlmc_cv_destroy(mlmc_cv* cv);
/* Number of parameters (4417 for in_dim 2, 4481 for 3); 0 for NULL. */
size_t mlmc_cv_nparams(const mlmc_cv* cv);
/* Copy the fp32 parameters to / from a host array of exactly nparams. */
mlmc_status mlmc_cv_get_params(const mlmc_cv* cv, float* host, size_t n);
mlmc_status mlmc_cv_set_params(mlmc_cv* cv, const float* host, size_t n);

/* Tabulated evaluation (on = 1) or the network itself (on = 0, the default)
 * in the estimation samplers (mlmc_level and mlmc_run with this network).
 * Tabulated: phi is evaluated once per parameter change and model on a grid
 * -- rows t_j = j T / R, stock values S_i = s_lo + i (s_hi - s_lo) / (ns - 1)
 * with s_lo, s_hi = S0 exp(-+4 sref sqrt T), and for Heston variances
 * v_k = k v_hi / (nv - 1), v_hi = 4 max(theta, v0); GBM R = 256, ns = 32,
 * nv = 1; Heston R = 16, ns = 16, nv = 32 -- and the samplers interpolate it
 * linearly in S (bilinearly in S and v; points beyond the grid take its
 * edge) in row floor(n R / n_f) for the left point of fine step n (coarse
 * step m: n = m M).  Any function of (t_n, X_n) keeps the control variate's
 * mean at zero, so the level means are unchanged; the table only changes the
 * variance removed and the cost (a few operations per point instead of a
 * network evaluation).  Training always evaluates the network itself.        */
mlmc_status mlmc_cv_set_tabulated(mlmc_cv* cv, int on);
/* The table of the tabulated form for `model` (built if needed), as
 * host[(j nv + k) ns + i] = phi(t_j, S_i, v_k); dims (host, 3 ints, may be
 * NULL) receives R, nv, ns.  host may be NULL (dims only); otherwise n must
 * be R nv ns.                                                               */
mlmc_status mlmc_cv_get_table(mlmc_cv* cv, const mlmc_model* model, float* host, size_t n,
                              int* dims);

/* Training objective on B samples per level l = 0..lmax from the training
 * streams (Philox streams 2 and 3, disjoint from estimation), sample indices
 * step * B .. step * B + B - 1:
 *   loss = sum_l sqrt(C_l Var_batch(Y_l)),  C_l the level cost,
 * (the MLMC cost functional, total cost ~ (sum_l sqrt(V_l C_l))^2) and its
 * gradient with respect to the fp32 parameters, computed by the device's
 * forward pass (per-sample Y), per-sample weights dLoss/dY, and a backward
 * pass that regenerates every path from its counters.
 *   grad: host array of nparams floats (may be NULL); var: lmax+1 batch
 *   variances (may be NULL); loss (may be NULL).  0 <= lmax <= 6,
 *   2 <= batch <= 2^24.                                                   */
mlmc_status mlmc_cv_loss_grad(mlmc_cv* cv, const mlmc_model* model, const mlmc_payoff* payoff,
                              int M, int lmax, uint64_t batch, uint64_t seed, uint64_t step,
                              float* grad, double* var, double* loss);
/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on
 * the objective above, each on fresh training samples (the step counter of
 * the network continues across calls).  loss_hist: host array of `steps`
 * losses (may be NULL).                                                    */
mlmc_status mlmc_cv_train(mlmc_cv* cv, const mlmc_model* model, const mlmc_payoff* payoff, int M,
                          int lmax, int steps, uint64_t batch, double lr, uint64_t seed,
                          float* loss_hist);

#ifdef __cplusplus
}
#endif
#endif
