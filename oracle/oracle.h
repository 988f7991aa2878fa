/*
 * CPU oracle for the multilevel Monte Carlo (MLMC) level sampler.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library never
 * links, includes or calls anything here, and nothing here is taken from the
 * GPU library: the two share no source, headers or constants.
 *
 * Everything is plain FP64 C, written to be read against the paper
 * (D. J. Higham, "An Introduction to Multilevel Monte Carlo for Option
 * Valuation"), section by section:
 *   - Euler--Maruyama, Sec. 2, eq. (eq:em);
 *   - level step sizes dt_l = M^-l T, Sec. 5, eq. (eq:mlmc:Dtl);
 *   - the level estimators, eqs. (eq:mlmc:Yzero) and (eq:Yldef), with the
 *     coarse path driven by sums of the fine Brownian increments and fresh
 *     random numbers for every level (Sec. 5, the paragraph after eq:Yldef);
 *   - cost = number of generator calls / coefficient evaluations (Sec. 3);
 *   - the choice of L and N_l (Sec. 5 "Constructive Upper Bound" remark and
 *     the complexity theorem), in the standard optimised form;
 *   - the European call and digital payoffs of Sec. 6, the Asian and lookback
 *     payoffs named in Sec. 7.1;
 *   - the control-variate idea of Sec. 5 ("Exploiting Structure") in the form
 *     of a discrete martingale sum phi(t_n, X_n) dW_n with a small MLP phi.
 * Items the paper leaves open (random number generator, stream layout,
 * Heston model, Asian/lookback definitions, the MLP, its training loss) are
 * documented at each function.
 *
 * Parity status of each function is stated in its comment; functions whose
 * result is not fixed by a closed form, an invariant or a brute-force check
 * say "parity unpinned".
 */
#ifndef MLMC_ORACLE_H
#define MLMC_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- models */
enum { ORC_GBM = 0, ORC_HESTON = 1 };
enum { ORC_CALL = 0, ORC_ASIAN = 1, ORC_LOOKBACK = 2, ORC_DIGITAL = 3, ORC_DIGITAL_COND = 4 };
/* Philox stream ids (counter word 3). */
enum { ORC_STREAM_NORMAL = 0, ORC_STREAM_BRIDGE = 1, ORC_STREAM_TRAIN_NORMAL = 2,
       ORC_STREAM_TRAIN_BRIDGE = 3, ORC_STREAM_STDMC = 4, ORC_STREAM_STDMC_BRIDGE = 5,
       ORC_STREAM_INIT = 6, ORC_STREAM_LEVEL_DRAW = 7 };

enum { ORC_EULER = 0, ORC_MILSTEIN = 1 };

typedef struct {
    int kind;             /* ORC_GBM or ORC_HESTON */
    double S0, r, sigma, T;               /* GBM: dS = r S dt + sigma S dW   */
    double kappa, theta, xi, rho, v0;     /* Heston variance parameters      */
    int scheme;           /* ORC_EULER, or ORC_MILSTEIN (GBM only)          */
    int antithetic;       /* 1: levels l >= 1 average the fine path with its
                             antithetic twin                                */
} orc_model;

typedef struct {
    int kind;             /* ORC_CALL, ORC_ASIAN, ORC_LOOKBACK, ORC_DIGITAL,
                             ORC_DIGITAL_COND                              */
    double K;             /* strike (unused by the floating lookback)       */
    double payout;        /* digital cash amount                            */
} orc_payoff;

/* Control variate network: phi(t, X) = out_scale * MLP(inputs).
 * Parameter vector layout (float64 here, fp32 master on the GPU):
 *   W1[H][D] (row-major), b1[H], W2[H][H] (row j = output unit), b2[H],
 *   w3[H], b3.   H = 64, D = 2 (GBM) or 3 (Heston).                      */
/* Tabulated form of the network (a reading; the paper has no network):
 * values[(j nv + k) ns + i] = phi(t_j, S_i, v_k) on the grid t_j = j T / rows,
 * S_i = s_lo + i (s_hi - s_lo)/(ns - 1), v_k = v_lo + k (v_hi - v_lo)/(nv - 1)
 * (nv = 1: no variance axis).  phi at a left point (t, S, v) is then read in
 * row floor(t rows / T) and interpolated linearly in S (bilinearly in S, v),
 * with S and v first clamped to the grid.  The grid for a model
 * (orc_cv_table_grid): s_lo, s_hi = S0 exp(-+4 sref sqrt T); GBM rows 256,
 * ns 32, nv 1; Heston rows 16, ns 16, nv 32, v in [0, 4 max(theta, v0)].   */
typedef struct {
    int rows, ns, nv;
    double s_lo, s_hi, v_lo, v_hi;
    const double *values;
} orc_cv_table;

typedef struct {
    int in_dim;           /* 2 or 3 */
    int hidden;           /* 64 */
    const double *params; /* in_dim*H + H + H*H + H + H + 1 values */
    int bf16_emulate;     /* 1: round W2 and the layer-1 activations to bf16
                             exactly where the GPU feeds its matrix cores     */
    const orc_cv_table *table;  /* non-NULL: phi is read from this table   */
} orc_cv;

typedef struct {
    double sum_y, sum_y2, sum_pf, sum_pf2, sum_pc, sum_pc2;
    double cost;          /* N * (n_f + n_c) path steps */
    uint64_t n, n_nonfinite;
} orc_level_result;

/* ------------------------------------------------------------------ RNG */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t x);
void orc_box_muller(uint32_t a, uint32_t b, double *z0, double *z1);
/* Counter words for Philox block j of path s at a level, in a stream. */
void orc_counter(uint32_t j, uint64_t s, int level, int stream, uint32_t ctr[4]);
/* Raw Philox words of path s: nblocks*4 words. */
void orc_path_words(uint64_t seed, int level, uint64_t s, int stream,
                    uint32_t nblocks, uint32_t *out);
/* Standard normals of path s: dim=1 -> z[n], n < nsteps;
 * dim=2 -> z[2n], z[2n+1] are the two factors of step n.  Paths needing
 * fewer than four normals share a generator block (see rng.c).           */
void orc_path_normals(uint64_t seed, int level, uint64_t s, int stream, int dim,
                      int nsteps, double *z);
/* Uniforms for the bridge minimum of step n (stream+1 of the normals). */
void orc_path_uniforms(uint64_t seed, int level, uint64_t s, int stream,
                       int nsteps, double *u);

/* -------------------------------------------------------------- sampler */
/* Coupled sample s of level l: fine path (M^l steps) and coarse path
 * (M^(l-1) steps, zero at l = 0).  Returns 0, or -1 for bad arguments.
 * stream: ORC_STREAM_NORMAL for estimation, ORC_STREAM_TRAIN_NORMAL for
 * control-variate training (bridge uniforms come from stream + 1).
 * cv may be NULL.  cvf/cvc (may be NULL) receive the control-variate sums
 * that were subtracted from pf/pc.                                         */
int orc_level_sample(const orc_model *m, const orc_payoff *p, int l, int M,
                     uint64_t seed, uint64_t s, int stream, const orc_cv *cv,
                     double *pf, double *pc, double *cvf, double *cvc);

/* Same dynamics, driven by given increments instead of the generator:
 * dw[nsteps*dim] Brownian increments (already scaled by sqrt(dt), second
 * factor uncorrelated), u[nsteps] bridge uniforms (may be NULL unless the
 * payoff is the lookback).  Returns the payoff of one path of nsteps steps
 * of size T/nsteps.  Used to pin the coupling.                             */
double orc_path_payoff(const orc_model *m, const orc_payoff *p, int nsteps,
                       const double *dw, const double *u);

/* Sums over paths s = offset .. offset+N-1 of level l (nthreads >= 1). */
int orc_level(const orc_model *m, const orc_payoff *p, int l, int M, uint64_t N,
              uint64_t seed, uint64_t offset, const orc_cv *cv, int nthreads,
              orc_level_result *out);
/* Per-path values of the same paths (pf[i], pc[i], i < N). */
int orc_level_paths(const orc_model *m, const orc_payoff *p, int l, int M,
                    uint64_t N, uint64_t seed, uint64_t offset, const orc_cv *cv,
                    int nthreads, double *pf, double *pc);

/* Standard Monte Carlo at level L (stream ORC_STREAM_STDMC): sums of P_L. */
int orc_stdmc(const orc_model *m, const orc_payoff *p, int L, int M, uint64_t N,
              uint64_t seed, uint64_t offset, int nthreads, orc_level_result *out);

/* --------------------------------------------------------------- driver */
/* Optimal sample counts N_l = ceil(2 eps^-2 sqrt(V_l/C_l) sum_k sqrt(V_k C_k)),
 * l = 0..L.                                                                  */
void orc_optimal_n(int L, const double *V, const double *C, double eps, double *N);
/* Level cost in path steps: 1 at l = 0, M^l + M^(l-1) above. */
double orc_level_cost(int l, int M, int antithetic);

typedef struct {
    double eps; int M, L_min, L_max; uint64_t n_pilot; uint64_t seed;
    double alpha, beta;   /* weak / variance rates used by the bias test and
                             the extrapolation of a new level (<=0: defaults
                             1 and 1)                                           */
    int nthreads;
    const orc_cv *cv;
} orc_run_opts;

typedef struct {
    double estimate; int L; int converged; int iterations;
    uint64_t N[16]; double sum_y[16], sum_y2[16], V[16], E[16], C[16];
    double alpha, beta, gamma; double cost;
} orc_run_result;

int orc_mlmc_run(const orc_model *m, const orc_payoff *p, const orc_run_opts *o,
                 orc_run_result *out);
/* Randomised single-term estimator (rhee_glynn.c). */
typedef struct {
    double estimate;      /* (1/N) sum_l S1_l / p_l                          */
    double variance;      /* per-sample variance of Z = Y_L / p_L            */
    double cost;          /* path steps                                      */
    int Lc;
    uint64_t N[16];       /* samples that drew each level                    */
    double p[16], sum_y[16], sum_y2[16];
    uint64_t n_nonfinite;
} orc_rg_result;

void orc_rg_probabilities(double q, int Lc, double *p, double *F);
int orc_rg_level_counts(uint64_t seed, uint64_t N, double q, int Lc, uint64_t *counts);
int orc_rhee_glynn(const orc_model *m, const orc_payoff *p, int M, int Lc, double q, uint64_t N,
                   uint64_t seed, int nthreads, orc_rg_result *out);

/* Least-squares slope of log_M |y_l| against l over l = 1..L (y_l > 0). */
double orc_fit_rate(int L, const double *y, int M);

/* ---------------------------------------------------------- closed forms */
double orc_norm_cdf(double x);
double orc_bs_call(double S0, double K, double r, double sigma, double T);
double orc_bs_digital(double S0, double K, double r, double sigma, double T, double payout);
double orc_lookback_float_call(double S0, double r, double sigma, double T);
double orc_geometric_asian_call(double S0, double K, double r, double sigma, double T);
double orc_heston_call(double S0, double K, double r, double T, double kappa,
                       double theta, double xi, double rho, double v0);
/* Exact Euler moments for the K = 0 payoff e^-rT S_N at level l:
 * out[0] = E[P_l], out[1] = Var[P_l - P_{l-1}] (Var[P_0] at l = 0).       */
void orc_euler_k0_moments(double S0, double r, double sigma, double T, int l, int M,
                          double out[2]);
/* One-step (level 0) Euler call: out[0] = E[P_0], out[1] = Var[P_0]. */
void orc_level0_call_moments(double S0, double K, double r, double sigma, double T,
                             double out[2]);

/* ------------------------------------------------------- control variate */
size_t orc_cv_nparams(int in_dim, int hidden);
/* Xavier-uniform weights from the init stream, zero biases. */
void orc_cv_init(int in_dim, int hidden, uint64_t init_seed, double *params);
/* Network inputs at (t, X): x[0] = t/T, x[1] = log(S/S0)/(sref sqrt T),
 * x[2] = (v - theta)/theta for Heston.                                       */
void orc_cv_inputs(const orc_model *m, double t, double S, double v, double *x);
double orc_cv_out_scale(const orc_model *m);
/* phi(t, X) for one point (includes out_scale); from cv->table if set. */
double orc_cv_phi(const orc_model *m, const orc_cv *cv, double t, double S, double v);
/* The grid of the tabulated form for model m (values left NULL). */
void orc_cv_table_grid(const orc_model *m, orc_cv_table *g);
/* Fill values (rows * nv * ns) with the network cv (its table ignored). */
void orc_cv_table_fill(const orc_model *m, const orc_cv *cv, const orc_cv_table *g,
                       double *values);
/* Accumulate g * d phi / d params into grad (includes out_scale). */
void orc_cv_phi_grad(const orc_model *m, const orc_cv *cv, double t, double S, double v,
                     double g, double *grad);

/* Training loss over levels 0..lmax with B paths per level drawn from the
 * training streams, path indices step*B + i:
 *   loss = sum_l sqrt(C_l * Var_batch(Y_l)),
 * and its gradient.  var_out[l] receives the batch variance.                */
double orc_cv_loss_grad(const orc_model *m, const orc_payoff *p, int M, int lmax,
                        uint64_t B, uint64_t seed, uint64_t step, const orc_cv *cv,
                        int nthreads, double *grad, double *var_out);
/* One Adam step (t = 1, 2, ...) on theta with moments m1, m2. */
void orc_adam(size_t n, double *theta, double *m1, double *m2, const double *g,
              double lr, double b1, double b2, double eps, int t);

#ifdef __cplusplus
}
#endif
#endif
