/*
 * Oracle coupled level sampler (test infrastructure only).
 *
 * Level l uses n_f = M^l Euler--Maruyama steps of size h = T/n_f
 * (eq. (eq:mlmc:Dtl)); the coarse path of the same sample uses n_c = n_f/M
 * steps of size H = M h, and each coarse Brownian increment is the sum of the
 * M fine increments it covers (Sec. 5, the description of eq. (eq:Yldef) and
 * Fig. 2).  Level 0 has no coarse path (eq. (eq:mlmc:Yzero)).  Each level
 * draws its own random numbers: the level index is part of the Philox counter.
 *
 * The fine path and the coarse path are computed by two separate, plain loops
 * from the same array of fine increments, so that each can be read on its own
 * against eq. (eq:em).
 *
 * Models (the paper treats dX = f dt + g dW in general, eq. (eq:sde)):
 *   GBM    dS = r S dt + sigma S dW                   (Sec. 6 uses this model)
 *   Heston dS = r S dt + sqrt(v) S dW1,
 *          dv = kappa (theta - v) dt + xi sqrt(v) dW2, corr(W1, W2) = rho,
 *          stepped by full-truncation Euler (v+ = max(v, 0) in both the drift
 *          and the diffusion of v and in the diffusion of S) -- a reading, as
 *          the paper has no Heston model.
 * The S update is written in increment form S + S (r dt + vol dW).
 *
 * Milstein (GBM only; the scheme the complexity discussion of Sec. 5 and the
 * Sec. 3 remark on higher strong order refer to): the scalar Milstein step
 * for dX = f dt + g dW adds (1/2) g g' (dW^2 - dt) to the Euler step, which
 * for g(S) = sigma S is (1/2) sigma^2 S (dW^2 - dt).  The coarse path uses the
 * same step with the summed increment and step M h.
 *
 * Antithetic estimator (Sec. 7, "Further Developments": antithetic variables
 * embedded in the multilevel estimator; a reading, as the paper gives no
 * formula): on levels l >= 1 the fine path has an antithetic twin driven by
 * the same increments in reverse order inside every coarse step
 * (n = cM + k -> cM + M-1-k; for M = 2 the two halves swap), with the bridge
 * uniforms and the second factor permuted alike, so the twin has the fine
 * path's law and the coarse increments are unchanged.  The twin pair is the
 * twin fine path with the coarse path built from the twin's increments; the
 * coarse step values are the same up to summation order, but the lookback's
 * refinement of each coarse step follows the twin's fine path.  The level
 * sample averages the pair and its twin pair:
 * Y = (P_f + P_f^a)/2 - (P_c + P_c^a)/2, reported as P_f := (P_f + P_f^a)/2
 * and P_c := (P_c + P_c^a)/2.
 *
 * Payoffs, all discounted by exp(-rT):
 *   call     max(S_N - K, 0)                               (Sec. 5)
 *   digital  payout 1{S_N > K}, payout/2 when S_N = K       (Sec. 6)
 *   Asian    max(A - K, 0), A = (1/T) sum_n (S_n + S_{n+1}) dt / 2 over the
 *            path's own grid (trapezoid; a reading of Sec. 7.1's "Asian")
 *   lookback S_N - m, m the path minimum with a Brownian-bridge correction: on
 *            each step of a path with frozen coefficients the minimum of the
 *            bridge from x0 to x1 is sampled exactly as
 *            (x0 + x1 - sqrt((x1 - x0)^2 - 2 b^2 dt ln U)) / 2,
 *            b = vol * S at the step start, U uniform from the bridge stream.
 *            For the coarse path, each coarse step is refined at the fine
 *            times by the frozen-coefficient process driven by the fine
 *            Brownian increments, and the same formula is applied on each
 *            fine sub-interval with the same U as the fine path.  This samples
 *            the exact minimum of the frozen-coefficient process over the
 *            coarse step, so its law is the level-(l-1) fine construction's.
 *            (a reading of Sec. 7.1's "lookback")
 *
 * Conditional digital (Sec. 7: a conditional Monte Carlo approach inside
 * the multilevel estimator; a reading, as no formula is given): the digital
 * payoff is replaced by its expectation given every Brownian increment of
 * the sample except the last fine one, x = dW_last ~ N(0, h).  Both paths of
 * a sample condition on the same information.  Given that information the
 * last step of either path is a polynomial S_N = A + B x + C x^2 in x:
 *   fine, Euler:      A = S (1 + r h),  B = vol S,  C = 0;
 *   fine, Milstein:   A = S (1 + r h - sigma^2 h / 2),  B = sigma S,
 *                     C = sigma^2 S / 2;
 *   coarse, Euler:    A = S (1 + r H + vol w),  B = vol S,  C = 0;
 *   coarse, Milstein: A = S (1 + r H + sigma w + sigma^2 (w^2 - H) / 2),
 *                     B = sigma S (1 + sigma w),  C = sigma^2 S / 2,
 * with S the state at the start of the last step and w the sum of the other
 * M - 1 fine increments of the last coarse step.  P(S_N > K) is then
 * Phi((A - K)/(|B| sqrt h)) for C = 0, and for C > 0 the Gaussian mass
 * outside the roots x1 < x2 of C x^2 + B x + A - K (all of it when there
 * are none); Phi(z) = erfc(-z / sqrt 2) / 2, the digital's tie rule when
 * B = C = 0.  By the tower property each path's expectation is the plain
 * digital's, so the levels still telescope.
 *
 * Control variate: if cv is given, P is replaced by
 *   P - sum_n phi(t_n, X_n) dW1_n
 * on each path's own grid, fine with fine increments, coarse with coarse
 * increments (left-point evaluation, so each term has conditional mean zero).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include "oracle.h"

static double vol_of(const orc_model *m, double v)
{
    if (m->kind == ORC_GBM) return m->sigma;
    return sqrt(v > 0.0 ? v : 0.0);
}

/* One Euler--Maruyama step, eq. (eq:em), or for GBM with the Milstein
 * scheme the Euler step plus (1/2) g g' (dW^2 - dt).  dw1 drives S; dwp is
 * the second, uncorrelated factor, combined into
 * dW2 = rho dW1 + sqrt(1-rho^2) dwp.                                       */
static void em_step(const orc_model *m, double *S, double *v, double dt,
                    double dw1, double dwp)
{
    if (m->kind == ORC_GBM) {
        double S0 = *S;
        *S = S0 + S0 * (m->r * dt + m->sigma * dw1);
        if (m->scheme == ORC_MILSTEIN) {
            double g = m->sigma * S0, dg = m->sigma;
            *S += 0.5 * g * dg * (dw1 * dw1 - dt);
        }
        return;
    }
    double vp = *v > 0.0 ? *v : 0.0;
    double sv = sqrt(vp);
    double dw2 = m->rho * dw1 + sqrt(1.0 - m->rho * m->rho) * dwp;
    double S_new = *S + *S * (m->r * dt + sv * dw1);
    double v_new = *v + m->kappa * (m->theta - vp) * dt + m->xi * sv * dw2;
    *S = S_new;
    *v = v_new;
}

static double bridge_min(double x0, double x1, double b, double dt, double u)
{
    double d = x1 - x0;
    return 0.5 * (x0 + x1 - sqrt(d * d - 2.0 * b * b * dt * log(u)));
}

static double norm_cdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

/* payout P(A + B x + C x^2 > K), x ~ N(0, h), C >= 0. */
static double digital_given(const orc_payoff *p, double A, double B, double C, double h)
{
    double sd = sqrt(h);
    if (C > 0.0) {
        double c0 = A - p->K;
        double disc = B * B - 4.0 * C * c0;
        if (disc <= 0.0) return p->payout;            /* no real root: always above */
        double x1 = (-B - sqrt(disc)) / (2.0 * C);
        double x2 = (-B + sqrt(disc)) / (2.0 * C);
        return p->payout * (norm_cdf(x1 / sd) + norm_cdf(-x2 / sd));
    }
    if (B != 0.0) return p->payout * norm_cdf((A - p->K) / (fabs(B) * sd));
    if (A > p->K) return p->payout;
    if (A == p->K) return 0.5 * p->payout;
    return 0.0;
}

static double final_payoff(const orc_model *m, const orc_payoff *p, double S,
                           double asian_sum, double mn)
{
    double disc = exp(-m->r * m->T);
    /* a path that overflowed stays visible as a non-finite payoff */
    if (!isfinite(S)) return NAN;
    switch (p->kind) {
    case ORC_CALL:
        return disc * (S > p->K ? S - p->K : 0.0);
    case ORC_DIGITAL:
        if (S > p->K) return disc * p->payout;
        if (S == p->K) return disc * 0.5 * p->payout;
        return 0.0;
    case ORC_ASIAN: {
        double A = asian_sum / m->T;
        return disc * (A > p->K ? A - p->K : 0.0);
    }
    case ORC_LOOKBACK:
        return disc * (S - mn);
    }
    return NAN;
}

/* Fine path of nsteps steps of size dt, increments dw1[n], dwp[n]. */
static double fine_path(const orc_model *m, const orc_payoff *p, int nsteps, double dt,
                        const double *dw1, const double *dwp, const double *u,
                        const orc_cv *cv, double *cv_sum, double gw, double *grad)
{
    double S = m->S0, v = m->v0, asian = 0.0, mn = INFINITY, cvs = 0.0;
    double S_last = S, vol_last = 0.0;
    for (int n = 0; n < nsteps; ++n) {
        double t = n * dt;
        if (cv) cvs += orc_cv_phi(m, cv, t, S, v) * dw1[n];
        /* Y contains -sum phi dW on the fine path */
        if (cv && grad) orc_cv_phi_grad(m, cv, t, S, v, -gw * dw1[n], grad);
        double S_start = S;
        double vol = vol_of(m, v);
        S_last = S_start;
        vol_last = vol;
        em_step(m, &S, &v, dt, dw1[n], dwp ? dwp[n] : 0.0);
        asian += 0.5 * (S_start + S) * dt;
        if (p->kind == ORC_LOOKBACK) {
            double mk = bridge_min(S_start, S, vol * S_start, dt, u[n]);
            if (mk < mn) mn = mk;
        }
    }
    if (cv_sum) *cv_sum = cvs;
    if (p->kind == ORC_DIGITAL_COND) {
        if (!isfinite(S)) return NAN;
        double A = S_last + S_last * m->r * dt, B = vol_last * S_last, C = 0.0;
        if (m->scheme == ORC_MILSTEIN) {
            A -= 0.5 * m->sigma * m->sigma * S_last * dt;
            C = 0.5 * m->sigma * m->sigma * S_last;
        }
        return exp(-m->r * m->T) * digital_given(p, A, B, C, dt);
    }
    return final_payoff(m, p, S, asian, mn);
}

/* Coarse path: nc steps of size M*h from the sums of M fine increments. */
static double coarse_path(const orc_model *m, const orc_payoff *p, int M, int nc, double h,
                          const double *dw1, const double *dwp, const double *u,
                          const orc_cv *cv, double *cv_sum, double gw, double *grad)
{
    double H = M * h;
    double S = m->S0, v = m->v0, asian = 0.0, mn = INFINITY, cvs = 0.0;
    for (int c = 0; c < nc; ++c) {
        double dw1c = 0.0, dwpc = 0.0;
        for (int k = 0; k < M; ++k) {
            dw1c += dw1[c * M + k];
            if (dwp) dwpc += dwp[c * M + k];
        }
        double t = c * H;
        if (cv) cvs += orc_cv_phi(m, cv, t, S, v) * dw1c;
        /* Y contains +sum phi dW^c on the coarse path */
        if (cv && grad) orc_cv_phi_grad(m, cv, t, S, v, gw * dw1c, grad);
        double S_start = S;
        double vol = vol_of(m, v);
        if (p->kind == ORC_LOOKBACK) {
            /* frozen-coefficient process at the fine times inside the step */
            double w_part = 0.0, x_prev = S_start;
            for (int k = 0; k < M; ++k) {
                w_part += dw1[c * M + k];
                double tau = (k + 1) * h;
                double x_next = S_start + S_start * (m->r * tau + vol * w_part);
                if (m->scheme == ORC_MILSTEIN)   /* the coarse Milstein step to tau */
                    x_next += 0.5 * vol * vol * S_start * (w_part * w_part - tau);
                double mk = bridge_min(x_prev, x_next, vol * S_start, h, u[c * M + k]);
                if (mk < mn) mn = mk;
                x_prev = x_next;
            }
        }
        if (p->kind == ORC_DIGITAL_COND && c == nc - 1) {
            /* condition on all but the last fine increment of this step */
            double w = 0.0;
            for (int k = 0; k < M - 1; ++k) w += dw1[c * M + k];
            em_step(m, &S, &v, H, dw1c, dwpc);
            if (!isfinite(S)) return NAN;
            double A = S_start + S_start * (m->r * H + vol * w), B = vol * S_start, C = 0.0;
            if (m->scheme == ORC_MILSTEIN) {
                double s2 = m->sigma * m->sigma;
                A += 0.5 * s2 * S_start * (w * w - H);
                B = m->sigma * S_start * (1.0 + m->sigma * w);
                C = 0.5 * s2 * S_start;
            }
            if (cv_sum) *cv_sum = cvs;
            return exp(-m->r * m->T) * digital_given(p, A, B, C, h);
        }
        em_step(m, &S, &v, H, dw1c, dwpc);
        asian += 0.5 * (S_start + S) * H;
    }
    if (cv_sum) *cv_sum = cvs;
    return final_payoff(m, p, S, asian, mn);
}

static int check_args(const orc_model *m, const orc_payoff *p, int l, int M)
{
    if (!m || !p) return -1;
    if (m->kind != ORC_GBM && m->kind != ORC_HESTON) return -1;
    if (m->scheme != ORC_EULER && m->scheme != ORC_MILSTEIN) return -1;
    if (m->scheme == ORC_MILSTEIN && m->kind != ORC_GBM) return -1;
    if (m->antithetic != 0 && m->antithetic != 1) return -1;
    if (p->kind < ORC_CALL || p->kind > ORC_DIGITAL_COND) return -1;
    if (l < 0 || l > 20 || M < 2 || M > 16) return -1;
    double nf = pow((double)M, (double)l);
    if (nf > (double)(1 << 24)) return -1;
    return 0;
}

typedef struct {
    double *dw1, *dwp, *u, *z;
    double *dw1a, *dwpa, *ua;     /* antithetic twin's increments, uniforms */
    int cap;
} workspace;

static void ws_init(workspace *w, int nf)
{
    w->cap = nf;
    w->dw1 = malloc(sizeof(double) * nf);
    w->dwp = malloc(sizeof(double) * nf);
    w->u = malloc(sizeof(double) * nf);
    w->z = malloc(sizeof(double) * 2 * nf);
    w->dw1a = malloc(sizeof(double) * nf);
    w->dwpa = malloc(sizeof(double) * nf);
    w->ua = malloc(sizeof(double) * nf);
}

static void ws_free(workspace *w)
{
    free(w->dw1); free(w->dwp); free(w->u); free(w->z);
    free(w->dw1a); free(w->dwpa); free(w->ua);
}

/* One coupled sample using a caller workspace. */
static void sample_ws(const orc_model *m, const orc_payoff *p, int l, int M,
                      uint64_t seed, uint64_t s, int stream, const orc_cv *cv,
                      workspace *w, double *pf, double *pc, double *cvf, double *cvc,
                      double gw, double *grad)
{
    int nf = 1;
    for (int i = 0; i < l; ++i) nf *= M;
    double h = m->T / nf;
    double sqh = sqrt(h);
    int dim = (m->kind == ORC_HESTON) ? 2 : 1;
    orc_path_normals(seed, l, s, stream, dim, nf, w->z);
    for (int n = 0; n < nf; ++n) {
        w->dw1[n] = sqh * w->z[dim * n];
        w->dwp[n] = (dim == 2) ? sqh * w->z[dim * n + 1] : 0.0;
    }
    if (p->kind == ORC_LOOKBACK) orc_path_uniforms(seed, l, s, stream + 1, nf, w->u);
    double cf = 0.0, cc = 0.0;
    double Pf = fine_path(m, p, nf, h, w->dw1, dim == 2 ? w->dwp : NULL, w->u, cv, &cf,
                          gw, grad);
    double Pc = 0.0;
    if (l > 0)
        Pc = coarse_path(m, p, M, nf / M, h, w->dw1, dim == 2 ? w->dwp : NULL, w->u, cv, &cc,
                         gw, grad);
    if (m->antithetic && l > 0) {
        /* the twin: increments reversed inside each coarse step */
        for (int c = 0; c < nf / M; ++c)
            for (int k = 0; k < M; ++k) {
                int from = c * M + (M - 1 - k);
                w->dw1a[c * M + k] = w->dw1[from];
                w->dwpa[c * M + k] = w->dwp[from];
                w->ua[c * M + k] = w->u[from];
            }
        double Pa = fine_path(m, p, nf, h, w->dw1a, dim == 2 ? w->dwpa : NULL, w->ua, NULL, NULL,
                              0.0, NULL);
        double Pca = coarse_path(m, p, M, nf / M, h, w->dw1a, dim == 2 ? w->dwpa : NULL, w->ua,
                                 NULL, NULL, 0.0, NULL);
        Pf = 0.5 * (Pf + Pa);
        Pc = 0.5 * (Pc + Pca);
    }
    *pf = Pf - cf;
    *pc = (l > 0) ? Pc - cc : 0.0;
    if (cvf) *cvf = cf;
    if (cvc) *cvc = cc;
}

int orc_level_sample(const orc_model *m, const orc_payoff *p, int l, int M,
                     uint64_t seed, uint64_t s, int stream, const orc_cv *cv,
                     double *pf, double *pc, double *cvf, double *cvc)
{
    if (check_args(m, p, l, M)) return -1;
    if (cv && (m->antithetic || m->scheme != ORC_EULER)) return -1;
    int nf = 1;
    for (int i = 0; i < l; ++i) nf *= M;
    workspace w;
    ws_init(&w, nf);
    sample_ws(m, p, l, M, seed, s, stream, cv, &w, pf, pc, cvf, cvc, 0.0, NULL);
    ws_free(&w);
    return 0;
}

void orc_internal_path_grad(const orc_model *m, const orc_payoff *p, int l, int M,
                            uint64_t seed, uint64_t s, int stream, const orc_cv *cv,
                            double w, double *grad)
{
    int nf = 1;
    for (int i = 0; i < l; ++i) nf *= M;
    workspace ws;
    ws_init(&ws, nf);
    double pf, pc;
    sample_ws(m, p, l, M, seed, s, stream, cv, &ws, &pf, &pc, NULL, NULL, w, grad);
    ws_free(&ws);
}

double orc_path_payoff(const orc_model *m, const orc_payoff *p, int nsteps,
                       const double *dw, const double *u)
{
    int dim = (m->kind == ORC_HESTON) ? 2 : 1;
    double *dw1 = malloc(sizeof(double) * nsteps);
    double *dwp = malloc(sizeof(double) * nsteps);
    for (int n = 0; n < nsteps; ++n) {
        dw1[n] = dw[dim * n];
        dwp[n] = (dim == 2) ? dw[dim * n + 1] : 0.0;
    }
    double P = fine_path(m, p, nsteps, m->T / nsteps, dw1, dim == 2 ? dwp : NULL, u, NULL, NULL,
                         0.0, NULL);
    free(dw1);
    free(dwp);
    return P;
}

/* ------------------------------------------------------------ threading */
typedef struct {
    const orc_model *m; const orc_payoff *p; const orc_cv *cv;
    int l, M, stream, mode;      /* mode 0: level sums, 1: per-path, 2: stdmc */
    uint64_t seed, first, count;
    double *pf, *pc;             /* per-path outputs (mode 1), offset by index */
    orc_level_result res;
} job;

static void *run_job(void *arg)
{
    job *jb = (job *)arg;
    int nf = 1;
    for (int i = 0; i < jb->l; ++i) nf *= jb->M;
    workspace w;
    ws_init(&w, nf);
    memset(&jb->res, 0, sizeof(jb->res));
    for (uint64_t i = 0; i < jb->count; ++i) {
        uint64_t s = jb->first + i;
        double pf, pc;
        if (jb->mode == 2) {
            /* standard MC: only the fine path at level L, own stream */
            sample_ws(jb->m, jb->p, jb->l, jb->M, jb->seed, s, ORC_STREAM_STDMC, NULL, &w,
                      &pf, &pc, NULL, NULL, 0.0, NULL);
            pc = 0.0;
        } else {
            sample_ws(jb->m, jb->p, jb->l, jb->M, jb->seed, s, jb->stream, jb->cv, &w,
                      &pf, &pc, NULL, NULL, 0.0, NULL);
        }
        if (jb->mode == 1) {
            jb->pf[i] = pf;
            jb->pc[i] = pc;
            continue;
        }
        double y = pf - pc;
        if (!isfinite(y)) {
            jb->res.n_nonfinite++;
            continue;
        }
        jb->res.sum_y += y;
        jb->res.sum_y2 += y * y;
        jb->res.sum_pf += pf;
        jb->res.sum_pf2 += pf * pf;
        jb->res.sum_pc += pc;
        jb->res.sum_pc2 += pc * pc;
    }
    ws_free(&w);
    return NULL;
}

static void run_jobs(job *proto, uint64_t N, uint64_t offset, int nthreads,
                     orc_level_result *out)
{
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > N && N > 0) nthreads = (int)N;
    job *jobs = calloc((size_t)nthreads, sizeof(job));
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    uint64_t base = 0;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t cnt = N / nthreads + ((uint64_t)t < N % nthreads ? 1 : 0);
        jobs[t] = *proto;
        jobs[t].first = offset + base;
        jobs[t].count = cnt;
        if (proto->mode == 1) {
            jobs[t].pf = proto->pf + base;
            jobs[t].pc = proto->pc + base;
        }
        base += cnt;
        if (nthreads == 1) run_job(&jobs[t]);
        else pthread_create(&th[t], NULL, run_job, &jobs[t]);
    }
    if (nthreads > 1)
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    if (out) {
        memset(out, 0, sizeof(*out));
        for (int t = 0; t < nthreads; ++t) {   /* fixed combine order */
            out->sum_y += jobs[t].res.sum_y;
            out->sum_y2 += jobs[t].res.sum_y2;
            out->sum_pf += jobs[t].res.sum_pf;
            out->sum_pf2 += jobs[t].res.sum_pf2;
            out->sum_pc += jobs[t].res.sum_pc;
            out->sum_pc2 += jobs[t].res.sum_pc2;
            out->n_nonfinite += jobs[t].res.n_nonfinite;
        }
        out->n = N;
    }
    free(jobs);
    free(th);
}

int orc_level(const orc_model *m, const orc_payoff *p, int l, int M, uint64_t N,
              uint64_t seed, uint64_t offset, const orc_cv *cv, int nthreads,
              orc_level_result *out)
{
    if (check_args(m, p, l, M) || !out) return -1;
    if (cv && (m->antithetic || m->scheme != ORC_EULER)) return -1;
    job proto = {0};
    proto.m = m; proto.p = p; proto.cv = cv; proto.l = l; proto.M = M;
    proto.stream = ORC_STREAM_NORMAL; proto.mode = 0; proto.seed = seed;
    run_jobs(&proto, N, offset, nthreads, out);
    out->cost = (double)N * orc_level_cost(l, M, m->antithetic);
    return 0;
}

int orc_level_paths(const orc_model *m, const orc_payoff *p, int l, int M,
                    uint64_t N, uint64_t seed, uint64_t offset, const orc_cv *cv,
                    int nthreads, double *pf, double *pc)
{
    if (check_args(m, p, l, M) || !pf || !pc) return -1;
    if (cv && (m->antithetic || m->scheme != ORC_EULER)) return -1;
    job proto = {0};
    proto.m = m; proto.p = p; proto.cv = cv; proto.l = l; proto.M = M;
    proto.stream = ORC_STREAM_NORMAL; proto.mode = 1; proto.seed = seed;
    proto.pf = pf; proto.pc = pc;
    run_jobs(&proto, N, offset, nthreads, NULL);
    return 0;
}

int orc_stdmc(const orc_model *m, const orc_payoff *p, int L, int M, uint64_t N,
              uint64_t seed, uint64_t offset, int nthreads, orc_level_result *out)
{
    if (check_args(m, p, L, M) || !out) return -1;
    if (m->antithetic) return -1;    /* the twin belongs to level differences */
    job proto = {0};
    proto.m = m; proto.p = p; proto.l = L; proto.M = M;
    proto.mode = 2; proto.seed = seed;
    run_jobs(&proto, N, offset, nthreads, out);
    int nf = 1;
    for (int i = 0; i < L; ++i) nf *= M;
    out->cost = (double)N * nf;
    return 0;
}

/* Path steps per sample: n_f + n_c, with the antithetic twin 2 n_f + n_c. */
double orc_level_cost(int l, int M, int antithetic)
{
    if (l == 0) return 1.0;
    double nf = pow((double)M, (double)l);
    return (antithetic ? 2.0 : 1.0) * nf + pow((double)M, (double)(l - 1));
}
