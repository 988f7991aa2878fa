/*
 * Oracle learned control variate (test infrastructure only).
 *
 * The paper's Sec. 5 ("Exploiting Structure") describes the classic control
 * variate: estimate E[X - Y] and add E[Y], where E[Y] must be known.  Here Y
 * is the discrete martingale sum_n phi(t_n, X_n) dW_n, whose mean is exactly
 * zero for any phi evaluated at the left point of each step (phi(t_n, X_n) is
 * known at t_n and E[dW_n | F_{t_n}] = 0), so the level estimators of
 * eqs. (eq:mlmc:Yzero) and (eq:Yldef) keep their means while their variances
 * shrink.  phi is a small MLP; everything about it is a reading, since the
 * paper has only the concept:
 *   inputs  x0 = t/T, x1 = ln(max(S, S0 2^-40)/S0) / (sref sqrt T),
 *           x2 = (v - theta)/theta (Heston only),
 *           sref = sigma (GBM) or sqrt(theta) (Heston);
 *   network x -> tanh(W1 x + b1) -> tanh(W2 h1 + b2) -> w3 . h2 + b3;
 *   output  phi = sref S0 * network(x); for Heston it multiplies dW1 only.
 * Training loss over levels 0..lmax (the MLMC cost functional, since total
 * cost is proportional to (sum_l sqrt(V_l C_l))^2):
 *   loss = sum_l sqrt(C_l Var_batch(Y_l)).
 * Optimiser: Adam (Kingma and Ba 2015).
 *
 * bf16 emulation mode: W2, the layer-1 activations, and the layer-2 error
 * signal are rounded to bf16 (round to nearest even, via fp32) exactly where
 * a bf16 matrix unit consumes them; all other arithmetic stays FP64.
 *
 * Pins: gradients against FP64 central finite differences; the level-0
 * optimum (one step, so phi(0, S0) is a scalar c with the closed-form
 * optimum Cov(P_0, dW)/T); mean-zero of the control-variate sum.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include "oracle.h"

static double bf16_round(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

size_t orc_cv_nparams(int in_dim, int hidden)
{
    return (size_t)in_dim * hidden + hidden + (size_t)hidden * hidden + hidden + hidden + 1;
}

typedef struct {
    const double *W1, *b1, *W2, *b2, *w3, *b3;
} net_view;

static net_view view_of(const double *p, int D, int H)
{
    net_view v;
    v.W1 = p;
    v.b1 = v.W1 + (size_t)D * H;
    v.W2 = v.b1 + H;
    v.b2 = v.W2 + (size_t)H * H;
    v.w3 = v.b2 + H;
    v.b3 = v.w3 + H;
    return v;
}

void orc_cv_init(int in_dim, int hidden, uint64_t init_seed, double *params)
{
    size_t n = orc_cv_nparams(in_dim, hidden);
    uint32_t nblocks = (uint32_t)((n + 3) / 4);
    uint32_t *w = malloc(sizeof(uint32_t) * 4 * nblocks);
    orc_path_words(init_seed, 0, 0, ORC_STREAM_INIT, nblocks, w);
    int D = in_dim, H = hidden;
    double a1 = sqrt(6.0 / (D + H)), a2 = sqrt(6.0 / (H + H)), a3 = sqrt(6.0 / (H + 1));
    size_t i = 0;
    for (size_t q = 0; q < (size_t)D * H; ++q, ++i) params[i] = a1 * (2.0 * orc_u01(w[i]) - 1.0);
    for (int q = 0; q < H; ++q, ++i) params[i] = 0.0;
    for (size_t q = 0; q < (size_t)H * H; ++q, ++i) params[i] = a2 * (2.0 * orc_u01(w[i]) - 1.0);
    for (int q = 0; q < H; ++q, ++i) params[i] = 0.0;
    for (int q = 0; q < H; ++q, ++i) params[i] = a3 * (2.0 * orc_u01(w[i]) - 1.0);
    params[i] = 0.0;
    free(w);
}

static double sref_of(const orc_model *m)
{
    return m->kind == ORC_GBM ? m->sigma : sqrt(m->theta);
}

double orc_cv_out_scale(const orc_model *m) { return sref_of(m) * m->S0; }

void orc_cv_inputs(const orc_model *m, double t, double S, double v, double *x)
{
    double floor_s = m->S0 * ldexp(1.0, -40);
    double s = S > floor_s ? S : floor_s;
    x[0] = t / m->T;
    x[1] = log(s / m->S0) / (sref_of(m) * sqrt(m->T));
    if (m->kind == ORC_HESTON) x[2] = (v - m->theta) / m->theta;
}

#define HMAX 128

typedef struct {
    double x[3], h1[HMAX], h1q[HMAX], h2[HMAX], y;
} fwd_cache;

static void forward(const orc_model *m, const orc_cv *cv, double t, double S, double v,
                    fwd_cache *c)
{
    int D = cv->in_dim, H = cv->hidden;
    net_view nv = view_of(cv->params, D, H);
    orc_cv_inputs(m, t, S, v, c->x);
    for (int k = 0; k < H; ++k) {
        double a = nv.b1[k];
        for (int d = 0; d < D; ++d) a += nv.W1[k * D + d] * c->x[d];
        c->h1[k] = tanh(a);
        c->h1q[k] = cv->bf16_emulate ? bf16_round(c->h1[k]) : c->h1[k];
    }
    double y = nv.b3[0];
    for (int j = 0; j < H; ++j) {
        double a = nv.b2[j];
        for (int k = 0; k < H; ++k) {
            double w = cv->bf16_emulate ? bf16_round(nv.W2[j * H + k]) : nv.W2[j * H + k];
            a += w * c->h1q[k];
        }
        c->h2[j] = tanh(a);
        y += nv.w3[j] * c->h2[j];
    }
    c->y = y;
}

static double clamp(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* Interpolate the table at (t, S, v): the row of the last grid time at or
 * before t, then linear in S (and in v) between the two grid points around
 * the clamped coordinate. */
static double table_value(const orc_model *m, const orc_cv_table *g, double t, double S, double v)
{
    int j = (int)floor(t / m->T * g->rows + 1e-9);
    if (j > g->rows - 1) j = g->rows - 1;
    double u = (S - g->s_lo) / ((g->s_hi - g->s_lo) / (g->ns - 1));
    u = isnan(u) ? 0.0 : clamp(u, 0.0, g->ns - 1);
    int i = (int)u < g->ns - 2 ? (int)u : g->ns - 2;
    double f = u - i;
    const double *row = g->values + (size_t)j * g->nv * g->ns;
    if (g->nv == 1) return (1.0 - f) * row[i] + f * row[i + 1];
    double w = (v - g->v_lo) / ((g->v_hi - g->v_lo) / (g->nv - 1));
    w = isnan(w) ? 0.0 : clamp(w, 0.0, g->nv - 1);
    int k = (int)w < g->nv - 2 ? (int)w : g->nv - 2;
    double e = w - k;
    const double *r0 = row + (size_t)k * g->ns, *r1 = r0 + g->ns;
    double a = (1.0 - f) * r0[i] + f * r0[i + 1];
    double b = (1.0 - f) * r1[i] + f * r1[i + 1];
    return (1.0 - e) * a + e * b;
}

double orc_cv_phi(const orc_model *m, const orc_cv *cv, double t, double S, double v)
{
    if (cv->table) return table_value(m, cv->table, t, S, v);
    fwd_cache c;
    forward(m, cv, t, S, v, &c);
    return orc_cv_out_scale(m) * c.y;
}

void orc_cv_table_grid(const orc_model *m, orc_cv_table *g)
{
    int heston = m->kind == ORC_HESTON;
    double spread = 4.0 * sref_of(m) * sqrt(m->T);
    g->rows = heston ? 16 : 256;
    g->ns = heston ? 16 : 32;
    g->nv = heston ? 32 : 1;
    g->s_lo = m->S0 * exp(-spread);
    g->s_hi = m->S0 * exp(spread);
    g->v_lo = 0.0;
    g->v_hi = heston ? 4.0 * (m->theta > m->v0 ? m->theta : m->v0) : 1.0;
    g->values = NULL;
}

void orc_cv_table_fill(const orc_model *m, const orc_cv *cv, const orc_cv_table *g,
                       double *values)
{
    orc_cv net = *cv;
    net.table = NULL;
    double ds = (g->s_hi - g->s_lo) / (g->ns - 1);
    double dv = g->nv > 1 ? (g->v_hi - g->v_lo) / (g->nv - 1) : 0.0;
    for (int j = 0; j < g->rows; ++j)
        for (int k = 0; k < g->nv; ++k)
            for (int i = 0; i < g->ns; ++i)
                values[((size_t)j * g->nv + k) * g->ns + i] =
                    orc_cv_phi(m, &net, j * m->T / g->rows, g->s_lo + i * ds, g->v_lo + k * dv);
}

void orc_cv_phi_grad(const orc_model *m, const orc_cv *cv, double t, double S, double v,
                     double g, double *grad)
{
    int D = cv->in_dim, H = cv->hidden;
    fwd_cache c;
    forward(m, cv, t, S, v, &c);
    net_view nv = view_of(cv->params, D, H);
    /* gradient slots, same layout as params */
    double *gW1 = grad, *gb1 = gW1 + (size_t)D * H, *gW2 = gb1 + H;
    double *gb2 = gW2 + (size_t)H * H, *gw3 = gb2 + H, *gb3 = gw3 + H;
    double dy = g * orc_cv_out_scale(m);
    gb3[0] += dy;
    double d2[HMAX], d2q[HMAX];
    for (int j = 0; j < H; ++j) {
        gw3[j] += dy * c.h2[j];
        d2[j] = dy * nv.w3[j] * (1.0 - c.h2[j] * c.h2[j]);
        d2q[j] = cv->bf16_emulate ? bf16_round(d2[j]) : d2[j];
        gb2[j] += d2[j];
        for (int k = 0; k < H; ++k) gW2[j * H + k] += d2q[j] * c.h1q[k];
    }
    for (int k = 0; k < H; ++k) {
        double e = 0.0;
        for (int j = 0; j < H; ++j) {
            double w = cv->bf16_emulate ? bf16_round(nv.W2[j * H + k]) : nv.W2[j * H + k];
            e += w * d2q[j];
        }
        double d1 = e * (1.0 - c.h1[k] * c.h1[k]);
        gb1[k] += d1;
        for (int d = 0; d < D; ++d) gW1[k * D + d] += d1 * c.x[d];
    }
}

/* Defined in sampler.c: regenerate one training path and accumulate
 * w * dY/dparams into grad (Y = (Pf - cvf) - (Pc - cvc)).               */
void orc_internal_path_grad(const orc_model *m, const orc_payoff *p, int l, int M,
                            uint64_t seed, uint64_t s, int stream, const orc_cv *cv,
                            double w, double *grad);

typedef struct {
    const orc_model *m; const orc_payoff *p; const orc_cv *cv;
    int l, M; uint64_t seed, first, count, base_index;
    const double *w;      /* per-path weights, indexed by i - base_index */
    double *Y;            /* per-path Y (pass 1) */
    double *grad;         /* per-thread gradient (pass 2) */
    int pass;
} cv_job;

static void *cv_run(void *arg)
{
    cv_job *j = (cv_job *)arg;
    for (uint64_t i = 0; i < j->count; ++i) {
        uint64_t idx = j->first + i;                  /* index within batch */
        uint64_t s = j->base_index + idx;             /* global path index */
        if (j->pass == 1) {
            double pf, pc;
            orc_level_sample(j->m, j->p, j->l, j->M, j->seed, s, ORC_STREAM_TRAIN_NORMAL,
                             j->cv, &pf, &pc, NULL, NULL);
            j->Y[idx] = pf - pc;
        } else {
            orc_internal_path_grad(j->m, j->p, j->l, j->M, j->seed, s,
                                   ORC_STREAM_TRAIN_NORMAL, j->cv, j->w[idx], j->grad);
        }
    }
    return NULL;
}

static void cv_parallel(cv_job *proto, uint64_t B, int nthreads, size_t np, double *grad)
{
    if (nthreads < 1) nthreads = 1;
    cv_job *jobs = calloc((size_t)nthreads, sizeof(cv_job));
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    uint64_t base = 0;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t cnt = B / nthreads + ((uint64_t)t < B % nthreads ? 1 : 0);
        jobs[t] = *proto;
        jobs[t].first = base;
        jobs[t].count = cnt;
        if (proto->pass == 2) jobs[t].grad = calloc(np, sizeof(double));
        base += cnt;
        pthread_create(&th[t], NULL, cv_run, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    if (proto->pass == 2) {
        for (int t = 0; t < nthreads; ++t) {
            for (size_t q = 0; q < np; ++q) grad[q] += jobs[t].grad[q];
            free(jobs[t].grad);
        }
    }
    free(jobs);
    free(th);
}

double orc_cv_loss_grad(const orc_model *m, const orc_payoff *p, int M, int lmax,
                        uint64_t B, uint64_t seed, uint64_t step, const orc_cv *cv,
                        int nthreads, double *grad, double *var_out)
{
    if (m->scheme != ORC_EULER || m->antithetic) return NAN;   /* Euler paths only */
    size_t np = orc_cv_nparams(cv->in_dim, cv->hidden);
    if (grad) memset(grad, 0, sizeof(double) * np);
    double *Y = malloc(sizeof(double) * B);
    double *w = malloc(sizeof(double) * B);
    double loss = 0.0;
    for (int l = 0; l <= lmax; ++l) {
        cv_job proto = {0};
        proto.m = m; proto.p = p; proto.cv = cv; proto.l = l; proto.M = M;
        proto.seed = seed; proto.base_index = step * B; proto.Y = Y; proto.w = w;
        proto.pass = 1;
        cv_parallel(&proto, B, nthreads, np, NULL);
        double mean = 0.0;
        for (uint64_t i = 0; i < B; ++i) mean += Y[i];
        mean /= (double)B;
        double var = 0.0;
        for (uint64_t i = 0; i < B; ++i) var += (Y[i] - mean) * (Y[i] - mean);
        var /= (double)(B - 1);
        if (var_out) var_out[l] = var;
        double C = orc_level_cost(l, M, 0);
        loss += sqrt(C * var);
        if (!grad) continue;
        double scale = (var > 0) ? sqrt(C / var) / (double)(B - 1) : 0.0;
        for (uint64_t i = 0; i < B; ++i) w[i] = scale * (Y[i] - mean);
        proto.pass = 2;
        cv_parallel(&proto, B, nthreads, np, grad);
    }
    free(Y);
    free(w);
    return loss;
}

void orc_adam(size_t n, double *theta, double *m1, double *m2, const double *g,
              double lr, double b1, double b2, double eps, int t)
{
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (size_t i = 0; i < n; ++i) {
        m1[i] = b1 * m1[i] + (1.0 - b1) * g[i];
        m2[i] = b2 * m2[i] + (1.0 - b2) * g[i] * g[i];
        double mh = m1[i] / c1, vh = m2[i] / c2;
        theta[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
