/*
 * Oracle MLMC driver (test infrastructure only).
 *
 * The paper fixes the estimator Y = sum_l Yhat_l (eqs. (eq:mlmc:ident),
 * (eq:mlmc:Yzero), (eq:Yldef)), the fact that the level variances add because
 * levels are independent (Sec. 5), the cost measure (Sec. 3: generator calls,
 * proportional to the number of steps), and leaves the choice of N_l to "a
 * cheap pre-processing step where appropriate variances are estimated and an
 * optimization problem is solved" (Sec. 5, "Constructive Upper Bound").  The
 * complexity theorem (Sec. 5) states the target E[(Y - E P)^2] < eps^2.
 *
 * Reading used here (standard MLMC):
 *  - eps is a root-mean-square error; the mean-square error is split evenly,
 *    bias^2 <= eps^2/2 and sum_l V_l/N_l <= eps^2/2.
 *  - minimising sum_l N_l C_l under sum_l V_l/N_l = eps^2/2 (Lagrange) gives
 *    N_l = ceil(2 eps^-2 sqrt(V_l/C_l) sum_k sqrt(V_k C_k)).
 *  - C_0 = 1 and C_l = M^l + M^(l-1) path steps (fine plus coarse).
 *  - for l >= 2, estimates are floored by the assumed rates: V_l >=
 *    V_{l-1} M^-beta and |E_l| >= |E_{l-1}| M^-alpha, which keeps a noisy
 *    small estimate from starving a level.
 *  - a level is sampled again only when its shortfall exceeds 1% of what it
 *    has; once no level needs more, the bias is estimated from the weak-order
 *    assumption |E[P - P_L]| ~ |E_L| / (M^alpha - 1) (eq. (eq:emweak) with
 *    alpha = 1), using max(|E_L|, |E_{L-1}| M^-alpha); if that exceeds
 *    eps/sqrt(2), a level is added (V_{L+1} = V_L M^-beta) up to L_max.
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

void orc_optimal_n(int L, const double *V, const double *C, double eps, double *N)
{
    double total = 0.0;
    for (int k = 0; k <= L; ++k) total += sqrt(V[k] * C[k]);
    for (int l = 0; l <= L; ++l)
        N[l] = ceil(2.0 / (eps * eps) * sqrt(V[l] / C[l]) * total);
}

double orc_fit_rate(int L, const double *y, int M)
{
    /* least squares of log_M y_l on l for l = 1..L */
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    int n = 0;
    for (int l = 1; l <= L; ++l) {
        if (!(y[l] > 0)) continue;
        double x = l, v = log(y[l]) / log((double)M);
        sx += x; sy += v; sxx += x * x; sxy += x * v; ++n;
    }
    if (n < 2) return NAN;
    return (n * sxy - sx * sy) / (n * sxx - sx * sx);
}

int orc_mlmc_run(const orc_model *m, const orc_payoff *p, const orc_run_opts *o,
                 orc_run_result *out)
{
    if (!m || !p || !o || !out) return -1;
    if (o->eps <= 0 || o->M < 2 || o->L_min < 1 || o->L_max < o->L_min || o->L_max > 15)
        return -1;
    double alpha = o->alpha > 0 ? o->alpha : 1.0;
    double beta = o->beta > 0 ? o->beta : 1.0;
    int M = o->M;
    double Ma = pow((double)M, alpha), Mb = pow((double)M, beta);

    memset(out, 0, sizeof(*out));
    int L = o->L_min;
    double n[16] = {0}, s1[16] = {0}, s2[16] = {0}, dN[16] = {0};
    double E[16], V[16], C[16], Nopt[16];
    for (int l = 0; l <= L; ++l) dN[l] = (double)o->n_pilot;
    int converged = 0, iterations = 0;
    for (;;) {
        ++iterations;
        for (int l = 0; l <= L; ++l) {
            if (dN[l] <= 0) continue;
            orc_level_result r;
            orc_level(m, p, l, M, (uint64_t)dN[l], o->seed, (uint64_t)n[l], o->cv,
                      o->nthreads, &r);
            s1[l] += r.sum_y;
            s2[l] += r.sum_y2;
            n[l] += dN[l];
            out->cost += r.cost;
        }
        for (int l = 0; l <= L; ++l) {
            C[l] = orc_level_cost(l, M, m->antithetic);
            E[l] = fabs(s1[l] / n[l]);
            V[l] = s2[l] / n[l] - (s1[l] / n[l]) * (s1[l] / n[l]);
            if (V[l] < 0) V[l] = 0;
        }
        for (int l = 2; l <= L; ++l) {
            if (E[l] < E[l - 1] / Ma) E[l] = E[l - 1] / Ma;
            if (V[l] < V[l - 1] / Mb) V[l] = V[l - 1] / Mb;
        }
        orc_optimal_n(L, V, C, o->eps, Nopt);
        int more = 0;
        for (int l = 0; l <= L; ++l) {
            double d = Nopt[l] - n[l];
            dN[l] = (d > 0.01 * n[l]) ? d : 0.0;
            if (dN[l] > 0) more = 1;
        }
        if (more) continue;
        double rem = fmax(E[L], E[L - 1] / Ma) / (Ma - 1.0);
        if (rem <= o->eps / sqrt(2.0)) { converged = 1; break; }
        if (L == o->L_max) break;
        ++L;
        V[L] = V[L - 1] / Mb;
        C[L] = orc_level_cost(L, M, m->antithetic);
        n[L] = 0; s1[L] = 0; s2[L] = 0;
        orc_optimal_n(L, V, C, o->eps, Nopt);
        for (int l = 0; l <= L; ++l) {
            double d = Nopt[l] - n[l];
            dN[l] = (l == L) ? (Nopt[l] > 1 ? Nopt[l] : 1.0) : ((d > 0.01 * n[l]) ? d : 0.0);
        }
    }
    out->L = L;
    out->converged = converged;
    out->iterations = iterations;
    out->estimate = 0.0;
    for (int l = 0; l <= L; ++l) {
        out->estimate += s1[l] / n[l];
        out->N[l] = (uint64_t)n[l];
        out->sum_y[l] = s1[l];
        out->sum_y2[l] = s2[l];
        out->E[l] = s1[l] / n[l];
        out->V[l] = s2[l] / n[l] - out->E[l] * out->E[l];
        out->C[l] = orc_level_cost(l, M, m->antithetic);
    }
    double absE[16], Vr[16];
    for (int l = 0; l <= L; ++l) { absE[l] = fabs(out->E[l]); Vr[l] = out->V[l]; }
    out->alpha = -orc_fit_rate(L, absE, M);
    out->beta = -orc_fit_rate(L, Vr, M);
    out->gamma = orc_fit_rate(L, out->C, M);
    return 0;
}
