/*
 * Oracle randomised single-term estimator (test infrastructure only).
 *
 * Sec. 7 cites Rhee and Glynn's extra level of randomisation that makes the
 * multilevel estimator unbiased.  Reading (the paper gives no formula): each
 * of the N samples draws its level L from p_l = (1 - q) q^l / (1 - q^(Lc+1)),
 * l = 0..Lc (a geometric law cut at the finest level Lc), and contributes
 * Z = Y_L / p_L, where Y_L is the level-L sample of eq. (eq:Yldef) (P_0 at
 * level 0).  Then E[Z] = sum_l E[Y_l] = E[P_Lc] (eq. (eq:mlmc:ident)) with no
 * choice of a finest level left to the bias test; Lc only bounds the grid.
 * The variance is finite when sum_l V_l / p_l is, i.e. q > M^-beta, and the
 * expected cost sum_l p_l C_l when q < M^-1: both need beta > 1 (Milstein).
 *
 * Level draw of sample i: word i mod 4 of the Philox block at counter
 * (0, i / 4, level field 0, stream 7), uniform u = ((x >> 8) + 1/2) 2^-24,
 * L = the first l with u < F(l) = sum_{k <= l} p_k.  Given the counts n_l,
 * the level-l samples are the sampler's samples 0 .. n_l - 1 of level l, so
 *   estimate = (1/N) sum_l S1_l / p_l,   E[Z^2] ~ (1/N) sum_l S2_l / p_l^2.
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

void orc_rg_probabilities(double q, int Lc, double *p, double *F)
{
    double norm = 1.0 - pow(q, (double)(Lc + 1));
    double acc = 0.0;
    for (int l = 0; l <= Lc; ++l) {
        p[l] = (1.0 - q) * pow(q, (double)l) / norm;
        acc += p[l];
        F[l] = acc;
    }
    F[Lc] = 1.0;   /* the last bin takes the rounding */
}

int orc_rg_level_counts(uint64_t seed, uint64_t N, double q, int Lc, uint64_t *counts)
{
    if (Lc < 0 || Lc > 15 || !(q > 0.0 && q < 1.0)) return -1;
    double p[16], F[16];
    orc_rg_probabilities(q, Lc, p, F);
    memset(counts, 0, sizeof(uint64_t) * (size_t)(Lc + 1));
    uint32_t w[4];
    for (uint64_t i = 0; i < N; ++i) {
        if (i % 4 == 0) orc_path_words(seed, 0, i / 4, ORC_STREAM_LEVEL_DRAW, 1, w);
        double u = orc_u01(w[i % 4]);
        int l = 0;
        while (l < Lc && !(u < F[l])) ++l;
        counts[l]++;
    }
    return 0;
}

int orc_rhee_glynn(const orc_model *m, const orc_payoff *p, int M, int Lc, double q, uint64_t N,
                   uint64_t seed, int nthreads, orc_rg_result *out)
{
    if (!m || !p || !out || N == 0 || M < 2) return -1;
    memset(out, 0, sizeof(*out));
    if (orc_rg_level_counts(seed, N, q, Lc, out->N)) return -1;
    double F[16];
    orc_rg_probabilities(q, Lc, out->p, F);
    double z1 = 0.0, z2 = 0.0;
    for (int l = 0; l <= Lc; ++l) {
        if (out->N[l] == 0) continue;
        orc_level_result r;
        if (orc_level(m, p, l, M, out->N[l], seed, 0, NULL, nthreads, &r)) return -1;
        out->sum_y[l] = r.sum_y;
        out->sum_y2[l] = r.sum_y2;
        out->cost += r.cost;
        out->n_nonfinite += r.n_nonfinite;
        z1 += r.sum_y / out->p[l];
        z2 += r.sum_y2 / (out->p[l] * out->p[l]);
    }
    out->Lc = Lc;
    out->estimate = z1 / (double)N;
    out->variance = z2 / (double)N - out->estimate * out->estimate;
    return 0;
}
