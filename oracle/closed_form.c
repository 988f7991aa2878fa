/*
 * Closed-form values used to pin the oracle (test infrastructure only).
 *
 * None of these appears in the paper, which prints no numbers; they are the
 * textbook exact values that the paper's estimators converge to:
 *  - Black--Scholes call and cash-or-nothing digital (the Sec. 6 experiment's
 *    payoffs under its GBM model);
 *  - the continuously monitored floating-strike lookback call
 *    (Goldman, Sosin and Gatto 1979), the limit of the bridge-corrected
 *    lookback;
 *  - the continuously averaged geometric Asian call (a lower bound for the
 *    arithmetic Asian);
 *  - the Heston (1993) call by Fourier inversion of the characteristic
 *    function in the Albrecher et al. (2007) form;
 *  - exact moments of the Euler--Maruyama scheme itself (eq. (eq:em)) for the
 *    payoff e^-rT S_N and for the one-step European call, which pin the
 *    sampler level by level without any discretisation bias.
 */
#include <math.h>
#include <complex.h>
#include "oracle.h"

double orc_norm_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }
static double norm_pdf(double x) { return exp(-0.5 * x * x) / sqrt(2.0 * 3.14159265358979323846); }

double orc_bs_call(double S0, double K, double r, double sigma, double T)
{
    double sq = sigma * sqrt(T);
    double d1 = (log(S0 / K) + (r + 0.5 * sigma * sigma) * T) / sq;
    double d2 = d1 - sq;
    return S0 * orc_norm_cdf(d1) - K * exp(-r * T) * orc_norm_cdf(d2);
}

double orc_bs_digital(double S0, double K, double r, double sigma, double T, double payout)
{
    double sq = sigma * sqrt(T);
    double d2 = (log(S0 / K) + (r - 0.5 * sigma * sigma) * T) / sq;
    return payout * exp(-r * T) * orc_norm_cdf(d2);
}

/* Floating-strike lookback call paying S_T - min_{[0,T]} S, started at its
 * running minimum (S_min = S0), no dividends, r > 0.                     */
double orc_lookback_float_call(double S0, double r, double sigma, double T)
{
    double sq = sigma * sqrt(T);
    double s2 = sigma * sigma;
    double a1 = (r + 0.5 * s2) * T / sq;
    double a2 = a1 - sq;
    double a3 = (-r + 0.5 * s2) * T / sq;
    double k = s2 / (2.0 * r);
    return S0 * orc_norm_cdf(a1) - S0 * k * orc_norm_cdf(-a1)
           - S0 * exp(-r * T) * (orc_norm_cdf(a2) - k * orc_norm_cdf(-a3));
}

/* Call on G = exp((1/T) int_0^T ln S dt): ln G ~ N(ln S0 + (r - s^2/2) T/2, s^2 T/3). */
double orc_geometric_asian_call(double S0, double K, double r, double sigma, double T)
{
    double mu = log(S0) + 0.5 * (r - 0.5 * sigma * sigma) * T;
    double var = sigma * sigma * T / 3.0;
    double sd = sqrt(var);
    double d2 = (mu - log(K)) / sd;
    double d1 = d2 + sd;
    return exp(-r * T) * (exp(mu + 0.5 * var) * orc_norm_cdf(d1) - K * orc_norm_cdf(d2));
}

/* Characteristic function of ln S_T under Heston (Albrecher et al. form). */
static double complex heston_cf(double complex u, double S0, double r, double T,
                                double kappa, double theta, double xi, double rho, double v0)
{
    double complex iu = I * u;
    double complex b = kappa - rho * xi * iu;
    double complex d = csqrt(b * b + xi * xi * (iu + u * u));
    double complex g = (b - d) / (b + d);
    double complex e = cexp(-d * T);
    double complex C = kappa * theta / (xi * xi) * ((b - d) * T - 2.0 * clog((1.0 - g * e) / (1.0 - g)));
    double complex D = (b - d) / (xi * xi) * (1.0 - e) / (1.0 - g * e);
    return cexp(iu * (log(S0) + r * T) + C + D * v0);
}

/* C = S0 P1 - K e^-rT P2 with the Gil-Pelaez probabilities, integrated by
 * composite Simpson on (0, 200] in u (integrand decays exponentially).     */
double orc_heston_call(double S0, double K, double r, double T, double kappa,
                       double theta, double xi, double rho, double v0)
{
    const int n = 40000;        /* even */
    const double umax = 200.0, du = umax / n;
    double complex phi_mi = heston_cf(-I, S0, r, T, kappa, theta, xi, rho, v0);
    double lk = log(K);
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i <= n; ++i) {
        double u = (i == 0) ? 1e-10 : i * du;
        double w = (i == 0 || i == n) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
        double complex eik = cexp(-I * u * lk);
        double complex f2 = heston_cf(u, S0, r, T, kappa, theta, xi, rho, v0);
        double complex f1 = heston_cf(u - I, S0, r, T, kappa, theta, xi, rho, v0) / phi_mi;
        s1 += w * creal(eik * f1 / (I * u));
        s2 += w * creal(eik * f2 / (I * u));
    }
    const double pi = 3.14159265358979323846;
    double P1 = 0.5 + s1 * du / 3.0 / pi;
    double P2 = 0.5 + s2 * du / 3.0 / pi;
    return S0 * P1 - K * exp(-r * T) * P2;
}

/* Exact moments of Euler--Maruyama GBM with payoff e^-rT S_N.
 * One fine step multiplies S by (1 + r h + sigma dW), dW ~ N(0, h):
 *   E[.] = 1 + r h,  E[.^2] = (1 + r h)^2 + sigma^2 h.
 * Over one coarse step the fine product F and the coarse factor
 * G = 1 + r H + sigma sum dW satisfy
 *   E[F G] = (1 + r h)^M (1 + r H) + sigma^2 M h (1 + r h)^(M-1),
 * and coarse steps are independent, so every moment is a power.          */
void orc_euler_k0_moments(double S0, double r, double sigma, double T, int l, int M,
                          double out[2])
{
    double disc = exp(-r * T);
    double nf = pow((double)M, (double)l);
    double h = T / nf;
    double Ef = S0 * pow(1.0 + r * h, nf);
    double Eff = S0 * S0 * pow((1.0 + r * h) * (1.0 + r * h) + sigma * sigma * h, nf);
    out[0] = disc * Ef;
    if (l == 0) {
        out[1] = disc * disc * (Eff - Ef * Ef);
        return;
    }
    double nc = nf / M, H = M * h;
    double Ec = S0 * pow(1.0 + r * H, nc);
    double Ecc = S0 * S0 * pow((1.0 + r * H) * (1.0 + r * H) + sigma * sigma * H, nc);
    double Efc = S0 * S0 * pow(pow(1.0 + r * h, M) * (1.0 + r * H)
                               + sigma * sigma * M * h * pow(1.0 + r * h, M - 1), nc);
    double mean_d = Ef - Ec;
    out[1] = disc * disc * (Eff + Ecc - 2.0 * Efc - mean_d * mean_d);
}

/* One Euler step: S_1 = S0 (1 + r T) + S0 sigma sqrt(T) Z, so S_1 ~ N(mu, s^2). */
void orc_level0_call_moments(double S0, double K, double r, double sigma, double T,
                             double out[2])
{
    double disc = exp(-r * T);
    double mu = S0 * (1.0 + r * T), s = S0 * sigma * sqrt(T);
    double a = mu - K, d = a / s;
    double m1 = a * orc_norm_cdf(d) + s * norm_pdf(d);
    double m2 = (a * a + s * s) * orc_norm_cdf(d) + a * s * norm_pdf(d);
    out[0] = disc * m1;
    out[1] = disc * disc * (m2 - m1 * m1);
}
