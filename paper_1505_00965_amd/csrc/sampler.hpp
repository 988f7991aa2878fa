// Fused coupled level sampler for gfx950: one lane advances PPT coupled
// (fine, coarse) Euler--Maruyama path pairs of level l, all in registers.
//
// Level l: n_f = M^l fine steps of size h = T/n_f (eq. (eq:mlmc:Dtl)); the
// coarse path takes n_f/M steps of size H = M h, each driven by the sum of
// the M fine Brownian increments it covers (eq. (eq:Yldef) and Fig. 2); level
// 0 has only the single-step path (eq. (eq:mlmc:Yzero)).  Steps follow
// eq. (eq:em) in increment form, S <- S + S (r dt + vol dW), which in fp32
// keeps the drift that the product form 1 + r dt would round away.
//
// Work per fine step lives in VGPRs: state, coarse increment sums, payoff
// accumulators.  The generator block j (four 32-bit words) feeds four fine
// steps of a one-factor model or two of the two-factor (Heston) model, so with
// M = 4 one block is exactly one coarse step of GBM.  Nothing touches memory
// inside the path loop.
#pragma once
#include "philox.hpp"

namespace mlmc {

// Sampler variants: the SDE and its time stepping.  GBM steps by
// Euler--Maruyama (kGBM) or by the Milstein scheme (kGBMMil); Heston by
// full-truncation Euler.
enum ModelKind : int { kGBM = 0, kHeston = 1, kGBMMil = 2 };
// One Brownian factor and a constant volatility sigma (both GBM variants).
__host__ __device__ constexpr bool one_factor(int model) { return model != kHeston; }
enum PayoffKind : int { kCall = 0, kAsian = 1, kLookback = 2, kDigital = 3, kDigitalCond = 4 };

// Model and payoff parameters converted once on the host.
template <typename Real>
struct StepParams {
    Real S0, r, sigma, kappa, theta, xi, rho, rho_c, v0;
    Real h, sqh, H, rh, rH;          // fine/coarse step sizes and r*dt
    Real c2, rh_m, rH_m;             // Milstein: sigma^2/2, (r - sigma^2/2) dt
    Real K, payout, disc, inv_T;     // payoff
    Real lnu_scale;                  // -2 h ln(2): bridge term e = lnu_scale * log2(U)
    Real asian_scale;                // h / (2T)
    // level 0 of a European call (one Euler step from S0):
    // S_1 - K = l0_base + l0_slope dW, l0_base = S0 (1 + r T) - K, l0_slope = S0 sigma
    Real l0_base, l0_slope;
};

// Fused multiply-add in the path's own precision (no promotion to fp64).
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename Real>
__device__ __forceinline__ Real fsqrt(Real x);
template <>
__device__ __forceinline__ float fsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <>
__device__ __forceinline__ double fsqrt<double>(double x) { return sqrt(x); }

template <typename Real>
__device__ __forceinline__ Real flog2(Real x);
template <>
__device__ __forceinline__ float flog2<float>(float x) { return __builtin_amdgcn_logf(x); }
template <>
__device__ __forceinline__ double flog2<double>(double x) { return log2(x); }

template <typename Real>
__device__ __forceinline__ Real fmaxT(Real a, Real b);
template <>
__device__ __forceinline__ float fmaxT<float>(float a, float b) { return __builtin_fmaxf(a, b); }
template <>
__device__ __forceinline__ double fmaxT<double>(double a, double b) { return __builtin_fmax(a, b); }

template <typename Real>
__device__ __forceinline__ Real uniform01(uint32_t x);
template <>
__device__ __forceinline__ float uniform01<float>(uint32_t x) { return u01f(x); }
template <>
__device__ __forceinline__ double uniform01<double>(uint32_t x) { return u01d(x); }

// Brownian increments sqrt(h) z0, sqrt(h) z1 of one Box--Muller pair.  In
// fp32 the step size goes into the radius, sqrt(-2 h ln u1) =
// sqrt(lnu_scale log2 u1), which saves the two products by sqrt(h); fp64
// scales the standard normals.
__device__ __forceinline__ void brownian_pair(uint32_t a, uint32_t b, const StepParams<float>& P,
                                              float& d0, float& d1)
{
    const float u1 = u01f(a), u2 = u01f(b);
    const float rho = __builtin_amdgcn_sqrtf(P.lnu_scale * __builtin_amdgcn_logf(u1));
    d0 = rho * __builtin_amdgcn_cosf(u2);
    d1 = rho * __builtin_amdgcn_sinf(u2);
}

__device__ __forceinline__ void brownian_pair(uint32_t a, uint32_t b, const StepParams<double>& P,
                                              double& d0, double& d1)
{
    double z0, z1;
    box_muller(a, b, z0, z1);
    d0 = P.sqh * z0;
    d1 = P.sqh * z1;
}

// Compensated (Kahan) accumulation for the Asian average: the path values
// are positive and of one magnitude, so the running compensation c keeps the
// sum of up to 65536 terms at ~1e-7 relative accuracy in fp32 (sum - c is
// the compensated total), in four lane operations per term.
template <typename Real>
__device__ __forceinline__ void comp_add(Real& sum, Real& comp, Real x)
{
    const Real y = x - comp;
    const Real t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

// Exact minimum of a Brownian bridge with frozen volatility b over a step,
// (x0 + x1 - sqrt((x1 - x0)^2 - 2 b^2 dt ln U)) / 2, with e = -2 dt ln U.
template <typename Real>
__device__ __forceinline__ Real bridge_min(Real x0, Real x1, Real b, Real e)
{
    const Real d = x1 - x0;
    return Real(0.5) * (x0 + x1 - fsqrt<Real>(d * d + (b * b) * e));
}

template <typename Real>
struct PathPair {
    Real S, v;                 // fine state
    Real Sc, vc;               // coarse state
    Real dw1c, dwpc;           // coarse increment sums (S factor, independent factor)
    Real asum, acomp;          // fine trapezoid sum (compensated)
    Real csum, ccomp;          // coarse trapezoid sum
    Real mn, mnc;              // bridge minima
    Real wpart;                // coarse lookback: fine Brownian path since the coarse step start
    Real cvf, cvc;             // control-variate sums (unused without a network)
    // conditional digital: state, volatility and increment of the last step
    Real Sl, vl, dwl;          // fine path
    Real Scl, vcl, wcl;        // coarse path (wcl: its whole last increment)
};

template <typename Real, int MODEL, int PAYOFF>
__device__ __forceinline__ void init_pair(PathPair<Real>& q, const StepParams<Real>& P)
{
    q.S = P.S0; q.v = P.v0; q.Sc = P.S0; q.vc = P.v0;
    q.dw1c = 0; q.dwpc = 0;
    q.asum = 0; q.acomp = 0; q.csum = 0; q.ccomp = 0;
    q.mn = Real(INFINITY); q.mnc = Real(INFINITY);
    q.wpart = 0; q.cvf = 0; q.cvc = 0;
    q.Sl = q.vl = q.dwl = 0; q.Scl = q.vcl = q.wcl = 0;
}

// Relative move of the frozen-coefficient coarse step after j fine times
// with Brownian increment w: r tau + vol w (+ sigma^2/2 (w^2 - tau) for
// Milstein), tau = j h; at j = M it is the coarse step itself.
template <typename Real, int MODEL>
__device__ __forceinline__ Real refine(const StepParams<Real>& P, Real vol, Real w, int j)
{
    const Real lin = fmaT(vol, w, P.rh * Real(j));
    if (MODEL == kGBMMil) return fmaT(P.c2, fmaT(w, w, -P.h * Real(j)), lin);
    return lin;
}

// One fine step with increments (dw1, dwp), bridge exponent e (lookback only)
// and position k = n mod M inside the current coarse step.
template <typename Real, int MODEL, int PAYOFF>
__device__ __forceinline__ void fine_step(PathPair<Real>& q, const StepParams<Real>& P, Real dw1,
                                          Real dwp, Real e, int k, bool coupled)
{
    const Real S0n = q.S;
    Real vol;
    if (MODEL == kGBM) {
        vol = P.sigma;
        q.S = fmaT(q.S, fmaT(P.sigma, dw1, P.rh), q.S);
    } else if (MODEL == kGBMMil) {
        // S + S (r h + sigma dW + sigma^2/2 (dW^2 - h))
        vol = P.sigma;
        q.S = fmaT(q.S, fmaT(P.c2, dw1 * dw1, fmaT(P.sigma, dw1, P.rh_m)), q.S);
    } else {
        const Real vp = q.v > Real(0) ? q.v : Real(0);
        vol = fsqrt<Real>(vp);
        const Real dw2 = fmaT(P.rho, dw1, P.rho_c * dwp);
        q.S = fmaT(q.S, fmaT(vol, dw1, P.rh), q.S);
        q.v = fmaT(P.xi * vol, dw2, fmaT(P.kappa * P.h, P.theta - vp, q.v));
    }
    if (PAYOFF == kAsian) comp_add(q.asum, q.acomp, q.S);   // sum of S_1 .. S_n
    if (PAYOFF == kDigitalCond) {
        q.Sl = S0n;
        q.vl = vol;
        q.dwl = dw1;
    }
    if (PAYOFF == kLookback) {
        const Real m = bridge_min(S0n, q.S, vol * S0n, e);
        q.mn = m < q.mn ? m : q.mn;
    }
    if (!coupled) return;
    // k == 0 opens a coarse step: assign rather than add to the zero the
    // previous coarse step left (same value; with k known at compile time it
    // saves the addition)
    q.dw1c = k == 0 ? dw1 : q.dw1c + dw1;
    if (MODEL == kHeston) q.dwpc = k == 0 ? dwp : q.dwpc + dwp;
    if (PAYOFF == kLookback) {
        // coarse path refined at the fine times with frozen coefficients:
        // X(tau) = Sc + Sc (r tau + vol_c W(tau)), W from the coarse step start
        const Real volc = one_factor(MODEL) ? P.sigma
                                            : fsqrt<Real>(q.vc > Real(0) ? q.vc : Real(0));
        const Real x0 = k == 0 ? q.Sc : fmaT(q.Sc, refine<Real, MODEL>(P, volc, q.wpart, k), q.Sc);
        q.wpart = k == 0 ? dw1 : q.wpart + dw1;
        const Real x1 = fmaT(q.Sc, refine<Real, MODEL>(P, volc, q.wpart, k + 1), q.Sc);
        const Real m = bridge_min(x0, x1, volc * q.Sc, e);
        q.mnc = m < q.mnc ? m : q.mnc;
    }
}

// One coarse step from the accumulated sums.
template <typename Real, int MODEL, int PAYOFF>
__device__ __forceinline__ void coarse_step(PathPair<Real>& q, const StepParams<Real>& P)
{
    const Real S0c = q.Sc;
    Real volc;
    if (MODEL == kGBM) {
        volc = P.sigma;
        q.Sc = fmaT(q.Sc, fmaT(P.sigma, q.dw1c, P.rH), q.Sc);
    } else if (MODEL == kGBMMil) {
        volc = P.sigma;
        q.Sc = fmaT(q.Sc, fmaT(P.c2, q.dw1c * q.dw1c, fmaT(P.sigma, q.dw1c, P.rH_m)), q.Sc);
    } else {
        const Real vp = q.vc > Real(0) ? q.vc : Real(0);
        const Real sv = fsqrt<Real>(vp);
        volc = sv;
        const Real dw2 = fmaT(P.rho, q.dw1c, P.rho_c * q.dwpc);
        q.Sc = fmaT(q.Sc, fmaT(sv, q.dw1c, P.rH), q.Sc);
        q.vc = fmaT(P.xi * sv, dw2, fmaT(P.kappa * P.H, P.theta - vp, q.vc));
    }
    if (PAYOFF == kDigitalCond) {
        q.Scl = S0c;
        q.vcl = volc;
        q.wcl = q.dw1c;
    }
    if (PAYOFF == kAsian) comp_add(q.csum, q.ccomp, q.Sc);
    q.dw1c = 0;
    q.dwpc = 0;
    q.wpart = 0;
}

template <typename Real, int PAYOFF>
__device__ __forceinline__ Real payoff_value(const StepParams<Real>& P, Real S, Real sum,
                                             Real comp, Real mn, Real dt)
{
    // a path that overflowed stays visible as a non-finite payoff: S - S is
    // +0 for finite S and NaN otherwise (one lane operation, no branch); the
    // discount multiplies in the same fused operation
    const Real nan_if_overflow = S - S;
    if (PAYOFF == kDigital) {
        const Real v = S > P.K ? P.disc * P.payout
                               : (S == P.K ? P.disc * Real(0.5) * P.payout : Real(0));
        return v + nan_if_overflow;
    }
    Real u;
    if (PAYOFF == kCall) {
        u = fmaxT<Real>(S - P.K, Real(0));
    } else if (PAYOFF == kAsian) {
        // trapezoid over the grid: dt (S_0/2 + S_1 + ... + S_{N-1} + S_N/2)
        //   = dt (sum_{n=1..N} S_n + (S_0 - S_N)/2)
        const Real tw = fmaT(Real(0.5), P.S0 - S, sum - comp);
        u = fmaxT<Real>(fmaT(tw, dt * P.inv_T, -P.K), Real(0));   // A - K
    } else {
        u = S - mn;   // floating-strike lookback
    }
    return fmaT(P.disc, u, nan_if_overflow);
}

// Standard normal distribution function, erfc(-z / sqrt 2) / 2.
__device__ __forceinline__ float norm_cdf(float z) { return 0.5f * erfcf(-0.70710678118654752f * z); }
__device__ __forceinline__ double norm_cdf(double z) { return 0.5 * erfc(-0.70710678118654752 * z); }

// payout P(A + B x + C x^2 > K) for x ~ N(0, h), C >= 0 (roots in the stable
// form q = -(B + sign(B) sqrt(disc))/2, x = q/C and (A - K)/q).
template <typename Real>
__device__ __forceinline__ Real digital_given(const StepParams<Real>& P, Real A, Real B, Real C)
{
    const Real c0 = A - P.K;
    if (C > Real(0)) {
        const Real disc = fmaT(B, B, Real(-4) * C * c0);
        if (disc <= Real(0)) return P.payout;
        const Real q = Real(-0.5) * (B + copysign(fsqrt<Real>(disc), B));
        Real x1 = q / C, x2 = c0 / q;
        if (x1 > x2) { const Real t = x1; x1 = x2; x2 = t; }
        return P.payout * (norm_cdf(x1 / P.sqh) + norm_cdf(-x2 / P.sqh));
    }
    if (B != Real(0)) return P.payout * norm_cdf(c0 / (fabs(B) * P.sqh));
    return c0 > Real(0) ? P.payout : (c0 == Real(0) ? Real(0.5) * P.payout : Real(0));
}

// The conditional digital of a path pair: expectation of the digital given
// every increment but the last fine one.  Given it, the last fine step is
// A + B x + C x^2 with x the last increment: Euler A = S (1 + r h),
// B = vol S, C = 0; Milstein A = S (1 + (r - sigma^2/2) h), B = sigma S,
// C = sigma^2 S / 2.  The coarse path's last step has the known part
// w = (its increment) - x: Euler A = S (1 + r H + vol w), B = vol S;
// Milstein A = S (1 + (r - sigma^2/2) H + sigma w + sigma^2 w^2 / 2),
// B = sigma S (1 + sigma w), C = sigma^2 S / 2.  Discounted; NaN when the
// path overflowed.
template <typename Real, int MODEL>
__device__ __forceinline__ Real cond_digital_fine(const StepParams<Real>& P, const PathPair<Real>& q)
{
    Real A, B = q.vl * q.Sl, C = Real(0);
    if (MODEL == kGBMMil) {
        A = fmaT(q.Sl, P.rh_m, q.Sl);
        C = P.c2 * q.Sl;
    } else {
        A = fmaT(q.Sl, P.rh, q.Sl);
    }
    return P.disc * digital_given(P, A, B, C) + (q.S - q.S);
}

template <typename Real, int MODEL>
__device__ __forceinline__ Real cond_digital_coarse(const StepParams<Real>& P, const PathPair<Real>& q)
{
    const Real w = q.wcl - q.dwl;
    Real A, B, C = Real(0);
    if (MODEL == kGBMMil) {
        A = fmaT(q.Scl, fmaT(P.c2, w * w, fmaT(P.sigma, w, P.rH_m)), q.Scl);
        B = P.sigma * q.Scl * fmaT(P.sigma, w, Real(1));
        C = P.c2 * q.Scl;
    } else {
        A = fmaT(q.Scl, fmaT(q.vcl, w, P.rH), q.Scl);
        B = q.vcl * q.Scl;
    }
    return P.disc * digital_given(P, A, B, C) + (q.Sc - q.Sc);
}

}  // namespace mlmc
