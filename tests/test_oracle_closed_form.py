"""Pins for the oracle's closed forms (CPU only).

Each closed form is checked by an independent computation: numerical
integration against the relevant density, Gauss--Hermite quadrature (exact for
the polynomial Euler moments), exact simulation, or a limiting case.
"""
import itertools

import numpy as np
from numpy.polynomial.hermite_e import hermegauss
from scipy import integrate, stats

S0, K, R, SIG, T = 100.0, 100.0, 0.05, 0.2, 1.0


def lognormal_expect(f, S0, r, sigma, T):
    """E[f(S_T)] for exact GBM by quadrature over the normal density."""
    g = lambda z: f(S0 * np.exp((r - 0.5 * sigma**2) * T + sigma * np.sqrt(T) * z)) \
        * stats.norm.pdf(z)
    return integrate.quad(g, -12, 12, limit=400, points=[0.0])[0]


def test_black_scholes_call_and_digital(orc):
    for sigma in (0.2, 0.25):
        disc = np.exp(-R * T)
        call = disc * lognormal_expect(lambda s: max(s - K, 0.0), S0, R, sigma, T)
        assert abs(orc.bs_call(S0, K, R, sigma, T) - call) < 1e-7
        dig = disc * stats.lognorm.sf(K, s=sigma * np.sqrt(T),
                                      scale=S0 * np.exp((R - 0.5 * sigma**2) * T))
        assert abs(orc.bs_digital(S0, K, R, sigma, T, 1.0) - dig) < 1e-12
        assert abs(orc.bs_digital(S0, K, R, sigma, T, 100.0) - 100 * dig) < 1e-10


def test_lookback_by_exact_simulation(orc):
    # ln S is Brownian with drift, so simulating it on a grid and sampling the
    # minimum of each step's bridge exactly gives the continuous minimum.
    rng = np.random.default_rng(11)
    n, steps = 200000, 16
    h = T / steps
    mu = (R - 0.5 * SIG**2) * h
    x = np.zeros(n)
    mn = np.zeros(n)
    for _ in range(steps):
        x1 = x + mu + SIG * np.sqrt(h) * rng.standard_normal(n)
        u = rng.random(n)
        m = 0.5 * (x + x1 - np.sqrt((x1 - x) ** 2 - 2 * SIG**2 * h * np.log(u)))
        mn = np.minimum(mn, m)
        x = x1
    pay = np.exp(-R * T) * S0 * (np.exp(x) - np.exp(mn))
    est, se = pay.mean(), pay.std() / np.sqrt(n)
    assert abs(orc.lookback_float_call(S0, R, SIG, T) - est) < 4 * se


def test_geometric_asian_by_distribution(orc):
    # int_0^T W dt ~ N(0, T^3/3): check the price by quadrature over that law
    var = SIG**2 * T / 3
    mu = np.log(S0) + 0.5 * (R - 0.5 * SIG**2) * T
    g = lambda z: max(np.exp(mu + np.sqrt(var) * z) - K, 0.0) * stats.norm.pdf(z)
    ref = np.exp(-R * T) * integrate.quad(g, -12, 12, limit=400)[0]
    assert abs(orc.geometric_asian_call(S0, K, R, SIG, T) - ref) < 1e-8
    # and the variance of the time integral of W by simulation
    rng = np.random.default_rng(5)
    W = np.cumsum(rng.standard_normal((20000, 400)) * np.sqrt(1 / 400), axis=1)
    assert abs(W.mean(axis=1).var() - 1 / 3) < 0.02


def test_heston_small_volofvol_limit(orc):
    # xi -> 0 with rho = 0: variance is deterministic, price -> Black-Scholes
    # with the average variance.
    kappa, theta, v0 = 2.0, 0.04, 0.09
    vbar = theta + (v0 - theta) * (1 - np.exp(-kappa * T)) / (kappa * T)
    bs = orc.bs_call(S0, K, R, np.sqrt(vbar), T)
    h = orc.heston_call(S0, K, R, T, kappa, theta, 1e-3, 0.0, v0)
    assert abs(h - bs) < 1e-4


def test_heston_against_fine_simulation(orc):
    # independent numpy full-truncation Euler at a fine step; bias O(h)
    rng = np.random.default_rng(21)
    n, steps = 100000, 256
    h = T / steps
    kappa, theta, xi, rho, v0 = 2.0, 0.04, 0.3, -0.7, 0.04
    lnS = np.full(n, np.log(S0))
    v = np.full(n, v0)
    for _ in range(steps):
        z1 = rng.standard_normal(n)
        z2 = rho * z1 + np.sqrt(1 - rho**2) * rng.standard_normal(n)
        vp = np.maximum(v, 0)
        lnS += (R - 0.5 * vp) * h + np.sqrt(vp * h) * z1
        v += kappa * (theta - vp) * h + xi * np.sqrt(vp * h) * z2
    pay = np.exp(-R * T) * np.maximum(np.exp(lnS) - K, 0)
    est, se = pay.mean(), pay.std() / np.sqrt(n)
    assert abs(orc.heston_call() - est) < 4 * se + 0.02


def test_heston_put_call_parity_and_moneyness(orc):
    # call price is decreasing and convex in K, within no-arbitrage bounds
    ks = [80.0, 90.0, 100.0, 110.0, 120.0]
    c = [orc.heston_call(K=k) for k in ks]
    assert all(a > b for a, b in zip(c, c[1:]))
    assert all(c[i - 1] - 2 * c[i] + c[i + 1] > 0 for i in range(1, 4))
    for k, ci in zip(ks, c):
        assert max(S0 - k * np.exp(-R * T), 0) < ci < S0


def _euler_moments_quadrature(l, M, sigma=SIG, r=R):
    """Exact E[P_l] and Var[P_l - P_{l-1}] for K = 0 by tensor Gauss-Hermite."""
    nf = M**l
    h = T / nf
    x, w = hermegauss(3)          # exact for degree <= 5 per variable
    w = w / w.sum()
    disc = np.exp(-r * T)
    E1 = E2 = 0.0
    for idx in itertools.product(range(3), repeat=nf):
        z = x[list(idx)]
        wt = np.prod(w[list(idx)])
        dW = np.sqrt(h) * z
        sf = S0 * np.prod(1 + r * h + sigma * dW)
        if l == 0:
            d = sf
        else:
            H = M * h
            sc = S0 * np.prod(1 + r * H + sigma * dW.reshape(-1, M).sum(axis=1))
            d = sf - sc
        E1 += wt * sf
        E2 += wt * d * d
    mean_d = E1 - (S0 * (1 + r * M * h) ** (nf // M) if l else 0.0)
    return disc * E1, disc**2 * (E2 - mean_d**2)


def test_euler_k0_moments_by_quadrature(orc):
    for (l, M) in [(0, 2), (1, 2), (2, 2), (1, 4), (3, 2)]:
        e, v = orc.euler_k0_moments(S0, R, SIG, T, l, M)
        qe, qv = _euler_moments_quadrature(l, M)
        assert abs(e - qe) < 1e-10 * qe
        assert abs(v - qv) < 1e-9 * qv


def test_level0_call_moments_by_quadrature(orc):
    disc = np.exp(-R * T)
    f = lambda z: max(S0 * (1 + R * T + SIG * np.sqrt(T) * z) - K, 0.0)
    m1 = integrate.quad(lambda z: f(z) * stats.norm.pdf(z), -12, 12, points=[-0.25])[0]
    m2 = integrate.quad(lambda z: f(z) ** 2 * stats.norm.pdf(z), -12, 12, points=[-0.25])[0]
    e, v = orc.level0_call_moments(S0, K, R, SIG, T)
    assert abs(e - disc * m1) < 1e-9
    assert abs(v - disc**2 * (m2 - m1 * m1)) < 1e-7
