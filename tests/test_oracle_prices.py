"""Closed-form pins of the oracle's path-dependent and stochastic-volatility
samplers (CPU only).

The telescoping identity (eq. (eq:mlmc:ident)) makes the sum of the level
means of levels 0..L equal E[P_L], the payoff of the finest Euler path, and
weak order one (eq. (eq:emweak)) puts E[P_L] within O(dt_L) of the
continuous-time price.  Each test below runs the oracle's level sampler with
sample counts from the variance/cost rule of Sec. 5 for a target standard
deviation, and requires

    |sum_l Yhat_l - price| <= 4 sd + |Yhat_L| / (M - 1)

where the last term is the bias estimate that weak order one gives from the
finest level (sum_{k > L} E[Y_k] ~ E[Y_L] / (M - 1)).  The prices do not come
from the sampler:
  - floating-strike lookback (named in Sec. 7.1): Goldman, Sosin and Gatto's
    continuous-monitoring formula (oracle closed form, itself pinned against
    exact simulation of the log price with exact bridge minima);
  - Heston call: the characteristic-function formula (oracle closed form,
    pinned by its xi -> 0 limit, parity and a fine simulation), at the
    configuration's strike 100 and at 120, where the sign of the correlation
    moves the price by 1.5;
  - arithmetic Asian (named in Sec. 7.1): no closed form; Vecer's
    one-dimensional PDE for the continuous average, solved by the oracle's
    Crank--Nicolson module (checked here against its exact K = 0 value, its
    zero-volatility limit and by grid refinement), and the continuous geometric Asian as a strict lower bound
    (arithmetic >= geometric mean).
Plausible slips fail: a bridge minimum without its correction term is off by
about 0.6 sigma sqrt(h) S0 (0.7 at h = 1/256), the opposite correlation sign
by 0.34 (K = 100) and 1.5 (K = 120).
"""
import math
import os

import numpy as np
import pytest

NTHREADS = max(1, min(8, os.cpu_count() or 1))


def mlmc_fixed(orc, m, p, M, L, sd, seed, pilot=20000):
    """Levels 0..L with N_l = ceil(sd^-2 sqrt(V_l/C_l) sum_k sqrt(V_k C_k))
    (the Lagrange solution of Sec. 5's cost/variance balance for variance
    sd^2), V_l from a pilot of `pilot` samples that the final sums include."""
    cost = np.array([orc.level_cost(l, M) for l in range(L + 1)])
    s1, s2, n = np.zeros(L + 1), np.zeros(L + 1), np.zeros(L + 1)

    def add(l, count, offset):
        r = orc.level(m, p, l, M, count, seed, offset, nthreads=NTHREADS)
        s1[l] += r["sum_y"]
        s2[l] += r["sum_y2"]
        n[l] += count

    for l in range(L + 1):
        add(l, pilot, 0)
    V = s2 / n - (s1 / n) ** 2
    N = np.ceil(np.sqrt(V / cost) * np.sum(np.sqrt(V * cost)) / sd**2)
    for l in range(L + 1):
        if N[l] > n[l]:
            add(l, int(N[l] - n[l]), int(n[l]))
    mean = s1 / n
    V = s2 / n - mean**2
    return {"estimate": float(mean.sum()), "sd": math.sqrt(float(np.sum(V / n))),
            "E_L": float(mean[-1]), "sd_L": math.sqrt(float(V[-1] / n[-1])), "N": n, "V": V}


def check_price(res, price, M, what):
    bias = abs(res["E_L"]) / (M - 1)
    tol = 4.0 * math.hypot(res["sd"], res["sd_L"] / (M - 1)) + bias
    err = res["estimate"] - price
    assert abs(err) <= tol, f"{what}: telescoped {res['estimate']:.5f} vs {price:.5f} (|err| {abs(err):.4f} > {tol:.4f})"
    return err, tol


@pytest.mark.parametrize("M,L", [(2, 8), (4, 5)])
def test_lookback_telescopes_to_goldman_sosin_gatto(orc, M, L):
    m, p = orc.model(), orc.payoff(kind=orc.LOOKBACK)
    price = orc.lookback_float_call()
    assert abs(price - 17.216802) < 1e-6
    res = mlmc_fixed(orc, m, p, M, L, 0.005, seed=11)
    check_price(res, price, M, f"lookback M={M} L={L}")
    # the bridge term matters: the discretely monitored minimum alone would
    # sit ~0.58 sigma sqrt(h_L) S0 above the continuous one (Broadie,
    # Glasserman and Kou's shift), far outside the tolerance at these h
    h = 1.0 / M**L
    assert 0.5826 * 0.2 * math.sqrt(h) * 100.0 > 10 * 4 * res["sd"]


@pytest.mark.parametrize("K", [100.0, 120.0])
def test_heston_telescopes_to_characteristic_function_price(orc, K):
    m, p = orc.model(kind=orc.HESTON), orc.payoff(kind=orc.CALL, K=K)
    price = orc.heston_call(K=K)
    if K == 100.0:
        assert abs(price - 10.394219) < 1e-6
    res = mlmc_fixed(orc, m, p, 4, 5, 0.006, seed=11)
    err, tol = check_price(res, price, 4, f"Heston call K={K}")
    # the opposite correlation is far outside the tolerance
    assert abs(orc.heston_call(K=K, rho=0.7) - price) > 5 * tol


def test_vecer_pde_solver(orc):
    vecer_asian_call = orc.asian_arith_call_pde
    # K = 0: the discounted mean of the average, S0 (1 - e^{-rT}) / (rT)
    assert abs(vecer_asian_call(100.0, 0.0, 0.05, 0.2, 1.0) - 100 * (1 - math.exp(-0.05)) / 0.05) < 1e-9
    # grid refinement and a wider domain move the price by < 1e-4
    a = vecer_asian_call(100.0, 100.0, 0.05, 0.2, 1.0)
    b = vecer_asian_call(100.0, 100.0, 0.05, 0.2, 1.0, nz=8000, nt=4000)
    c = vecer_asian_call(100.0, 100.0, 0.05, 0.2, 1.0, nz=9000, zlo=-4.0, zhi=5.0)
    assert abs(a - b) < 1e-4 and abs(a - c) < 1e-4
    # almost no volatility: the forward of the average, max(S0 z0, 0)
    z0 = (1 - math.exp(-0.05)) / 0.05 - math.exp(-0.05)
    assert abs(vecer_asian_call(100.0, 100.0, 0.05, 1e-4, 1.0) - 100 * z0) < 1e-3


@pytest.mark.parametrize("M,L", [(2, 8), (4, 5)])
def test_asian_telescopes_to_continuous_average_price(orc, M, L):
    m, p = orc.model(), orc.payoff(kind=orc.ASIAN)
    price = orc.asian_arith_call_pde(100.0, 100.0, 0.05, 0.2, 1.0)
    geo = orc.geometric_asian_call()
    assert abs(geo - 5.546819) < 1e-6 and price > geo
    res = mlmc_fixed(orc, m, p, M, L, 0.003, seed=11)
    check_price(res, price, M, f"Asian M={M} L={L}")
    # arithmetic mean >= geometric mean, path by path
    assert res["estimate"] - 4 * res["sd"] > geo
