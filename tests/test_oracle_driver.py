"""Pins for the oracle's MLMC driver (CPU only).

The paper leaves the choice of N_l to an optimisation (Sec. 5, "Constructive
Upper Bound") and states the theorem's target E[(Y - E P)^2] < eps^2.  The
sample-count formula is pinned against a numerical constrained minimisation;
the whole driver against the closed-form price over independent seeds.
"""
import numpy as np
import pytest
from scipy import optimize


def test_optimal_n_solves_the_allocation_problem(orc):
    rng = np.random.default_rng(0)
    for trial in range(5):
        L = int(rng.integers(1, 7))
        V = 10.0 ** rng.uniform(-4, 2, size=L + 1)
        Cl = np.array([orc.level_cost(l, 4) for l in range(L + 1)])
        eps = 0.05
        N = orc.optimal_n(V, Cl, eps)
        # minimise sum N C subject to sum V/N = eps^2/2 numerically in log N
        cons = {"type": "eq", "fun": lambda x: np.sum(V / np.exp(x)) / (eps**2 / 2) - 1}
        x0 = np.log(N)
        res = optimize.minimize(lambda x: np.sum(np.exp(x) * Cl) / np.sum(N * Cl), x0 + 0.3,
                                constraints=[cons], method="SLSQP",
                                options={"ftol": 1e-14, "maxiter": 500})
        assert res.success
        assert np.allclose(np.exp(res.x), N, rtol=2e-3, atol=1.0)
        assert np.all(N == np.ceil(N))
        assert np.sum(V / N) <= eps**2 / 2 * (1 + 1e-12)


def test_level_cost(orc):
    assert orc.level_cost(0, 4) == 1
    assert orc.level_cost(1, 4) == 5
    assert orc.level_cost(8, 4) == 4**8 + 4**7


def test_fit_rate(orc):
    y = [5.0] + [3.0 * 4.0 ** (-1.5 * l) for l in range(1, 6)]
    assert abs(orc.fit_rate(y, 4) + 1.5) < 1e-12


def test_rmse_over_seeds(orc):
    # E[(Y - E P)^2] < eps^2 (complexity theorem), with a sampling margin
    m, p = orc.model(), orc.payoff()
    eps = 0.2              # 2e-3 * S0
    exact = orc.bs_call()
    errs = []
    for seed in range(1, 33):
        r = orc.mlmc_run(m, p, eps, M=4, seed=seed, nthreads=8)
        assert r["converged"]
        errs.append(r["estimate"] - exact)
        V = np.maximum(np.array(r["V"]), 0)
        assert np.sum(V / np.array(r["N"])) <= eps**2 / 2 * 1.05
    rmse = np.sqrt(np.mean(np.square(errs)))
    assert rmse < eps * 1.35, (rmse, errs)


def test_driver_shape(orc):
    # more paths on cheap levels; more levels as eps falls (Sec. 6 description)
    m, p = orc.model(), orc.payoff()
    r1 = orc.mlmc_run(m, p, 0.2, M=4, seed=3, nthreads=8)
    r2 = orc.mlmc_run(m, p, 0.02, M=4, seed=3, nthreads=8)
    for r in (r1, r2):
        # non-increasing (levels held at the pilot count tie), strictly overall
        assert all(a >= b for a, b in zip(r["N"], r["N"][1:]))
        assert r["N"][0] > r["N"][-1]
    assert r2["L"] >= r1["L"]
    assert r2["N"][0] > r1["N"][0]
    assert 0.5 < r2["beta"] < 1.6 and 0.9 < r2["gamma"] < 1.1


def test_lmax_reached_without_convergence(orc):
    m, p = orc.model(), orc.payoff()
    r = orc.mlmc_run(m, p, 0.002, M=4, L_min=2, L_max=2, n_pilot=2000, seed=1, nthreads=8)
    assert r["L"] == 2 and not r["converged"]


def test_bad_arguments(orc):
    m, p = orc.model(), orc.payoff()
    with pytest.raises(ValueError):
        orc.mlmc_run(m, p, -1.0)
    with pytest.raises(ValueError):
        orc.mlmc_run(m, p, 0.1, L_min=3, L_max=2)
