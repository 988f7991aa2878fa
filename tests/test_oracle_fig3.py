"""Sec. 6 (Fig. 3) on the oracle: the qualitative claims the paper makes about
its one experiment, checked on the fp64 CPU driver at the larger accuracy
requests (the GPU test runs all five).

The paper prints no numbers for Fig. 3, only shapes: more paths on the cheap
levels; levels added as eps falls; eps^2 x cost about constant for the call
(Euler with a Lipschitz payoff, so the cost grows like eps^-2 (log eps)^2);
standard Monte Carlo on the finest grid costing more and growing faster
(eps^-3 for weak order 1); the same ordering for the digital.
"""
import numpy as np
import pytest

from paper_1505_00965_amd import workloads as W


def level_cost(l, M):
    return 1.0 if l == 0 else float(M ** l + M ** (l - 1))


def sweep(orc, pay, eps_list):
    m, p = orc.model(**W.FIG3_MODEL), orc.payoff(**pay)
    R = W.FIG3_RUN
    out = []
    for i, eps in enumerate(eps_list):
        r = orc.mlmc_run(m, p, eps, M=R["M"], L_min=R["L_min"], L_max=R["L_max"],
                         n_pilot=R["n_pilot"], seed=1 + 1000 * i, nthreads=8)
        assert r["converged"]
        L = r["L"]
        cost = sum(n * level_cost(l, R["M"]) for l, n in enumerate(r["N"]))
        # standard MC on the finest grid: sample variance eps^2 / 2
        s = orc.stdmc(m, p, L, R["M"], 20000, 1 + 1000 * i, nthreads=8)
        v = s["sum_pf2"] / s["n"] - (s["sum_pf"] / s["n"]) ** 2
        std = np.ceil(2 * v / eps ** 2) * R["M"] ** L
        out.append(dict(eps=eps, L=L, N=r["N"], cost=cost, std=std, est=r["estimate"]))
    return out


def test_fig3_call_shapes(orc):
    recs = sweep(orc, W.FIG3_CALL, W.FIG3_EPS[:4])
    for r in recs:
        print(r["eps"], r["L"], r["N"], r["cost"] * r["eps"] ** 2, r["std"] * r["eps"] ** 2)
        assert all(b < a for a, b in zip(r["N"], r["N"][1:])), r["N"]
        assert r["std"] > 2 * r["cost"]
        exact = orc.bs_call(100.0, 100.0, 0.05, 0.25, 1.0)
        assert abs(r["est"] - exact) < 3 * r["eps"]
    Ls = [r["L"] for r in recs]
    assert all(b >= a for a, b in zip(Ls, Ls[1:])) and Ls[-1] > Ls[0]
    e2m = [r["cost"] * r["eps"] ** 2 for r in recs]
    e2s = [r["std"] * r["eps"] ** 2 for r in recs]
    assert e2s[-1] > 4 * e2s[0]                  # about eps^-1 growth over a decade
    assert max(e2m) / min(e2m) < 3.0             # roughly flat
    assert max(e2m) / min(e2m) < (e2s[-1] / e2s[0]) / 2


def test_fig3_digital_shapes(orc):
    recs = sweep(orc, W.FIG3_DIGITAL, W.FIG3_EPS[:2])
    for r in recs:
        print(r["eps"], r["L"], r["N"], r["cost"] * r["eps"] ** 2, r["std"] * r["eps"] ** 2)
        assert all(b < a for a, b in zip(r["N"], r["N"][1:])), r["N"]
        assert r["std"] > r["cost"]
        exact = orc.bs_digital(100.0, 100.0, 0.05, 0.25, 1.0, payout=100.0)
        assert abs(r["est"] - exact) < 3 * r["eps"]
    assert recs[1]["L"] > recs[0]["L"]
