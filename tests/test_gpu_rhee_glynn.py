"""Randomised single-term estimator on the GPU vs the oracle.

Level draws are integer work: the per-level counts must equal the oracle's
bit for bit.  fp64 level sums and the estimate match the oracle to 1e-9;
fp32 Milstein estimates average to the Black--Scholes price.
"""
import numpy as np
import pytest

from paper_1505_00965_amd import mlmc, workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M,Lc,q", [(2, 15, 2.0**-1.5), (4, 9, 4.0**-1.5), (2, 6, 0.6)])
def test_counts_and_fp64_sums_equal_the_oracle(gctx, orc, M, Lc, q):
    md = dict(W.GBM_MODEL, scheme=1)
    gm, om = mlmc.model(**md), orc.model(**md)
    for pname in ("call", "asian"):
        gp, op = mlmc.payoff(**W.PAYOFFS[pname]), orc.payoff(**W.PAYOFFS[pname])
        for N, seed in ((1, 3), (4097, 5), (200003, 11)):
            g = gctx.mlmc_rhee_glynn(gm, gp, M, Lc, q, N, seed, precision=64)
            o = orc.rhee_glynn(om, op, M, Lc, q, N, seed, nthreads=8)
            assert g["N"] == o["N"], (N, seed)
            assert sum(g["N"]) == N
            for l in range(Lc + 1):
                assert abs(g["sum_y"][l] - o["sum_y"][l]) <= 1e-9 * max(1.0, abs(o["sum_y"][l]))
            assert abs(g["estimate"] - o["estimate"]) <= 1e-9 * max(1.0, abs(o["estimate"]))
            assert g["cost"] == o["cost"]


def test_unbiased_fp32_milstein(gctx, orc):
    gm = mlmc.model(**dict(W.GBM_MODEL, scheme=1))
    gp = mlmc.payoff(**W.CALL)
    est = np.array([gctx.mlmc_rhee_glynn(gm, gp, 2, 15, 2.0**-1.5, 1 << 20, s)["estimate"]
                    for s in range(1, 31)])
    se = est.std(ddof=1) / np.sqrt(est.size)
    print("mean", est.mean(), "bs", orc.bs_call(), "se", se)
    assert abs(est.mean() - orc.bs_call()) < 4.5 * se + 2e-4


def test_bad_arguments(gctx):
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    for kw in (dict(M=2, L_cap=16, q=0.5, N=10), dict(M=4, L_cap=10, q=0.5, N=10),
               dict(M=2, L_cap=5, q=1.0, N=10), dict(M=2, L_cap=5, q=0.5, N=0)):
        with pytest.raises(mlmc.MLMCError) as e:
            gctx.mlmc_rhee_glynn(gm, gp, kw["M"], kw["L_cap"], kw["q"], kw["N"], 1)
        assert e.value.status == mlmc.MLMC_EINVAL
