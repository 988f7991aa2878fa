"""Conditional digital on the GPU vs the oracle.

Per path |dP| <= 1e-4 S0 (fp32 paths) and 1e-9 S0 (fp64) with payout 1:
the conditional payoff is smooth in the path state, so unlike the plain
digital no sample may flip.  fp64 adaptive runs take the oracle's decisions.
"""
import numpy as np
import pytest

from paper_1505_00965_amd import mlmc, workloads as W

pytestmark = pytest.mark.gpu
S0 = 100.0
VARIANTS = [(0, 0, 0), (0, 1, 0), (1, 0, 0), (0, 0, 1), (0, 1, 1), (1, 0, 1)]
CASES = [(2, 0), (2, 1), (2, 2), (2, 5), (4, 1), (4, 2), (4, 4)]


def models(orc, kind, scheme, anti):
    d = dict(W.GBM_MODEL if kind == 0 else W.HESTON_MODEL, scheme=scheme, antithetic=anti)
    return mlmc.model(**d), orc.model(**d)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("precision", [64, 32])
def test_per_path_parity(gctx, orc, variant, precision):
    import torch
    gm, om = models(orc, *variant)
    gp, op = mlmc.payoff(**W.DIGITAL_COND), orc.payoff(**W.DIGITAL_COND)
    N = 2000
    for (M, l) in CASES:
        for offset in (0, 9):
            print(f"case variant={variant} prec={precision} M={M} l={l} off={offset}", flush=True)
            pf = torch.empty(N, dtype=torch.float64, device="cuda")
            pc = torch.empty(N, dtype=torch.float64, device="cuda")
            res = gctx.mlmc_level_paths(gm, gp, l, M, N, 3, pf, pc, path_offset=offset,
                                        precision=precision)
            pf, pc = pf.cpu().numpy(), pc.cpu().numpy()
            rf, rc = orc.level_paths(om, op, l, M, N, 3, offset, nthreads=8)
            tol = 1e-9 * S0 if precision == 64 else 1e-4 * S0
            err = max(np.abs(pf - rf).max(), np.abs(pc - rc).max())
            assert err <= tol, (M, l, offset, err)
            y = pf - pc
            assert abs(res["sum_y"] - y.sum()) <= 1e-12 * max(1.0, np.abs(y).sum())
            if l == 0:
                assert np.ptp(pf) < 1e-12          # level 0 is deterministic


@pytest.mark.parametrize("variant", [(0, 0, 0), (0, 1, 0), (1, 0, 0)])
def test_fp64_run_takes_the_oracle_decisions(gctx, orc, variant):
    gm, om = models(orc, *variant)
    gp, op = mlmc.payoff(**W.DIGITAL_COND), orc.payoff(**W.DIGITAL_COND)
    for eps, M in ((0.01, 4), (0.005, 2)):
        g = gctx.mlmc_run(gm, gp, eps, M=M, seed=2, precision=64)
        o = orc.mlmc_run(om, op, eps, M=M, seed=2, nthreads=8)
        print(variant, eps, g["L"], g["N"])
        assert g["L"] == o["L"] and g["N"] == o["N"]
        assert abs(g["estimate"] - o["estimate"]) <= 1e-9 * abs(o["estimate"])


def test_conditioning_gain_on_the_gpu(gctx, orc):
    """Level variances of the plain and the conditional digital, Milstein."""
    gm = mlmc.model(**dict(W.GBM_MODEL, scheme=1))
    ratios, vc = [], []
    for l in range(3, 8):
        a = gctx.mlmc_level(gm, mlmc.payoff(**W.DIGITAL), l, 2, 1 << 20, 5)
        b = gctx.mlmc_level(gm, mlmc.payoff(**W.DIGITAL_COND), l, 2, 1 << 20, 5)
        va = a["sum_y2"] / a["n"] - (a["sum_y"] / a["n"]) ** 2
        vb = b["sum_y2"] / b["n"] - (b["sum_y"] / b["n"]) ** 2
        ratios.append(va / vb)
        vc.append(vb)
        # the same samples: the plain payoff minus the conditional one has mean zero
        assert abs(a["sum_y"] - b["sum_y"]) / a["n"] < 4.5 * np.sqrt(va / a["n"])
    beta = -np.polyfit(np.arange(3, 8), np.log2(vc), 1)[0]
    print("variance ratios", ratios, "beta", beta)
    assert min(ratios) > 100 and beta > 1.1
    # the telescoped conditional estimate is the Black--Scholes digital
    est, var = 0.0, 0.0
    for l in range(0, 8):
        r = gctx.mlmc_level(gm, mlmc.payoff(**W.DIGITAL_COND), l, 2, 1 << 20, 7)
        m_ = r["sum_y"] / r["n"]
        est += m_
        var += (r["sum_y2"] / r["n"] - m_ * m_) / r["n"]
    assert abs(est - orc.bs_digital()) < 4.5 * np.sqrt(var) + 2e-3


def test_conditional_digital_rejected_with_the_network(gctx):
    cv = mlmc.ControlVariate(gctx, 2)
    with pytest.raises(mlmc.MLMCError):
        gctx.mlmc_level(mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.DIGITAL_COND), 1, 4, 100, 1,
                        cv=cv)
    with pytest.raises(mlmc.MLMCError):
        cv.train(mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.DIGITAL_COND), M=4, lmax=1, steps=1,
                 batch=64, lr=1e-3, seed=1)
    cv.close()
