"""GPU adaptive driver vs the oracle's driver and the closed form.

The N_l arithmetic runs on the device in fp64 and must equal the oracle's
bit for bit; a whole fp64 run must take the same decisions as the oracle's
(same L, same N_l, same iterations); fp32 runs must meet the complexity
theorem's E[(Y - E P)^2] < eps^2 over independent seeds.
"""
import numpy as np
import pytest

from paper_1505_00965_amd import mlmc, workloads as W

pytestmark = pytest.mark.gpu


def test_optimal_n_bit_exact(gctx, orc):
    rng = np.random.default_rng(1)
    for _ in range(50):
        L = int(rng.integers(0, 10))
        V = 10.0 ** rng.uniform(-6, 3, size=L + 1)
        C = np.array([orc.level_cost(l, 4) for l in range(L + 1)])
        eps = float(10.0 ** rng.uniform(-3, 0))
        g = np.array(gctx.mlmc_optimal_n(list(V), list(C), eps))
        o = orc.optimal_n(V, C, eps)
        assert np.array_equal(g, o), (g, o)


@pytest.mark.parametrize("eps,M", [(0.2, 4), (0.1, 4), (0.05, 2)])
def test_fp64_run_takes_the_oracle_decisions(gctx, orc, eps, M):
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    om, op = orc.model(**W.GBM_MODEL), orc.payoff(**W.CALL)
    g = gctx.mlmc_run(gm, gp, eps, M=M, seed=3, precision=64)
    o = orc.mlmc_run(om, op, eps, M=M, seed=3, nthreads=8)
    print("gpu", g["N"], g["estimate"], "oracle", o["N"], o["estimate"])
    assert g["L"] == o["L"] and g["iterations"] == o["iterations"]
    assert g["N"] == o["N"]
    assert abs(g["estimate"] - o["estimate"]) <= 1e-9 * abs(o["estimate"])
    assert g["converged"]


@pytest.mark.parametrize("pname,kind", [("call", 0), ("asian", 0), ("lookback", 0), ("call", 1)])
def test_fp32_run_close_to_oracle_run(gctx, orc, pname, kind):
    md = W.GBM_MODEL if kind == 0 else W.HESTON_MODEL
    gm, gp = mlmc.model(**md), mlmc.payoff(**W.PAYOFFS[pname])
    om, op = orc.model(**md), orc.payoff(**W.PAYOFFS[pname])
    g = gctx.mlmc_run(gm, gp, 0.1, M=4, seed=5, precision=32)
    o = orc.mlmc_run(om, op, 0.1, M=4, seed=5, nthreads=8)
    # the fp32 variance estimates take the oracle's decisions, so both runs
    # sum the same samples
    assert g["L"] == o["L"] and g["N"] == o["N"]
    # every sample's Y is within the per-path bound 1e-4 S0 of the oracle's,
    # so each level sum within N_l of it and the estimate within (L+1) of it
    delta = 1e-4 * md["S0"]
    for l, n in enumerate(o["N"][:o["L"] + 1]):
        assert abs(g["sum_y"][l] - o["sum_y"][l]) <= n * delta, (l, g["sum_y"][l], o["sum_y"][l])
    diff = abs(g["estimate"] - o["estimate"])
    print(f"{pname} kind {kind}: |fp32 estimate - oracle| = {diff:.3e} (bound {(o['L'] + 1) * delta})")
    assert diff <= (o["L"] + 1) * delta


def test_rmse_over_seeds_fp32(gctx, orc):
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    eps = 1e-3 * 100
    exact = orc.bs_call()
    errs = []
    for seed in range(1, 33):
        r = gctx.mlmc_run(gm, gp, eps, M=4, seed=seed)
        assert r["converged"]
        errs.append(r["estimate"] - exact)
    rmse = float(np.sqrt(np.mean(np.square(errs))))
    print("rmse", rmse)
    assert rmse < 1.35 * eps


def test_notconv_and_bad_args(gctx):
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    r = gctx.mlmc_run(gm, gp, 0.002, M=4, L_min=2, L_max=2, n_pilot=2000, allow_notconv=True)
    assert not r["converged"] and r["L"] == 2
    with pytest.raises(mlmc.MLMCError) as e:
        gctx.mlmc_run(gm, gp, 0.002, M=4, L_min=2, L_max=2, n_pilot=2000)
    assert e.value.status == mlmc.MLMC_ENOTCONV
    for kw in (dict(eps=-1.0), dict(eps=0.1, L_min=3, L_max=2), dict(eps=0.1, M=3),
               dict(eps=0.1, n_pilot=1)):
        eps = kw.pop("eps")
        with pytest.raises(mlmc.MLMCError) as e:
            gctx.mlmc_run(gm, gp, eps, **kw)
        assert e.value.status == mlmc.MLMC_EINVAL


def test_timing_mask_records_only_its_slots(gctx):
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    gctx.set_timing_slots([0, mlmc.STAT_DRIVER])
    r = gctx.mlmc_run(gm, gp, 0.05, M=4, seed=2)
    st = gctx.kernel_stats()
    gctx.set_timing(False)
    assert st[0]["launches"] >= 1 and st[0]["ms"] > 0
    assert st[0]["fine_steps"] == sum(r["N"][:1])          # level 0: one step per sample
    assert st[mlmc.STAT_DRIVER]["launches"] == r["iterations"]
    assert all(st[l]["launches"] == 0 for l in range(1, 16))
    with pytest.raises(mlmc.MLMCError) as e:
        gctx._check(gctx._lib.mlmc_set_timing_mask(gctx.h, 1 << mlmc.STAT_SLOTS))
    assert e.value.status == mlmc.MLMC_EINVAL
    # all slots again, then off
    gctx.set_timing(True)
    gctx.mlmc_run(gm, gp, 0.05, M=4, seed=2)
    st = gctx.kernel_stats()
    gctx.set_timing(False)
    assert all(st[l]["launches"] >= 1 for l in range(r["L"] + 1))


def test_timing_stride_stamps_one_launch_in_k(gctx):
    """With stride k the slot's statistics cover launches 1, k+1, 2k+1, ...
    of the slot: ceil(n/k) of its n launches, here level-0 launches of
    fixed size, so the sampled average is that of every launch."""
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    N = 1 << 16
    for k, n in ((1, 7), (3, 7), (4, 8), (9, 5)):
        gctx.set_timing_slots([0])
        gctx.set_timing_stride(k)
        for i in range(n):
            gctx.mlmc_level(gm, gp, 0, 4, N, 1 + i)
        st = gctx.kernel_stats()[0]
        gctx.set_timing(False)
        gctx.set_timing_stride(1)
        assert st["launches"] == -(-n // k), (k, n, st)
        assert st["fine_steps"] == st["launches"] * N and st["ms"] > 0
    with pytest.raises(mlmc.MLMCError) as e:
        gctx.set_timing_stride(0)
    assert e.value.status == mlmc.MLMC_EINVAL
    # paused: nothing stamped, the statistics kept; whole runs stamped
    gctx.set_timing_slots([mlmc.STAT_PERSISTENT])
    runs = []
    for i in range(4):
        gctx.set_timing_paused(i % 2 == 1)
        runs.append(gctx.mlmc_run(gm, gp, 0.05, M=4, seed=2 + i, persistent=1))
    gctx.set_timing_paused(False)
    st = gctx.kernel_stats()[mlmc.STAT_PERSISTENT]
    gctx.set_timing(False)
    assert st["launches"] == sum(r["iterations"] + 1 for r in runs[::2])
    assert st["fine_steps"] == sum(n * 4**l for r in runs[::2] for l, n in enumerate(r["N"]))


@pytest.mark.parametrize("persistent", [False, True])
def test_timed_runs_give_the_untimed_results(gctx, persistent):
    """Kernel timing changes only how launches are stamped: the estimates,
    N_l and level sums of a timed run are the untimed run's."""
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    runs = []
    for mode in ("off", "all", "level0"):
        if mode == "all":
            gctx.set_timing(True)
        elif mode == "level0":
            gctx.set_timing_slots([0])
        rs = [gctx.mlmc_run(gm, gp, 0.01, M=4, seed=s, persistent=persistent) for s in (3, 4)]
        gctx.set_timing(False)
        runs.append(rs)
    for rs in runs[1:]:
        for a, b in zip(runs[0], rs):
            assert a["N"] == b["N"] and a["L"] == b["L"]
            assert abs(a["estimate"] - b["estimate"]) <= 1e-12 * abs(a["estimate"])


def test_first_run_of_a_context_equals_later_runs():
    """A context's first run clears the driver state and spread groups with
    a kernel; later runs (after a normal end) let the first update build the
    state.  Both must give the same run, also after runs of other shapes and
    after a run that stopped with an error."""
    from paper_1505_00965_amd import mlmc as m_
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    ctx = m_.Context(0)
    try:
        first = ctx.mlmc_run(gm, gp, 0.01, M=4, seed=12)
        others = [ctx.mlmc_run(gm, mlmc.payoff(**W.ASIAN), 0.02, M=2, seed=3),
                  ctx.mlmc_run(gm, gp, 0.005, M=4, seed=5, persistent=1)]
        with pytest.raises(mlmc.MLMCError):
            ctx.mlmc_run(gm, gp, 0.002, M=4, L_min=2, L_max=2, n_pilot=2000)   # ENOTCONV
        again = [ctx.mlmc_run(gm, gp, 0.01, M=4, seed=12) for _ in range(2)]
    finally:
        ctx.close()
    assert all(o["converged"] for o in others)
    for r in again:
        assert r["N"] == first["N"] and r["L"] == first["L"]
        assert r["iterations"] == first["iterations"]
        assert abs(r["estimate"] - first["estimate"]) <= 1e-12 * abs(first["estimate"])
