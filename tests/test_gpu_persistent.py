"""Persistent all-levels form vs the per-level sampler.

The persistent kernel draws exactly the samples the per-level launches draw
(same counters), so its (payoff, level) sums must equal mlmc_level's up to
fp64 summation order, whatever the item split and launch shape; the
graph-driven adaptive run must take the per-level run's decisions.
"""
import numpy as np
import pytest

from paper_1505_00965_amd import mlmc, workloads as W

pytestmark = pytest.mark.gpu


def close(a, b, rel=1e-11):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300) + 1e-13


@pytest.mark.parametrize("kind", [0, 1])
def test_batch_equals_per_level(gctx, kind):
    md = W.GBM_MODEL if kind == 0 else W.HESTON_MODEL
    gm = mlmc.model(**md)
    pays = [mlmc.payoff(**W.PAYOFFS[n]) for n in ("call", "asian", "lookback", "digital")]
    L, M = 5, 4
    N = [[int(2**16 // 4**l * (k + 1)) + 37 * l for l in range(L + 1)] for k in range(4)]
    N[2][3] = 0                      # an empty (payoff, level)
    offs = [[1000 * k + (l << 33) for l in range(L + 1)] for k in range(4)]
    for shape in [(256, 2, 4), (64, 1, 8), (512, 4, 2)]:
        gctx.set_persistent_launch(*shape)
        got = gctx.mlmc_levels_batch(gm, pays, M, L, N, seed=9, offsets=offs)
        for k, p in enumerate(pays):
            for l in range(L + 1):
                ref = gctx.mlmc_level(gm, p, l, M, N[k][l], 9, path_offset=offs[k][l])
                g = got[k][l]
                assert g["n"] == N[k][l]
                for key in ("sum_y", "sum_y2", "sum_pf", "sum_pc"):
                    assert close(g[key], ref[key]), (shape, k, l, key, g[key], ref[key])
    gctx.set_persistent_launch(0, 0, 0)


def test_batch_random_patterns(gctx):
    """Random (payoff, level) counts, zeros and single samples among them, on
    one to four payoffs and up to eight levels: the plan packs the non-empty
    pairs and gives each its items; every pair must equal its own launch."""
    import numpy as np
    rng = np.random.default_rng(2024)
    gm = mlmc.model(**W.GBM_MODEL)
    names = ("call", "asian", "lookback", "digital")
    for trial in range(6):
        npay = int(rng.integers(1, 5))
        L = int(rng.choice([0, 3, 7]))
        M = int(rng.choice([2, 4]))
        pays = [mlmc.payoff(**W.PAYOFFS[names[int(rng.integers(0, 4))]]) for _ in range(npay)]
        N = [[int(rng.choice([0, 1, 63, 257, 4099, 70001])) // (M ** min(l, 3)) + (l == L)
              for l in range(L + 1)] for _ in range(npay)]
        got = gctx.mlmc_levels_batch(gm, pays, M, L, N, seed=100 + trial)
        for k, p in enumerate(pays):
            for l in range(L + 1):
                g = got[k][l]
                assert g["n"] == N[k][l], (trial, k, l)
                if N[k][l] == 0:
                    assert g["sum_y"] == 0.0 and g["sum_y2"] == 0.0
                    continue
                ref = gctx.mlmc_level(gm, p, l, M, N[k][l], 100 + trial)
                # the same terms added in another order: the error is bounded
                # by a few ulps of sum |Y| <= sqrt(N sum Y^2)
                scale_y = (N[k][l] * ref["sum_y2"]) ** 0.5
                assert abs(g["sum_y"] - ref["sum_y"]) <= 1e-12 * scale_y + 1e-300, (trial, k, l)
                assert close(g["sum_y2"], ref["sum_y2"], 1e-11), (trial, k, l)


def test_graph_replay_with_new_sizes(gctx):
    gm = mlmc.model(**W.GBM_MODEL)
    pays = [mlmc.payoff(**W.CALL)]
    for rep, scale in enumerate((1, 3, 1, 2)):
        N = [[5000 * scale // (l + 1) for l in range(4)]]
        got = gctx.mlmc_levels_batch(gm, pays, 4, 3, N, seed=rep)
        for l in range(4):
            ref = gctx.mlmc_level(gm, pays[0], l, 4, N[0][l], rep)
            assert close(got[0][l]["sum_y"], ref["sum_y"]), (rep, l)


def test_mlmc_shaped_batch_full_size(gctx, orc):
    """The benchmark's MLMC-shaped launch: N_l = 2^26 4^-l, l = 0..8, four payoffs;
    per-level means within 5 sigma of independent oracle estimates."""
    gm = mlmc.model(**W.GBM_MODEL)
    names = ("call", "asian", "lookback", "digital")
    pays = [mlmc.payoff(**W.PAYOFFS[n]) for n in names]
    L = 8
    N = [[W.persistent_n(l) for l in range(L + 1)] for _ in pays]
    got = gctx.mlmc_levels_batch(gm, pays, 4, L, N, seed=1)
    om = orc.model(**W.GBM_MODEL)
    for k, n in enumerate(names):
        op = orc.payoff(**W.PAYOFFS[n])
        for l in (0, 2, 4):
            g = got[k][l]
            gmean = g["sum_y"] / g["n"]
            gvar = g["sum_y2"] / g["n"] - gmean**2
            o = orc.level(om, op, l, 4, 20000, 77, nthreads=8)
            omean = o["sum_y"] / 20000
            ovar = o["sum_y2"] / 20000 - omean**2
            assert abs(gmean - omean) < 5 * np.sqrt(gvar / g["n"] + ovar / 20000), (n, l)
        assert all(got[k][l]["n_nonfinite"] == 0 for l in range(L + 1))


def test_persistent_run_matches_per_level_run(gctx):
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    for eps in (0.1, 0.02):
        a = gctx.mlmc_run(gm, gp, eps, M=4, seed=4, persistent=False)
        b = gctx.mlmc_run(gm, gp, eps, M=4, seed=4, persistent=True)
        assert a["N"] == b["N"] and a["L"] == b["L"] and a["iterations"] == b["iterations"]
        assert close(a["estimate"], b["estimate"], 1e-10)


@pytest.mark.parametrize("kind,scheme,pname", [(0, 1, "asian"), (1, 0, "call"), (0, 0, "lookback")])
def test_graph_run_variants_match_per_level_run(gctx, kind, scheme, pname):
    md = dict(W.GBM_MODEL if kind == 0 else W.HESTON_MODEL, scheme=scheme)
    gm, gp = mlmc.model(**md), mlmc.payoff(**W.PAYOFFS[pname])
    for eps, M in ((0.1, 4), (0.05, 2)):
        a = gctx.mlmc_run(gm, gp, eps, M=M, seed=6, persistent=0)
        b = gctx.mlmc_run(gm, gp, eps, M=M, seed=6, persistent=1)
        assert a["N"] == b["N"] and a["L"] == b["L"] and a["iterations"] == b["iterations"]
        assert close(a["estimate"], b["estimate"], 1e-10)
    with pytest.raises(mlmc.MLMCError):
        gctx.mlmc_run(gm, gp, 0.1, persistent=2)


def test_graph_run_stopped_at_l_max_matches_per_level_run(gctx):
    """Graph launches are queued one iteration ahead of the host; the launch
    past the last update must leave the finished state as it is, also when
    the run ends at L_max without passing the bias test."""
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    kw = dict(M=4, L_min=2, L_max=2, n_pilot=2000, seed=8, allow_notconv=True)
    a = gctx.mlmc_run(gm, gp, 0.002, persistent=0, **kw)
    b = gctx.mlmc_run(gm, gp, 0.002, persistent=1, **kw)
    assert not a["converged"] and not b["converged"] and a["L"] == b["L"] == 2
    assert a["N"] == b["N"] and a["iterations"] == b["iterations"]
    # the two forms add the same samples in another order
    for k in ("sum_y", "sum_y2"):
        assert all(close(x, y, 1e-10) for x, y in zip(a[k], b[k])), k
    assert close(a["estimate"], b["estimate"], 1e-10) and close(a["rmse_est"], b["rmse_est"], 1e-8)


def test_graph_run_timing_counts_every_launch_and_step(gctx):
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    gctx.set_timing_slots([mlmc.STAT_PERSISTENT])
    r = gctx.mlmc_run(gm, gp, 0.01, M=4, seed=5, persistent=1)
    st = gctx.kernel_stats()[mlmc.STAT_PERSISTENT]
    gctx.set_timing(False)
    # one launch per update and the one queued past the last
    assert st["launches"] == r["iterations"] + 1 and st["ms"] > 0
    assert st["fine_steps"] == sum(n * 4**l for l, n in enumerate(r["N"]))
    assert st["coarse_steps"] == sum(n * 4**(l - 1) for l, n in enumerate(r["N"]) if l)
    # a second run starts from a fresh state
    r2 = gctx.mlmc_run(gm, gp, 0.01, M=4, seed=5, persistent=1)
    assert r2["N"] == r["N"] and close(r2["estimate"], r["estimate"], 1e-12)


def test_graph_runs_between_batches_and_shape_changes(gctx):
    """The device descriptor is uploaded only when it changes and a run may
    return with an empty launch still queued: runs interleaved with batches
    (another descriptor) and with a new persistent shape (a new graph) must
    reproduce the first run."""
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.ASIAN)
    ref = gctx.mlmc_run(gm, gp, 0.02, M=4, seed=9, persistent=1)
    again = gctx.mlmc_run(gm, gp, 0.02, M=4, seed=9, persistent=1)
    pays = [mlmc.payoff(**W.CALL), mlmc.payoff(**W.DIGITAL)]
    batch = gctx.mlmc_levels_batch(gm, pays, 4, 2, [[3000, 300, 30]] * 2, seed=9)
    after_batch = gctx.mlmc_run(gm, gp, 0.02, M=4, seed=9, persistent=1)
    gctx.set_persistent_launch(128, 2, 8)
    try:
        reshaped = gctx.mlmc_run(gm, gp, 0.02, M=4, seed=9, persistent=1)
    finally:
        gctx.set_persistent_launch(0, 0, 0)
    batch2 = gctx.mlmc_levels_batch(gm, pays, 4, 2, [[3000, 300, 30]] * 2, seed=9)
    for r in (again, after_batch, reshaped):
        assert r["N"] == ref["N"] and r["L"] == ref["L"]
        assert close(r["estimate"], ref["estimate"], 1e-10)
    for k in range(2):
        for l in range(3):
            assert batch[k][l]["n"] == batch2[k][l]["n"]
            assert close(batch[k][l]["sum_y"], batch2[k][l]["sum_y"], 1e-10)


def test_planned_run_after_planned_run_starts_like_a_fresh_start(gctx):
    """A device-planned run that follows one of the same problem starts with
    its sampler (the update queued past the last one built the fresh state
    and planned the pilot); it must give what a run through the start kernel
    gives: for another seed, after a per-level run (no prepared start), after
    a run of another problem (another descriptor), and prepared again."""
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    kw = dict(M=4, persistent=1)
    gctx.mlmc_run(gm, gp, 0.02, seed=1, **kw)
    prepared = gctx.mlmc_run(gm, gp, 0.02, seed=2, **kw)
    gctx.mlmc_run(gm, gp, 0.02, M=4, seed=1, persistent=0)
    started = gctx.mlmc_run(gm, gp, 0.02, seed=2, **kw)
    other = gctx.mlmc_run(gm, gp, 0.05, seed=3, **kw)
    after_other = gctx.mlmc_run(gm, gp, 0.02, seed=2, **kw)
    again = gctx.mlmc_run(gm, gp, 0.02, seed=2, **kw)
    assert other["L"] <= prepared["L"]
    for r in (started, after_other, again):
        assert r["N"] == prepared["N"] and r["L"] == prepared["L"]
        assert r["iterations"] == prepared["iterations"]
        assert close(r["estimate"], prepared["estimate"], 1e-10)
    # runs that finish at their first update (the pilot meets the target)
    # and runs stopped at L_max without convergence prepare the next start too
    for eps, extra in ((0.8, {}), (0.002, dict(L_max=2, allow_notconv=True))):
        first = gctx.mlmc_run(gm, gp, eps, seed=5, **kw, **extra)
        prepared = gctx.mlmc_run(gm, gp, eps, seed=6, **kw, **extra)
        gctx.mlmc_levels_batch(gm, [gp], 4, 1, [[1000, 100]], seed=1)
        started = gctx.mlmc_run(gm, gp, eps, seed=6, **kw, **extra)
        assert prepared["N"] == started["N"] and prepared["iterations"] == started["iterations"]
        assert close(prepared["estimate"], started["estimate"], 1e-10)
        if not extra:
            assert first["iterations"] == 1


def test_batch_bad_args(gctx):
    gm = mlmc.model(**W.GBM_MODEL)
    with pytest.raises(mlmc.MLMCError):
        gctx.mlmc_levels_batch(gm, [mlmc.payoff(**W.CALL)] * 5, 4, 2, [[10] * 3] * 5, 1)
    with pytest.raises(mlmc.MLMCError):
        gctx.mlmc_levels_batch(gm, [mlmc.payoff(**W.CALL)], 3, 2, [[10] * 3], 1)


@pytest.mark.parametrize("kind", [0, 1])
def test_batch_items_across_the_counter_high_word(gctx, kind):
    """Items whose generator units cross a multiple of 2^32 run in two parts;
    the sums must equal the per-level launches' (which split the same way)."""
    md = W.GBM_MODEL if kind == 0 else W.HESTON_MODEL
    gm = mlmc.model(**md)
    pays = [mlmc.payoff(**W.PAYOFFS[n]) for n in ("call", "asian", "lookback", "digital")]
    L, M = 3, 4
    q0 = 4 if kind == 0 else 2           # samples per generator unit at level 0
    N = [[5000 + 300 * k + 11 * l for l in range(L + 1)] for k in range(4)]
    offs = [[(q0 if l == 0 else 1) * (1 << 32) - 2000 - 7 * k for l in range(L + 1)]
            for k in range(4)]
    got = gctx.mlmc_levels_batch(gm, pays, M, L, N, seed=4, offsets=offs)
    for k, p in enumerate(pays):
        for l in range(L + 1):
            ref = gctx.mlmc_level(gm, p, l, M, N[k][l], 4, path_offset=offs[k][l])
            g = got[k][l]
            assert g["n"] == N[k][l]
            for key in ("sum_y", "sum_y2", "sum_pf", "sum_pc"):
                assert close(g[key], ref[key]), (k, l, key, g[key], ref[key])
