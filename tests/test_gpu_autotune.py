"""Autotuner: picks measured shapes, caches them, and never changes results."""
import json
import os

import pytest

from paper_1505_00965_amd import mlmc, workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_cache_and_invariance(tmp_path):
    path = str(tmp_path / "tune.json")
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    with mlmc.Context(0) as ctx:
        ref = [ctx.mlmc_level(gm, gp, l, 4, 50000, 3) for l in (0, 2, 5)]
        ctx.autotune(gm, gp, M=4, precision=32, cache_path=path)
        shapes = [ctx.tuned_shape(gm, gp, l) for l in (0, 2, 5)]
        for b, p in shapes:
            assert b in (64, 128, 256, 512, 1024) and p in (1, 2, 4)
        assert shapes[0][1] in (1, 2)            # one-step levels take at most 2 blocks per lane
        got = [ctx.mlmc_level(gm, gp, l, 4, 50000, 3) for l in (0, 2, 5)]
        for a, b in zip(ref, got):
            assert abs(a["sum_y"] - b["sum_y"]) <= 1e-12 * abs(a["sum_y"])
    data = json.load(open(path))
    (machine, entries), = data.items()
    assert "gfx950" in machine and len(entries) == 7       # levels 0..5, then 6 and deeper
    # a new context reads the cache instead of measuring
    with mlmc.Context(0) as ctx:
        assert ctx.tuned_shape(gm, gp, 2) == (0, 0)
        ctx.autotune(gm, gp, M=4, precision=32, cache_path=path)
        assert [ctx.tuned_shape(gm, gp, l) for l in (0, 2, 5)] == shapes
    assert os.path.getsize(path) > 0


def test_autotune_persistent_cache_and_invariance(tmp_path):
    """The persistent form's tuner picks a shape from its candidate set, sets
    it, caches it, and the batch sums do not depend on it."""
    import time
    path = str(tmp_path / "tune_persist.json")
    gm = mlmc.model(**W.GBM_MODEL)
    pays = [mlmc.payoff(**W.CALL), mlmc.payoff(**W.LOOKBACK)]
    L, M = 5, 4
    N = [[200000 // 4**l + 1 for l in range(L + 1)] for _ in pays]
    with mlmc.Context(0) as ctx:
        ref = ctx.mlmc_levels_batch(gm, pays, M, L, N, seed=21)
        shape = ctx.autotune_persistent(gm, pays, M=M, L=L, cache_path=path)
        b, p, c = shape
        assert b in (128, 256, 512) and p in (1, 2, 4) and c in (2, 4, 8) and b * c <= 2048
        got = ctx.mlmc_levels_batch(gm, pays, M, L, N, seed=21)
        for k in range(len(pays)):
            for l in range(L + 1):
                a, g = ref[k][l], got[k][l]
                assert a["n"] == g["n"]
                scale = (a["n"] * a["sum_y2"]) ** 0.5
                assert abs(a["sum_y"] - g["sum_y"]) <= 1e-12 * scale + 1e-300, (k, l)
    data = json.load(open(path))
    (machine, entries), = data.items()
    assert "gfx950" in machine and list(entries.values()) == [list(shape)]
    # a new context reads the cache instead of measuring
    with mlmc.Context(0) as ctx:
        t0 = time.perf_counter()
        again = ctx.autotune_persistent(gm, pays, M=M, L=L, cache_path=path)
        assert again == shape and time.perf_counter() - t0 < 0.5
    with mlmc.Context(0) as ctx:
        with pytest.raises(mlmc.MLMCError):
            ctx.autotune_persistent(gm, pays * 3, M=M, L=L)     # six payoffs


def test_autotune_keys_separate_scheme_twin_and_payoff_mix(tmp_path):
    """A shape tuned for Euler paths is not served to Milstein or antithetic
    runs, and a persistent shape tuned for one payoff mix is not served to
    another mix with the same first payoff."""
    path = str(tmp_path / "tune_keys.json")
    gp = mlmc.payoff(**W.CALL)
    euler = mlmc.model(**W.GBM_MODEL)
    milstein = mlmc.model(**dict(W.GBM_MODEL, scheme=1))
    twin = mlmc.model(**dict(W.GBM_MODEL, antithetic=1))
    with mlmc.Context(0) as ctx:
        ctx.autotune(euler, gp, M=4, precision=32, cache_path=path)
        assert ctx.tuned_shape(euler, gp, 3) != (0, 0)
        assert ctx.tuned_shape(milstein, gp, 3) == (0, 0)
        assert ctx.tuned_shape(twin, gp, 3) == (0, 0)
        # a tuned shape still drops to one sample per lane for small counts:
        # the sums equal the default shape's up to fp64 summation order
        small = ctx.mlmc_level(euler, gp, 3, 4, 3000, 5)
        ctx.set_launch(256, 1)
        ref = ctx.mlmc_level(euler, gp, 3, 4, 3000, 5)
        ctx.set_launch(0, 0)
        assert abs(small["sum_y"] - ref["sum_y"]) <= 1e-12 * abs(ref["sum_y"]) + 1e-12
    pays_a = [mlmc.payoff(**W.CALL), mlmc.payoff(**W.ASIAN)]
    pays_b = [mlmc.payoff(**W.CALL), mlmc.payoff(**W.LOOKBACK)]
    with mlmc.Context(0) as ctx:
        ctx.autotune_persistent(euler, pays_a, M=4, L=3, cache_path=path)
        ctx.autotune_persistent(euler, pays_b, M=4, L=3, cache_path=path)
    entries = next(iter(json.load(open(path)).values()))
    persist = [k for k in entries if k.startswith("persist:")]
    assert len(persist) == 2 and len(set(persist)) == 2


def test_autotune_run_tunes_the_device_planned_form(tmp_path):
    """The run tuner times whole device-planned runs of the caller's
    configuration, sets and caches a shape from the persistent candidate set,
    and the run's decisions and estimate do not depend on it."""
    import time
    path = str(tmp_path / "tune_run.json")
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.ASIAN)
    kw = dict(M=4, L_min=2, L_max=6, n_pilot=2000, seed=3)
    with mlmc.Context(0) as ctx:
        ref = ctx.mlmc_run(gm, gp, 0.02, persistent=1, **kw)
        shape = ctx.autotune_run(gm, gp, 0.02, cache_path=path, **kw)
        b, p, c = shape
        assert b in (128, 256, 512) and p in (1, 2, 4) and c in (2, 4, 8) and b * c <= 2048
        got = ctx.mlmc_run(gm, gp, 0.02, persistent=1, **kw)
        assert got["N"] == ref["N"] and got["L"] == ref["L"]
        assert abs(got["estimate"] - ref["estimate"]) <= 1e-10 * abs(ref["estimate"])
        with pytest.raises(mlmc.MLMCError) as e:      # only the device-planned form is tuned
            ctx._check(ctx._lib.mlmc_autotune_run(
                ctx.h, mlmc.C.byref(gm), mlmc.C.byref(gp),
                mlmc.C.byref(mlmc.RunOpts(0.02, 4, 2, 6, 2000, 3, 32, 0, 0.0, 0.0, None, 0)),
                None, None))
        assert e.value.status == mlmc.MLMC_EINVAL
        ctx.set_persistent_launch(0, 0, 0)
    entries = next(iter(json.load(open(path)).values()))
    assert [k for k in entries if k.startswith("run:")] and list(entries.values()) == [list(shape)]
    with mlmc.Context(0) as ctx:
        t0 = time.perf_counter()
        assert ctx.autotune_run(gm, gp, 0.02, cache_path=path, **kw) == shape
        assert time.perf_counter() - t0 < 0.5
