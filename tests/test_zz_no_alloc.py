"""mlmc_level_noalloc (no context, no device allocation) against mlmc_level.

Both entry points draw the same samples (the same counters) and add them
into a group of 64 fp64 records that is folded in record order, so their
sums agree up to the order of the fp64 atomic additions into the records
(a few ulps of sum |Y| <= sqrt(N sum Y^2)); counts and costs are exact.
Two calls in a row, the second with a smaller input, check that the static
scratch group is cleared between calls.
"""
import pytest

from paper_1505_00965_amd import mlmc, workloads as W

pytestmark = pytest.mark.gpu


def same_sums(a, b, what):
    assert a["n"] == b["n"] and a["n_nonfinite"] == b["n_nonfinite"], what
    assert a["cost"] == b["cost"], what
    scale = (a["n"] * max(a["sum_y2"], b["sum_y2"])) ** 0.5
    assert abs(a["sum_y"] - b["sum_y"]) <= 1e-12 * scale + 1e-300, (what, a["sum_y"], b["sum_y"])
    for k in ("sum_y2", "sum_pf", "sum_pf2", "sum_pc", "sum_pc2"):
        tol = 1e-12 * max(abs(a[k]), abs(b[k]), 1e-300)
        if k in ("sum_pf", "sum_pc"):
            tol = 1e-12 * (a["n"] * max(a[k + "2"], b[k + "2"])) ** 0.5 + 1e-300
        assert abs(a[k] - b[k]) <= tol, (what, k, a[k], b[k])


@pytest.mark.parametrize("kind,pname,l,M,precision", [
    (0, "call", 0, 4, 32), (0, "asian", 3, 4, 32), (0, "lookback", 6, 4, 32),
    (1, "call", 2, 4, 32), (0, "call", 4, 2, 64)])
def test_noalloc_matches_mlmc_level_twice(gctx, kind, pname, l, M, precision):
    import torch
    md = W.GBM_MODEL if kind == 0 else W.HESTON_MODEL
    gm, gp = mlmc.model(**md), mlmc.payoff(**W.PAYOFFS[pname])
    stream = torch.cuda.current_stream()
    out = torch.zeros(9, dtype=torch.float64, device="cuda")
    # the second call is smaller: a stale group from the first would show
    for N, off in ((300000 >> (2 * min(l, 3)), 5), (7001 >> min(l, 3), (1 << 32) - 1000)):
        print(f"case kind={kind} payoff={pname} l={l} M={M} fp{precision} N={N} off={off}",
              flush=True)
        mlmc.mlmc_level_noalloc(gm, gp, l, M, N, 3, out, path_offset=off, precision=precision,
                                stream=stream)
        stream.synchronize()
        got = mlmc.level_result_from(out)
        ref = gctx.mlmc_level(gm, gp, l, M, N, 3, path_offset=off, precision=precision)
        same_sums(got, ref, (kind, pname, l, N, off))


def test_noalloc_bad_arguments():
    import torch
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    out = torch.zeros(9, dtype=torch.float64, device="cuda")
    with pytest.raises(mlmc.MLMCError) as e:
        mlmc.mlmc_level_noalloc(gm, gp, 2, 3, 100, 1, out)           # M = 3
    assert e.value.status == mlmc.MLMC_EINVAL and "M must be" in str(e.value)
    with pytest.raises(mlmc.MLMCError) as e:
        mlmc.mlmc_level_noalloc(gm, gp, 2, 4, (1 << 40) + 1, 1, out)  # beyond the maximum
    assert e.value.status == mlmc.MLMC_EINVAL and "2^40" in str(e.value)
    with pytest.raises(mlmc.MLMCError) as e:
        mlmc.mlmc_level_noalloc(gm, gp, 2, 4, 100, 1, None)
    assert e.value.status == mlmc.MLMC_EINVAL
