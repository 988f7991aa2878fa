"""GBM paths split across lanes vs the FP64 oracle.

Levels whose paths cannot fill the device run each path on several lanes,
each lane a segment of steps from a unit start, the segment summaries
combined in path order.  Same bar as the one-path-per-lane sampler: per path
|dP| <= 1e-4 S0 (digital samples within the path error of the strike may
flip), level sums equal to the fp64 re-sum of the GPU's own paths.
"""
import numpy as np
import pytest

from paper_1505_00965_amd import mlmc, workloads as W

pytestmark = pytest.mark.gpu
S0 = 100.0


def split_lanes(nf, N, num_cu):
    """The library's rule (lanes per path), restated for the test's cases."""
    if N == 0 or nf < 16:
        return 1
    want = num_cu * 1024 // N
    G = 64
    while G > 1 and (G > want or (nf // 4) % G != 0):
        G //= 2
    return G if G >= 4 else 1


def num_cu():
    import torch
    return torch.cuda.get_device_properties(0).multi_processor_count


CASES = [(4, 4), (4, 5), (2, 6), (2, 8), (4, 2)]


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("pname", ["call", "asian", "lookback", "digital"])
def test_split_paths_match_the_oracle(gctx, orc, scheme, pname):
    import torch
    md = dict(W.GBM_MODEL, scheme=scheme)
    gm, om = mlmc.model(**md), orc.model(**md)
    gp, op = mlmc.payoff(**W.PAYOFFS[pname]), orc.payoff(**W.PAYOFFS[pname])
    used = set()
    for M, l in CASES:
        for N, offset in ((37, 0), (700, 5), (3000, (1 << 32) - 1001)):
            G = split_lanes(M**l, N, num_cu())
            used.add(G)
            print(f"case scheme={scheme} payoff={pname} M={M} l={l} N={N} off={offset} G={G}",
                  flush=True)
            pf = torch.empty(N, dtype=torch.float64, device="cuda")
            pc = torch.empty(N, dtype=torch.float64, device="cuda")
            res = gctx.mlmc_level_paths(gm, gp, l, M, N, 11, pf, pc, path_offset=offset)
            pf, pc = pf.cpu().numpy(), pc.cpu().numpy()
            rf, rc = orc.level_paths(om, op, l, M, N, 11, offset, nthreads=8)
            bad = (np.abs(pf - rf) > 1e-4 * S0) | (np.abs(pc - rc) > 1e-4 * S0)
            if pname == "digital" and bad.any():
                k0 = orc.payoff(kind=0, K=0.0)
                sf, sc = orc.level_paths(om, k0, l, M, N, 11, offset, nthreads=8)
                disc = np.exp(-om.r * om.T)
                near = (np.abs(sf / disc - 100.0) < 2e-2) | (np.abs(sc / disc - 100.0) < 2e-2)
                assert np.all(near[bad]), (M, l, N, np.where(bad & ~near))
                assert bad.sum() <= max(2, 1e-2 * N)
            else:
                assert not bad.any(), (M, l, N, np.abs(pf - rf).max(), np.abs(pc - rc).max())
            y = pf - pc
            for key, ref in (("sum_y", y.sum()), ("sum_y2", (y * y).sum()),
                             ("sum_pf", pf.sum()), ("sum_pc", pc.sum())):
                assert abs(res[key] - ref) <= 1e-12 * max(1.0, np.abs(y).sum(), abs(ref)), key
            assert res["n"] == N and res["n_nonfinite"] == 0
    assert {4, 16, 64} <= used        # the cases reach every lane count


def test_split_level_means_match_one_path_per_lane(gctx, orc):
    """A deep level estimated with few paths (split) and many (unsplit):
    both level means agree with each other and with the oracle's to their
    standard errors."""
    gm, om = mlmc.model(**W.GBM_MODEL), orc.model(**W.GBM_MODEL)
    gp = mlmc.payoff(**W.ASIAN)
    l, M = 5, 4
    parts = [gctx.mlmc_level(gm, gp, l, M, 2000, 3, path_offset=2000 * i) for i in range(60)]
    n = sum(r["n"] for r in parts)
    m_split = sum(r["sum_y"] for r in parts) / n
    v_split = sum(r["sum_y2"] for r in parts) / n - m_split**2
    big = gctx.mlmc_level(gm, gp, l, M, 1 << 20, 4)
    m_big = big["sum_y"] / big["n"]
    v_big = big["sum_y2"] / big["n"] - m_big**2
    se = np.sqrt(v_split / n + v_big / big["n"])
    print("split", m_split, v_split, "unsplit", m_big, v_big, "se", se)
    assert split_lanes(M**l, 2000, num_cu()) > 1 and split_lanes(M**l, 1 << 20, num_cu()) == 1
    assert abs(m_split - m_big) < 4.5 * se
    assert 0.8 < v_split / v_big < 1.25
