"""Pins for the oracle's tabulated control variate (CPU only).

The tabulated form reads phi from a table of the network on a (time, S[, v])
grid, interpolated linearly in S (bilinearly in S and v) in the row of the
last grid time at or before the evaluation time.  Pins: a table of a
function that is linear in S and v between grid points is reproduced
exactly (so the interpolation weights, the clamping at the grid's edges and
the row choice are right); the table of a network agrees with the network at
the grid points and, between them, to within the linear-interpolation bound;
the control-variate sum keeps mean zero (its terms are functions of the left
point, Sec. 5 "Exploiting Structure"); and a coupled level sample with the
table equals one written out from the oracle's normals.
"""
import numpy as np
import pytest

S0, T = 100.0, 1.0


def net(orc, in_dim, seed=3, scale=2.0):
    p = orc.cv_init(in_dim, 64, seed) * scale
    rng = np.random.default_rng(seed)
    p = p + 0.1 * rng.standard_normal(p.size) * (p == 0)
    return p


def grid_axes(g):
    S = g.s_lo + np.arange(g.ns) * (g.s_hi - g.s_lo) / (g.ns - 1)
    v = g.v_lo + np.arange(g.nv) * ((g.v_hi - g.v_lo) / (g.nv - 1) if g.nv > 1 else 0.0)
    return S, v


@pytest.mark.parametrize("kind", [0, 1])
def test_grid_of_the_model(orc, kind):
    m = orc.model(kind=kind)
    g = orc.cv_table_grid(m)
    sref = 0.2                                  # sigma, or sqrt(theta) = 0.2
    assert (g.rows, g.ns, g.nv) == ((256, 32, 1) if kind == 0 else (16, 16, 32))
    assert abs(g.s_lo - S0 * np.exp(-4 * sref)) < 1e-12 and abs(g.s_hi - S0 * np.exp(4 * sref)) < 1e-9
    if kind == 1:
        assert g.v_lo == 0.0 and abs(g.v_hi - 0.16) < 1e-15


@pytest.mark.parametrize("kind", [0, 1])
def test_linear_table_is_reproduced(orc, kind):
    m = orc.model(kind=kind)
    g = orc.cv_table_grid(m)
    S, v = grid_axes(g)
    j = np.arange(g.rows)[:, None, None]
    vals = 3.0 + 0.5 * j + 0.1 * S[None, None, :] + (2.0 * v[None, :, None] if g.nv > 1 else 0.0)
    cv = orc.CVNet(net(orc, 3 if kind else 2), 3 if kind else 2, 64, table=vals, grid=g)
    rng = np.random.default_rng(1)
    for _ in range(200):
        row = int(rng.integers(0, g.rows))
        # a time inside the row's interval, and its left end exactly
        t = (row + float(rng.uniform(0, 0.999))) * T / g.rows
        s = float(rng.uniform(g.s_lo - 20.0, g.s_hi + 50.0))
        vv = float(rng.uniform(-0.05, 0.3))
        sc = min(max(s, g.s_lo), g.s_hi)
        vc = min(max(vv, g.v_lo), g.v_hi) if g.nv > 1 else 0.0
        want = 3.0 + 0.5 * row + 0.1 * sc + 2.0 * vc
        for tt in (t, row * T / g.rows):
            got = orc.cv_phi(m, cv, tt, s, vv)
            assert abs(got - want) < 1e-9, (row, tt, s, vv, got, want)


@pytest.mark.parametrize("kind", [0, 1])
def test_network_table_matches_the_network(orc, kind):
    d = 3 if kind else 2
    m = orc.model(kind=kind)
    g = orc.cv_table_grid(m)
    exact = orc.CVNet(net(orc, d), d, 64)
    vals = orc.cv_table_fill(m, exact, g)
    tab = orc.CVNet(net(orc, d), d, 64, table=vals, grid=g)
    S, v = grid_axes(g)
    rng = np.random.default_rng(2)
    for _ in range(50):
        j, i, k = int(rng.integers(g.rows)), int(rng.integers(g.ns)), int(rng.integers(g.nv))
        t = j * T / g.rows
        assert abs(vals[j, k, i] - orc.cv_phi(m, exact, t, S[i], v[k])) < 1e-12
        assert abs(orc.cv_phi(m, tab, t, S[i], v[k]) - vals[j, k, i]) < 1e-9
    # between grid points near S0: linear interpolation error ~ dS^2 |phi''| / 8
    dS = S[1] - S[0]
    errs = []
    for s in np.linspace(80.0, 125.0, 37):
        t = 0.5
        a = orc.cv_phi(m, tab, t, s, 0.04)
        b = orc.cv_phi(m, exact, t, s, 0.04) if kind == 0 else None
        if b is not None:
            # second difference of the network at this S bounds the error
            h = dS
            curv = abs(orc.cv_phi(m, exact, t, s + h, 0.04) - 2 * b + orc.cv_phi(m, exact, t, s - h, 0.04))
            errs.append(abs(a - b))
            assert abs(a - b) <= curv / 8 * 2 + 1e-9, (s, a, b, curv)
    assert len(errs) == (37 if kind == 0 else 0)


@pytest.mark.parametrize("kind,pk", [(0, 1), (0, 0), (1, 0)])
def test_tabulated_control_variate_has_mean_zero(orc, kind, pk):
    d = 3 if kind else 2
    m, p = orc.model(kind=kind), orc.payoff(kind=pk)
    g = orc.cv_table_grid(m)
    exact = orc.CVNet(net(orc, d), d, 64)
    tab = orc.CVNet(net(orc, d), d, 64, table=orc.cv_table_fill(m, exact, g), grid=g)
    N, l, M = 20000, 2, 4
    pf0, pc0 = orc.level_paths(m, p, l, M, N, 5, 0, nthreads=8)
    pf1, pc1 = orc.level_paths(m, p, l, M, N, 5, 0, cv=tab, nthreads=8)
    for dlt in (pf0 - pf1, pc0 - pc1):           # the control-variate sums
        assert abs(dlt.mean()) < 4.5 * dlt.std() / np.sqrt(N)
    # and it removes variance (the network is random, so only a weak claim:
    # the sums are not zero)
    assert np.std(pf0 - pf1) > 0


def test_tabulated_level_sample_written_out(orc):
    """One coupled GBM sample at level 2 (M = 4) with the table, recomputed
    from the oracle's normals: fine step n reads row n rows / 16, coarse step
    c row 4 c rows / 16."""
    m, p = orc.model(), orc.payoff(kind=0)
    g = orc.cv_table_grid(m)
    exact = orc.CVNet(net(orc, 2), 2, 64)
    vals = orc.cv_table_fill(m, exact, g)
    tab = orc.CVNet(net(orc, 2), 2, 64, table=vals, grid=g)
    S_ax, _ = grid_axes(g)
    l, M, seed = 2, 4, 9

    def interp(row, S):
        u = min(max((S - g.s_lo) / (S_ax[1] - S_ax[0]), 0.0), g.ns - 1)
        i = min(int(u), g.ns - 2)
        f = u - i
        return (1 - f) * vals[row, 0, i] + f * vals[row, 0, i + 1]

    for s in (0, 1, 7):
        pf, pc, cf, cc = orc.level_sample(m, p, l, M, seed, s, cv=tab)
        z = orc.path_normals(seed, l, s, 0, 1, 16)
        h = T / 16
        dw = np.sqrt(h) * z
        S, cvf = S0, 0.0
        for n in range(16):
            cvf += interp(n * g.rows // 16, S) * dw[n]
            S = S + S * (0.05 * h + 0.2 * dw[n])
        Sc, cvc = S0, 0.0
        for c in range(4):
            dwc = dw[4 * c:4 * c + 4].sum()
            cvc += interp(4 * c * g.rows // 16, Sc) * dwc
            Sc = Sc + Sc * (0.05 * 4 * h + 0.2 * dwc)
        assert abs(cf - cvf) < 1e-10 and abs(cc - cvc) < 1e-10, (s, cf, cvf, cc, cvc)
