"""Pins for the oracle's Milstein scheme and antithetic estimator (CPU only).

The paper names both without formulas: Milstein as the more strongly
accurate scheme that gives beta > gamma = 1 and O(eps^-2) cost (Sec. 3 and
the remark after the complexity theorem of Sec. 5), antithetic variables
inside the multilevel estimator (Sec. 7).  Checked against things other than
the sampler:
  - brute force: tiny N and l, every path recomputed by separately written
    numpy loops (multiplicative form of the Milstein step, explicit twin);
  - exact moments of the Milstein K = 0 payoff: E[S_N] = S0 (1 + r h)^N and
    E[S_N^2] = S0^2 (a^2 + b^2 + 2 c^2)^N with a = 1 + r h, b^2 = sigma^2 h,
    c = sigma^2 h / 2 (from E z^2 = 1, E z^4 = 3);
  - strong order one (against the exact GBM solution on the same path),
    weak order one, variance decay beta ~ 2 for the call;
  - the antithetic twin: same law (level means agree with the plain
    estimator), GBM European payoffs unchanged (the terminal value is a
    product of per-step factors, which the permutation leaves alone), the
    coarse terminal value unchanged, and the twin of the twin is the path.
"""
import numpy as np
import pytest

S0, K, R, SIG, T = 100.0, 100.0, 0.05, 0.2, 1.0
HES = dict(kappa=2.0, theta=0.04, xi=0.3, rho=-0.7, v0=0.04)


def step_factor(dw, h, scheme):
    f = 1.0 + R * h + SIG * dw
    if scheme == 1:
        f += 0.5 * SIG * SIG * (dw * dw - h)
    return f


def brute_gbm(pk, dw, u, scheme):
    """GBM fine path, multiplicative form, all four payoffs."""
    n = len(dw)
    h = T / n
    S = S0
    Ss, mins = [S], []
    for i in range(n):
        S_new = S * step_factor(dw[i], h, scheme)
        if pk == 2:
            b = SIG * S
            mins.append(0.5 * (S + S_new - np.sqrt((S_new - S) ** 2 - 2 * b * b * h * np.log(u[i]))))
        S = S_new
        Ss.append(S)
    return payoff_of(pk, np.array(Ss), h, mins)


def payoff_of(pk, Ss, h, mins):
    disc = np.exp(-R * T)
    S = Ss[-1]
    if pk == 0:
        return disc * max(S - K, 0)
    if pk == 1:
        return disc * max(np.sum(0.5 * (Ss[:-1] + Ss[1:]) * h) / T - K, 0)
    if pk == 2:
        return disc * (S - min(mins))
    return disc * (1.0 if S > K else (0.5 if S == K else 0.0))


def brute_gbm_coarse(pk, dw, u, M, scheme):
    """Coarse path from summed increments; the lookback refines each coarse
    step at the fine times with the coarse step's own (frozen) formula."""
    nf = len(dw)
    h = T / nf
    H = M * h
    S = S0
    Ss, mn = [S], np.inf
    for c in range(nf // M):
        seg = dw[c * M:(c + 1) * M]
        if pk == 2:
            W = np.concatenate([[0.0], np.cumsum(seg)])
            tau = np.arange(M + 1) * h
            X = S * (1 + R * tau + SIG * W)
            if scheme == 1:
                X = X + 0.5 * SIG * SIG * S * (W * W - tau)
            for k in range(M):
                d = X[k + 1] - X[k]
                b = SIG * S
                mn = min(mn, 0.5 * (X[k] + X[k + 1] - np.sqrt(d * d - 2 * b * b * h * np.log(u[c * M + k]))))
        S = S * step_factor(seg.sum(), H, scheme)
        Ss.append(S)
    disc = np.exp(-R * T)
    if pk == 2:
        return disc * (S - mn)
    return payoff_of(pk, np.array(Ss), H, [])


def twin(x, M):
    """Reverse the order inside each block of M (the antithetic permutation)."""
    return x.reshape(-1, M)[:, ::-1].ravel()


@pytest.mark.parametrize("pk", [0, 1, 2, 3])
@pytest.mark.parametrize("anti", [0, 1])
def test_brute_force_tiny_milstein_and_antithetic(orc, pk, anti):
    m = orc.model(scheme=1, antithetic=anti)
    p = orc.payoff(kind=pk, K=K, payout=1.0)
    for M in (2, 4):
        for l in (0, 1, 2):
            nf = M**l
            h = T / nf
            pf_all, pc_all = orc.level_paths(m, p, l, M, 8, seed=2, offset=5)
            for i in range(8):
                s = 5 + i
                dw = np.sqrt(h) * orc.path_normals(2, l, s, 0, 1, nf)
                u = orc.path_uniforms(2, l, s, 1, nf)
                pf = brute_gbm(pk, dw, u, 1)
                pc = brute_gbm_coarse(pk, dw, u, M, 1) if l else 0.0
                if anti and l:
                    pf = 0.5 * (pf + brute_gbm(pk, twin(dw, M), twin(u, M), 1))
                    pc = 0.5 * (pc + brute_gbm_coarse(pk, twin(dw, M), twin(u, M), M, 1))
                assert abs(pf - pf_all[i]) <= 1e-11 * max(1.0, abs(pf)), (M, l, i)
                assert abs(pc - pc_all[i]) <= 1e-11 * max(1.0, abs(pc)), (M, l, i)


def test_antithetic_heston_brute_force(orc):
    # Heston, Euler: the twin permutes both factors and the bridge uniforms
    m = orc.model(kind=1, antithetic=1)
    m0 = orc.model(kind=1)
    for pk in (0, 1):
        p = orc.payoff(kind=pk)
        for M, l in ((2, 1), (4, 2)):
            nf = M**l
            h = T / nf
            pf_all, pc_all = orc.level_paths(m, p, l, M, 6, seed=4)
            for s in range(6):
                z = orc.path_normals(4, l, s, 0, 2, nf).reshape(nf, 2)
                dw = np.sqrt(h) * z
                a = np.stack([twin(dw[:, 0], M), twin(dw[:, 1], M)], axis=1)
                pf = 0.5 * (orc.path_payoff(m0, p, dw.ravel()) + orc.path_payoff(m0, p, a.ravel()))
                assert abs(pf - pf_all[s]) <= 1e-11 * max(1.0, abs(pf)), (pk, M, s)


@pytest.mark.parametrize("M", [2, 4])
def test_milstein_k0_moments_exact(orc, M):
    m = orc.model(scheme=1)
    p = orc.payoff(kind=0, K=0.0)
    N = 60000
    disc = np.exp(-R * T)

    def moments(nsteps):
        h = T / nsteps
        a, b2, c = 1 + R * h, SIG * SIG * h, 0.5 * SIG * SIG * h
        return disc * S0 * a**nsteps, (disc * S0) ** 2 * (a * a + b2 + 2 * c * c) ** nsteps

    for l in range(0, 5 if M == 2 else 4):
        r = orc.level(m, p, l, M, N, seed=6, nthreads=8)
        e1, e2 = moments(M**l)
        mf = r["sum_pf"] / N
        vf = e2 - e1 * e1
        assert abs(mf - e1) < 4.5 * np.sqrt(vf / N), l
        assert abs(r["sum_pf2"] / N / e2 - 1) < 4.5 * np.sqrt(8 * vf / e2 ** 2 / N) + 2e-3, l
        if l:
            c1, c2 = moments(M ** (l - 1))
            mc = r["sum_pc"] / N
            assert abs(mc - c1) < 4.5 * np.sqrt((c2 - c1 * c1) / N), l
            vy = r["sum_y2"] / N - (r["sum_y"] / N) ** 2
            assert abs(r["sum_y"] / N - (e1 - c1)) < 4.5 * np.sqrt(vy / N), l


def _strong_errors(orc, scheme, levels, n=400):
    errs = []
    for l in levels:
        nf = 2**l
        h = T / nf
        e = []
        for s in range(n):
            dw = np.sqrt(h) * orc.path_normals(8, l, s, 0, 1, nf)
            exact = S0 * np.exp((R - 0.5 * SIG**2) * T + SIG * dw.sum())
            sn = orc.path_payoff(orc.model(scheme=scheme), orc.payoff(kind=0, K=0.0), dw)
            e.append(abs(sn * np.exp(R * T) - exact))
        errs.append(np.mean(e))
    return errs


def test_milstein_strong_order_one(orc):
    lv = np.arange(2, 8)
    mil = _strong_errors(orc, 1, lv)
    em = _strong_errors(orc, 0, lv)
    s_mil = np.polyfit(lv, np.log2(mil), 1)[0]
    s_em = np.polyfit(lv, np.log2(em), 1)[0]
    print("strong slopes: Milstein", s_mil, "Euler", s_em)
    assert -1.2 < s_mil < -0.8, (s_mil, mil)
    assert -0.7 < s_em < -0.3
    assert mil[-1] < 0.2 * em[-1]


def test_milstein_weak_order_one_and_beta_two(orc):
    m, p = orc.model(scheme=1), orc.payoff()
    bs = orc.bs_call()
    N = 200000
    acc, errs, V = 0.0, [], []
    for l in range(0, 7):
        r = orc.level(m, p, l, 2, N, seed=7, nthreads=8)
        mean = r["sum_y"] / N
        V.append(r["sum_y2"] / N - mean**2)
        acc += mean
        if l:
            errs.append(abs(acc - bs))
    beta = -np.polyfit(np.arange(2, 7), np.log2(V[2:]), 1)[0]
    print("beta", beta, "errors", errs)
    assert 1.7 < beta < 2.3, V
    # the telescoped estimate converges to Black--Scholes at O(h)
    assert errs[-1] < 0.02 and errs[-1] < errs[0]


@pytest.mark.parametrize("scheme", [0, 1])
def test_antithetic_keeps_level_means(orc, scheme):
    N = 60000
    for kind, pk, M in ((0, 1, 2), (0, 2, 4), (1, 0, 4), (1, 1, 2)):
        if kind == 1 and scheme == 1:
            continue
        p = orc.payoff(kind=pk)
        for l in (1, 2, 3):
            a = orc.level(orc.model(kind=kind, scheme=scheme, antithetic=1), p, l, M, N, seed=8,
                          nthreads=8)
            b = orc.level(orc.model(kind=kind, scheme=scheme), p, l, M, N, seed=9, nthreads=8)
            ma, mb = a["sum_y"] / N, b["sum_y"] / N
            va = a["sum_y2"] / N - ma**2
            vb = b["sum_y2"] / N - mb**2
            assert abs(ma - mb) < 4.5 * np.sqrt(va / N + vb / N), (kind, pk, l)
            # the coarse law is untouched: same mean of P_c
            pca, pcb = a["sum_pc"] / N, b["sum_pc"] / N
            vpa = a["sum_pc2"] / N - pca**2
            vpb = b["sum_pc2"] / N - pcb**2
            assert abs(pca - pcb) < 4.5 * np.sqrt(vpa / N + vpb / N), (kind, pk, l)


@pytest.mark.parametrize("scheme", [0, 1])
def test_antithetic_leaves_gbm_european_payoffs(orc, scheme):
    for pk in (0, 3):
        p = orc.payoff(kind=pk)
        for M, l in ((2, 3), (4, 2)):
            a = orc.level_paths(orc.model(scheme=scheme, antithetic=1), p, l, M, 500, seed=3)
            b = orc.level_paths(orc.model(scheme=scheme), p, l, M, 500, seed=3)
            assert np.allclose(a[0], b[0], rtol=1e-12, atol=1e-12)
            assert np.allclose(a[1], b[1], rtol=1e-12, atol=1e-12)


def test_antithetic_reduces_path_dependent_variance(orc):
    """What the twin gains where the payoff depends on the path."""
    N = 40000
    for kind, pk, M, scheme, gain in ((0, 1, 2, 0, 5.0), (0, 1, 2, 1, 5.0), (0, 2, 2, 1, 1.2),
                                      (1, 0, 4, 0, 1.2)):
        a = orc.level(orc.model(kind=kind, scheme=scheme, antithetic=1), orc.payoff(kind=pk), 3, M,
                      N, seed=10, nthreads=8)
        b = orc.level(orc.model(kind=kind, scheme=scheme), orc.payoff(kind=pk), 3, M, N, seed=10,
                      nthreads=8)
        va = a["sum_y2"] / N - (a["sum_y"] / N) ** 2
        vb = b["sum_y2"] / N - (b["sum_y"] / N) ** 2
        print(kind, pk, scheme, "variance ratio", vb / va)
        assert vb / va > gain, (kind, pk, scheme, vb / va)


def test_costs_and_bad_arguments(orc):
    assert orc.level_cost(0, 4, 1) == 1.0
    assert orc.level_cost(3, 2, 0) == 12.0
    assert orc.level_cost(3, 2, 1) == 20.0
    p = orc.payoff()
    with pytest.raises(ValueError):      # Milstein is implemented for GBM only
        orc.level(orc.model(kind=1, scheme=1), p, 1, 2, 10, 1)
    with pytest.raises(ValueError):
        orc.level(orc.model(scheme=2), p, 1, 2, 10, 1)
    with pytest.raises(ValueError):      # the twin belongs to level differences
        orc.stdmc(orc.model(antithetic=1), p, 2, 2, 10, 1)
    r = orc.level(orc.model(antithetic=1), p, 2, 2, 10, 1)
    assert r["cost"] == 10 * (2 * 4 + 2)
