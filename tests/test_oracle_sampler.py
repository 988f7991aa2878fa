"""Pins for the oracle's coupled level sampler (CPU only).

Checks, against things other than the sampler itself:
  - brute force: tiny N and l, every path recomputed by a separately written
    numpy loop from the oracle's (separately pinned) normals;
  - the coupling of Sec. 5 (eq. (eq:Yldef), Fig. 2): the coarse path of level
    l is exactly the level-(l-1) path driven by summed fine increments;
  - exact Euler moments (K = 0 payoff, one-step call) level by level;
  - the telescoping identity (eq. (eq:mlmc:ident));
  - weak order one (eq. (eq:emweak)), strong order one half (eq. (eq:strong)),
    the O(dt_l) variance decay (eqs. (eq:mlmc:varPlbd), (eq:mlmc:varPlm1)),
    and the slower decay for the digital payoff (Sec. 7.1);
  - the digital tie rule of Sec. 6.
"""
import numpy as np
import pytest

S0, K, R, SIG, T = 100.0, 100.0, 0.05, 0.2, 1.0
HES = dict(kappa=2.0, theta=0.04, xi=0.3, rho=-0.7, v0=0.04)


def brute_path(kind, model, payoff_kind, K_, payout, dw1, dwp, u, r=R, sigma=SIG):
    """One path by a separately written loop (multiplicative / explicit form)."""
    n = len(dw1)
    h = T / n
    S, v = S0, HES["v0"]
    Ss = [S]
    mins = []
    for i in range(n):
        if kind == 0:
            vol = sigma
            S_new = S * (1.0 + r * h + sigma * dw1[i])
        else:
            vp = max(v, 0.0)
            vol = np.sqrt(vp)
            dw2 = HES["rho"] * dw1[i] + np.sqrt(1 - HES["rho"] ** 2) * dwp[i]
            S_new = S * (1.0 + r * h + vol * dw1[i])
            v = v + HES["kappa"] * (HES["theta"] - vp) * h + HES["xi"] * vol * dw2
        if payoff_kind == 2:
            b = vol * S
            mins.append(0.5 * (S + S_new - np.sqrt((S_new - S) ** 2 - 2 * b * b * h * np.log(u[i]))))
        S = S_new
        Ss.append(S)
    disc = np.exp(-r * T)
    Ss = np.array(Ss)
    if payoff_kind == 0:
        return disc * max(S - K_, 0)
    if payoff_kind == 1:
        A = np.sum(0.5 * (Ss[:-1] + Ss[1:]) * h) / T
        return disc * max(A - K_, 0)
    if payoff_kind == 2:
        return disc * (S - min(mins))
    return disc * payout * (1.0 if S > K_ else (0.5 if S == K_ else 0.0))


def brute_coarse_lookback(model_kind, dw1, dwp, u, M, r=R, sigma=SIG):
    """Coarse lookback written out: sub-bridges on the frozen-coefficient path."""
    nf = len(dw1)
    h = T / nf
    H = M * h
    S, v = S0, HES["v0"]
    mn = np.inf
    for c in range(nf // M):
        seg = dw1[c * M:(c + 1) * M]
        vol = SIG if model_kind == 0 else np.sqrt(max(v, 0.0))
        W = np.concatenate([[0.0], np.cumsum(seg)])
        tau = np.arange(M + 1) * h
        X = S * (1 + r * tau + vol * W)
        for k in range(M):
            d = X[k + 1] - X[k]
            b = vol * S
            mn = min(mn, 0.5 * (X[k] + X[k + 1] - np.sqrt(d * d - 2 * b * b * h * np.log(u[c * M + k]))))
        if model_kind == 0:
            S = S * (1 + r * H + SIG * seg.sum())
        else:
            vp = max(v, 0.0)
            dwc2 = HES["rho"] * seg.sum() + np.sqrt(1 - HES["rho"] ** 2) * dwp[c * M:(c + 1) * M].sum()
            S_new = S * (1 + r * H + np.sqrt(vp) * seg.sum())
            v = v + HES["kappa"] * (HES["theta"] - vp) * H + HES["xi"] * np.sqrt(vp) * dwc2
            S = S_new
    return np.exp(-r * T) * (S - mn)


@pytest.mark.parametrize("model_kind", [0, 1])
@pytest.mark.parametrize("pk", [0, 1, 2, 3])
def test_brute_force_tiny(orc, model_kind, pk):
    m = orc.model(kind=model_kind)
    p = orc.payoff(kind=pk, K=K, payout=1.0)
    dim = 2 if model_kind else 1
    for M in (2, 4):
        for l in (0, 1, 2):
            nf = M**l
            h = T / nf
            pf_all, pc_all = orc.level_paths(m, p, l, M, 8, seed=1, offset=3)
            for i in range(8):
                s = 3 + i
                z = orc.path_normals(1, l, s, 0, dim, nf).reshape(nf, dim)
                dw1 = np.sqrt(h) * z[:, 0]
                dwp = np.sqrt(h) * z[:, 1] if dim == 2 else np.zeros(nf)
                u = orc.path_uniforms(1, l, s, 1, nf)
                pf = brute_path(model_kind, m, pk, K, 1.0, dw1, dwp, u)
                assert abs(pf - pf_all[i]) <= 1e-11 * max(1.0, abs(pf)), (M, l, i)
                if l == 0:
                    assert pc_all[i] == 0.0
                    continue
                if pk == 2:
                    pc = brute_coarse_lookback(model_kind, dw1, dwp, u, M)
                else:
                    dw1c = dw1.reshape(-1, M).sum(axis=1)
                    dwpc = dwp.reshape(-1, M).sum(axis=1)
                    pc = brute_path(model_kind, m, pk, K, 1.0, dw1c, dwpc, None)
                assert abs(pc - pc_all[i]) <= 1e-11 * max(1.0, abs(pc)), (M, l, i)


@pytest.mark.parametrize("model_kind", [0, 1])
@pytest.mark.parametrize("pk", [0, 1, 3])
def test_coarse_is_previous_level_path_bit_exact(orc, model_kind, pk):
    # coarse payoff at level l == path payoff with the summed increments
    m = orc.model(kind=model_kind)
    p = orc.payoff(kind=pk)
    dim = 2 if model_kind else 1
    for M, l in [(2, 1), (2, 3), (4, 2), (4, 3)]:
        nf = M**l
        h = T / nf
        for s in range(5):
            pf, pc, _, _ = orc.level_sample(m, p, l, M, 1, s)
            z = orc.path_normals(1, l, s, 0, dim, nf).reshape(nf, dim)
            dw = np.sqrt(h) * z
            dwc = np.zeros((nf // M, dim))
            for c in range(nf // M):           # same summation order as the sampler
                acc = np.zeros(dim)
                for k in range(M):
                    acc = acc + dw[c * M + k]
                dwc[c] = acc
            assert orc.path_payoff(m, p, dwc.ravel()) == pc
            assert orc.path_payoff(m, p, dw.ravel()) == pf


@pytest.mark.parametrize("M", [2, 4])
def test_k0_level_moments_exact(orc, M):
    m = orc.model()
    p = orc.payoff(kind=0, K=0.0)
    N = 40000
    for l in range(0, 5 if M == 2 else 4):
        r = orc.level(m, p, l, M, N, seed=1, nthreads=8)
        e_exact, v_exact = orc.euler_k0_moments(S0, R, SIG, T, l, M)
        mean = r["sum_y"] / N
        var = r["sum_y2"] / N - mean**2
        if l == 0:
            assert abs(mean - e_exact) < 4.5 * np.sqrt(v_exact / N)
        else:
            e_prev, _ = orc.euler_k0_moments(S0, R, SIG, T, l - 1, M)
            assert abs(mean - (e_exact - e_prev)) < 4.5 * np.sqrt(v_exact / N)
            # the mean of the coarse path alone is the previous level's mean
            pc_mean = r["sum_pc"] / N
            pc_var = r["sum_pc2"] / N - pc_mean**2
            assert abs(pc_mean - e_prev) < 4.5 * np.sqrt(pc_var / N)
        # variance within a chi-square-style margin (kurtosis allowance)
        assert abs(var / v_exact - 1) < 0.08


def test_heston_k0_level_means_exact(orc):
    # the truncated diffusion has zero conditional mean, so E[S_N] = S0 (1+rh)^nf
    m = orc.model(kind=1)
    p = orc.payoff(kind=0, K=0.0)
    N = 40000
    for l in range(0, 4):
        r = orc.level(m, p, l, 4, N, seed=2, nthreads=8)
        nf = 4**l
        e = np.exp(-R * T) * S0 * (1 + R * T / nf) ** nf
        e_prev = np.exp(-R * T) * S0 * (1 + R * T / (nf // 4)) ** (nf // 4) if l else 0.0
        var = r["sum_y2"] / N - (r["sum_y"] / N) ** 2
        assert abs(r["sum_y"] / N - (e - e_prev)) < 4.5 * np.sqrt(var / N)


def test_level0_call_exact(orc):
    m, p = orc.model(), orc.payoff()
    N = 200000
    r = orc.level(m, p, 0, 2, N, seed=5, nthreads=8)
    e, v = orc.level0_call_moments(S0, K, R, SIG, T)
    mean = r["sum_y"] / N
    assert abs(mean - e) < 4.5 * np.sqrt(v / N)
    assert abs((r["sum_y2"] / N - mean**2) / v - 1) < 0.03


def _levels(orc, m, p, M, Lmax, N, seed=1):
    out = []
    for l in range(Lmax + 1):
        r = orc.level(m, p, l, M, N, seed=seed, nthreads=8)
        mean = r["sum_y"] / N
        out.append((mean, r["sum_y2"] / N - mean**2, r))
    return out


def test_telescoping_identity(orc):
    # sum_l Yhat_l estimates E[P_L]; compare with a direct estimate of E[P_L]
    for pk in (0, 1, 2, 3):
        m, p = orc.model(), orc.payoff(kind=pk)
        L, M, N = 3, 4, 30000
        lv = _levels(orc, m, p, M, L, N)
        tele = sum(x[0] for x in lv)
        var_tele = sum(x[1] / N for x in lv)
        d = orc.stdmc(m, p, L, M, N, seed=9, nthreads=8)
        dm = d["sum_y"] / N
        dv = d["sum_y2"] / N - dm**2
        assert abs(tele - dm) < 4.5 * np.sqrt(var_tele + dv / N), pk
        # E[coarse at level l] == E[fine at level l-1]
        for l in range(1, L + 1):
            r = lv[l][2]
            pcm = r["sum_pc"] / N
            pcv = r["sum_pc2"] / N - pcm**2
            prev = lv[l - 1][2]
            pfm = prev["sum_pf"] / N
            pfv = prev["sum_pf2"] / N - pfm**2
            assert abs(pcm - pfm) < 4.5 * np.sqrt(pcv / N + pfv / N), (pk, l)


def test_weak_order_one_call(orc):
    # |E[P_l] - BS| = O(dt_l): the error of the telescoped sum halves per level
    m, p = orc.model(), orc.payoff()
    bs = orc.bs_call()
    # exact level-0 error from the closed form, then per-level corrections
    e0, _ = orc.level0_call_moments(S0, K, R, SIG, T)
    lv = _levels(orc, m, p, 2, 6, 400000, seed=3)
    errs, acc = [], e0
    for l in range(1, 7):
        acc += lv[l][0]
        errs.append(abs(acc - bs))
    slope = np.polyfit(np.arange(1, 7), np.log2(errs), 1)[0]
    assert -1.4 < slope < -0.6, (slope, errs)


def test_variance_decay_rates(orc):
    M, N = 4, 60000
    betas = {}
    for pk in (0, 1, 2, 3):
        m, p = orc.model(), orc.payoff(kind=pk)
        lv = _levels(orc, m, p, M, 5, N, seed=4)
        V = np.array([x[1] for x in lv])
        betas[pk] = -np.polyfit(np.arange(2, 6), np.log(V[2:]) / np.log(M), 1)[0]
    assert 0.8 < betas[0] < 1.25, betas     # call: O(dt_l)
    assert 0.8 < betas[1] < 1.6, betas      # Asian
    assert 0.8 < betas[2] < 1.25, betas     # bridge lookback
    assert 0.3 < betas[3] < 0.7, betas      # digital: O(dt_l^(1/2))


def test_strong_order_half(orc):
    # E|S_N - S(T)| against the exact solution on the same Brownian path
    errs = []
    for l in range(2, 8):
        nf = 2**l
        h = T / nf
        e = []
        for s in range(600):
            z = orc.path_normals(7, l, s, 0, 1, nf)
            dw = np.sqrt(h) * z
            exact = S0 * np.exp((R - 0.5 * SIG**2) * T + SIG * dw.sum())
            p = orc.payoff(kind=0, K=0.0)
            sn = orc.path_payoff(orc.model(), p, dw) * np.exp(R * T)
            e.append(abs(sn - exact))
        errs.append(np.mean(e))
    slope = np.polyfit(np.arange(2, 8), np.log2(errs), 1)[0]
    assert -0.7 < slope < -0.3, (slope, errs)


def test_digital_tie_rule(orc):
    # r = 0 and zero increments keep S_N = S0 = K exactly: pays half
    m = orc.model(r=0.0)
    p = orc.payoff(kind=3, K=100.0, payout=100.0)
    assert orc.path_payoff(m, p, np.zeros(4)) == 50.0
    assert orc.path_payoff(m, p, np.full(4, 1e-3)) == 100.0
    assert orc.path_payoff(m, p, np.full(4, -1e-3)) == 0.0


def test_black_scholes_limit_cfg_parity_set(orc):
    # the parity configuration: M=2, l=0..5, N=20000, seed 1
    m, p = orc.model(), orc.payoff()
    lv = _levels(orc, m, p, 2, 5, 20000, seed=1)
    est = sum(x[0] for x in lv)
    sd = np.sqrt(sum(x[1] / 20000 for x in lv))
    bias = 0.03   # weak error at l = 5 (dt = 1/32) is well below this
    assert abs(est - orc.bs_call()) < 4 * sd + bias


def test_bad_arguments(orc):
    m, p = orc.model(), orc.payoff()
    with pytest.raises(ValueError):
        orc.level(m, p, -1, 2, 10, 1)
    with pytest.raises(ValueError):
        orc.level(m, p, 1, 1, 10, 1)
    with pytest.raises(ValueError):
        orc.level(m, orc.payoff(kind=7), 1, 2, 10, 1)
