"""Learned control variate on the GPU vs the oracle.

Per-sample parity is checked against the oracle in bf16-emulation mode (W2
and the layer-1 activations rounded to bf16 where the matrix cores read
them); the difference to the plain fp64 network is reported.  Rounding a
layer-1 activation to bf16 is a quantisation decision taken on an fp32 value
on the GPU and an fp64 value in the oracle, so a value within ~1 fp32 ulp of
a bf16 rounding midpoint can land on different neighbours (one bf16 ulp,
2^-8 relative); a path with such a flip moves by up to a few 1e-2.  The
observed share of such samples is at most 0.66% (flip_budget).  The bar:
|dP| <= 1e-3 S0 for every sample, and |dP| <= 1e-4 S0 for all but 1.5% of
the samples of a level l >= 1 case (none at level 0).  The control-variate
sum has mean zero, so estimates keep their expectation.
"""
import numpy as np
import pytest

from paper_1505_00965_amd import mlmc, workloads as W

pytestmark = pytest.mark.gpu
S0 = 100.0


def flip_budget(n, evals):
    """Samples of n allowed beyond 1e-4 S0.

    Set from the rates observed on MI355X with the networks of these tests
    (every case prints a CVFLIPS line): at most 27 of 4096 samples (0.66%,
    level 2, M = 4) on the 4096-sample cases and 7 of 2048 (0.34%) on the
    full-size launches, none at level 0 (one evaluation, at (0, S0)); the
    count does not grow with the number of evaluation points beyond level 2.
    The budget is about twice the worst observed rate."""
    return 0 if evals == 1 else int(np.ceil(0.015 * n))


def random_net(orc, in_dim, seed=3, scale=2.0):
    p = orc.cv_init(in_dim, 64, seed) * scale
    rng = np.random.default_rng(seed)
    p = p + 0.1 * rng.standard_normal(p.size) * (p == 0)   # non-zero biases
    return p.astype(np.float32)


def gpu_paths(gctx, m, p, l, M, N, seed, cv, offset=0):
    import torch
    pf = torch.empty(N, dtype=torch.float64, device="cuda")
    pc = torch.empty(N, dtype=torch.float64, device="cuda")
    gctx.mlmc_level_paths(m, p, l, M, N, seed, pf, pc, path_offset=offset, cv=cv)
    return pf.cpu().numpy(), pc.cpu().numpy()


def test_init_matches_oracle(gctx, orc):
    for d in (2, 3):
        cv = mlmc.ControlVariate(gctx, d, 64, init_seed=7)
        g = cv.get_params().astype(np.float64)
        o = orc.cv_init(d, 64, 7)
        assert g.size == o.size == (4417 if d == 2 else 4481)
        assert np.abs(g - o).max() < 1e-6
        cv.close()


def test_params_roundtrip(gctx, orc):
    cv = mlmc.ControlVariate(gctx, 2)
    p = random_net(orc, 2)
    cv.set_params(p)
    assert np.array_equal(cv.get_params(), p)
    with pytest.raises(mlmc.MLMCError):
        cv.set_params(p[:-1])
    bad = p.copy()
    bad[5] = np.nan
    with pytest.raises(mlmc.MLMCError):
        cv.set_params(bad)
    cv.close()


def flip_stats(pf, pc, rf, rc):
    """Samples beyond 1e-4 S0 and the largest |dP| of a case."""
    d = np.maximum(np.abs(pf - rf), np.abs(pc - rc))
    return int((d > 1e-4 * S0).sum()), float(d.max())


@pytest.mark.parametrize("kind,pname,M", [(0, "call", 4), (0, "asian", 4), (0, "lookback", 2),
                                          (0, "digital", 4), (1, "call", 4)])
def test_forward_parity_bf16_emulation(gctx, orc, kind, pname, M):
    md = W.GBM_MODEL if kind == 0 else W.HESTON_MODEL
    gm, om = mlmc.model(**md), orc.model(**md)
    gp, op = mlmc.payoff(**W.PAYOFFS[pname]), orc.payoff(**W.PAYOFFS[pname])
    d = 3 if kind else 2
    params = random_net(orc, d)
    cv = mlmc.ControlVariate(gctx, d)
    cv.set_params(params)
    emu = orc.CVNet(params.astype(np.float64), d, 64, bf16_emulate=True)
    f64 = orc.CVNet(params.astype(np.float64), d, 64, bf16_emulate=False)
    N = 4096
    for l in (0, 1, 2, 3):
        for off in (0, 5):
            print(f"case kind={kind} payoff={pname} M={M} l={l} off={off}", flush=True)
            pf, pc = gpu_paths(gctx, gm, gp, l, M, N, 11, cv, offset=off)
            rf, rc = orc.level_paths(om, op, l, M, N, 11, off, cv=emu, nthreads=8)
            nbad, err = flip_stats(pf, pc, rf, rc)
            bad = (np.abs(pf - rf) > 1e-4 * S0) | (np.abs(pc - rc) > 1e-4 * S0)
            evals = M**l + (M ** (l - 1) if l else 0)
            print(f"CVFLIPS kind={kind} payoff={pname} M={M} l={l} off={off} N={N} "
                  f"evals={evals} beyond={nbad} max={err:.3e}", flush=True)
            if pname == "digital" and bad.any():
                k0 = orc.payoff(kind=0, K=0.0)
                sf, sc = orc.level_paths(om, k0, l, M, N, 11, off, nthreads=8)
                disc = np.exp(-om.r * om.T)
                # a flipped digital changes P by the payout; the control-variate sums agree
                near = (np.abs(sf / disc - 100.0) < 2e-2) | (np.abs(sc / disc - 100.0) < 2e-2)
                bad = bad & ~near
                nbad = int(bad.sum())
                err = float(np.maximum(np.abs(pf - rf), np.abs(pc - rc))[~near].max())
            assert nbad <= flip_budget(N, evals) and err <= 1e-3 * S0, (l, off, err, nbad)
            xf, xc = orc.level_paths(om, op, l, M, 200, 11, off, cv=f64, nthreads=8)
            print(f"  max |dP| vs bf16 emulation {err:.2e}; vs fp64 network "
                  f"{max(np.abs(pf[:200] - xf).max(), np.abs(pc[:200] - xc).max()):.2e}")
    cv.close()


def test_forward_parity_full_size_sampled(gctx, orc):
    """Launch sizes where the sampler's grid-stride loop runs several chunks
    per block (2^20 samples, levels 1..3, GBM Asian and Heston call): 2048
    seeded random samples of each launch recomputed one by one by the
    oracle in bf16-emulation mode."""
    import torch
    rng = np.random.default_rng(20)
    for kind, pname in ((0, "asian"), (1, "call")):
        md = W.GBM_MODEL if kind == 0 else W.HESTON_MODEL
        gm, om = mlmc.model(**md), orc.model(**md)
        gp, op = mlmc.payoff(**W.PAYOFFS[pname]), orc.payoff(**W.PAYOFFS[pname])
        d = 3 if kind else 2
        params = random_net(orc, d, seed=8)
        cv = mlmc.ControlVariate(gctx, d)
        cv.set_params(params)
        emu = orc.CVNet(params.astype(np.float64), d, 64, bf16_emulate=True)
        N = 1 << 20
        for l in (1, 2, 3):
            print(f"case full-size kind={kind} payoff={pname} l={l} N={N}", flush=True)
            pf, pc = gpu_paths(gctx, gm, gp, l, 4, N, 13, cv, offset=7)
            idx = np.sort(rng.choice(N, 2048, replace=False))
            rf = np.empty(idx.size)
            rc = np.empty(idx.size)
            for j, i in enumerate(idx):
                rf[j], rc[j], _, _ = orc.level_sample(om, op, l, 4, 13, 7 + int(i), cv=emu)
            nbad, err = flip_stats(pf[idx], pc[idx], rf, rc)
            evals = 4**l + 4 ** (l - 1)
            print(f"CVFLIPS full-size kind={kind} payoff={pname} M=4 l={l} N=2048 "
                  f"evals={evals} beyond={nbad} max={err:.3e}", flush=True)
            assert nbad <= flip_budget(idx.size, evals) and err <= 1e-3 * S0, (l, nbad, err)
            assert np.all(np.isfinite(pf)) and np.all(np.isfinite(pc))
        cv.close()
        torch.cuda.empty_cache()


def test_adam_step_and_trajectory_match_oracle(gctx, orc):
    """The device's Adam update (Kingma and Ba) against the oracle's, on the
    gradients the device computes: ten training steps, each compared element
    by element after the oracle applies the same step to its own copy of
    the parameters and moments."""
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.ASIAN)
    params = random_net(orc, 2, seed=12)
    cv = mlmc.ControlVariate(gctx, 2)
    cv.set_params(params)
    theta = params.astype(np.float64)
    m1, m2 = np.zeros_like(theta), np.zeros_like(theta)
    lr, B, lmax, M, seed = 1e-3, 1024, 2, 4, 31
    for t in range(10):
        before = cv.get_params().astype(np.float64)
        # the gradient the next training step computes (same batch, same step)
        _, g, _ = cv.loss_grad(gm, gp, M, lmax, B, seed, step=t)
        cv.train(gm, gp, M=M, lmax=lmax, steps=1, batch=B, lr=lr, seed=seed)
        after = cv.get_params().astype(np.float64)
        one = before.copy()
        a1, a2 = m1.copy(), m2.copy()
        orc.adam(one, a1, a2, g.astype(np.float64), lr=lr, t=t + 1)
        orc.adam(theta, m1, m2, g.astype(np.float64), lr=lr, t=t + 1)
        # one step from the device's parameters: fp32 rounding of the update
        # and of the parameter only
        step_err = np.abs(after - one)
        assert np.all(step_err <= 1e-5 * lr + 2.4e-7 * np.abs(one)), (t, step_err.max())
        # ten steps from the same start: the trajectories stay together
        traj = np.abs(after - theta)
        assert np.all(traj <= (t + 1) * (1e-5 * lr + 2.4e-7 * np.abs(theta))), (t, traj.max())
        moved = np.abs(after - before)
        if t == 0:
            # the first step moves every parameter with a gradient by lr sign(g)
            assert np.median(moved) > 0.9 * lr
    cv.close()


def test_control_variate_keeps_the_mean(gctx, orc):
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.ASIAN)
    cv = mlmc.ControlVariate(gctx, 2)
    cv.set_params(random_net(orc, 2, seed=9, scale=3.0))
    N = 200000
    for l in (0, 2):
        pf0, pc0 = gpu_paths(gctx, gm, gp, l, 4, N, 4, None)
        pf1, pc1 = gpu_paths(gctx, gm, gp, l, 4, N, 4, cv)
        for d in (pf0 - pf1, pc0 - pc1):      # the control-variate sums themselves
            if np.all(d == 0):
                continue
            assert abs(d.mean()) < 4.5 * d.std() / np.sqrt(N), (l, d.mean(), d.std())
    cv.close()


def test_run_with_control_variate(gctx, orc):
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    cv = mlmc.ControlVariate(gctx, 2)
    eps = 0.2
    errs = [gctx.mlmc_run(gm, gp, eps, M=4, seed=s, cv=cv)["estimate"] - orc.bs_call()
            for s in range(1, 17)]
    assert np.sqrt(np.mean(np.square(errs))) < 1.35 * eps
    # the network on level 0 only: still unbiased
    errs = [gctx.mlmc_run(gm, gp, eps, M=4, seed=s, cv=cv, cv_levels=1)["estimate"] - orc.bs_call()
            for s in range(1, 17)]
    assert np.sqrt(np.mean(np.square(errs))) < 1.35 * eps
    with pytest.raises(mlmc.MLMCError):
        gctx.mlmc_run(gm, gp, eps, cv=cv, precision=64)
    with pytest.raises(mlmc.MLMCError):     # the device-planned form takes the table
        gctx.mlmc_run(gm, gp, eps, cv=cv, persistent=True)
    with pytest.raises(mlmc.MLMCError):     # Heston needs a 3-input network
        gctx.mlmc_level(mlmc.model(**W.HESTON_MODEL), gp, 1, 4, 100, 1, cv=cv)
    cv.close()


@pytest.mark.parametrize("kind,pname", [(0, "asian"), (0, "call"), (1, "call")])
def test_loss_gradient_parity(gctx, orc, kind, pname):
    md = W.GBM_MODEL if kind == 0 else W.HESTON_MODEL
    gm, om = mlmc.model(**md), orc.model(**md)
    gp, op = mlmc.payoff(**W.PAYOFFS[pname]), orc.payoff(**W.PAYOFFS[pname])
    d = 3 if kind else 2
    params = random_net(orc, d, seed=5)
    cv = mlmc.ControlVariate(gctx, d)
    cv.set_params(params)
    B, lmax, M = 512, 2, 4
    loss, g, var = cv.loss_grad(gm, gp, M, lmax, B, seed=9, step=3)
    emu = orc.CVNet(params.astype(np.float64), d, 64, bf16_emulate=True)
    oloss, og, ovar = orc.cv_loss_grad(om, op, M, lmax, B, 9, 3, emu, nthreads=8)
    print(f"loss gpu {loss:.8g} oracle {oloss:.8g}; var {var} vs {list(ovar)}")
    assert abs(loss - oloss) <= 1e-4 * abs(oloss)
    assert np.allclose(var, ovar, rtol=1e-4)
    g = g.astype(np.float64)
    rel = np.linalg.norm(g - og) / np.linalg.norm(og)
    cos = g @ og / (np.linalg.norm(g) * np.linalg.norm(og))
    print(f"gradient rel L2 {rel:.3e}, cosine {cos:.8f}")
    assert rel <= 2e-2 and cos >= 0.999
    # every parameter group gets the right gradient, not only the big ones
    offs = [0, 64 * d, 64 * d + 64, 64 * d + 64 + 4096, 64 * d + 128 + 4096, 64 * d + 192 + 4096,
            g.size]
    for a, b in zip(offs, offs[1:]):
        rg = np.linalg.norm(g[a:b] - og[a:b]) / max(np.linalg.norm(og[a:b]), 1e-30)
        assert rg <= 5e-2, (a, b, rg)
    cv.close()


def test_level0_training_reaches_closed_form(gctx, orc):
    # one step: phi(0, S0) is a scalar c; optimum c* = Cov(P_0, dW)/T, V_0 = 31.371655
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    cv = mlmc.ControlVariate(gctx, 2, init_seed=1)
    hist = cv.train(gm, gp, M=4, lmax=0, steps=300, batch=16384, lr=1e-2, seed=21)
    assert hist[-1] < hist[0]
    r = gctx.mlmc_level(gm, gp, 0, 4, 1 << 22, 5, cv=cv)
    v0 = r["sum_y2"] / r["n"] - (r["sum_y"] / r["n"]) ** 2
    print("trained V_0", v0, "loss", hist[0], "->", hist[-1])
    assert v0 < 1.05 * 31.371655
    e0, _ = orc.level0_call_moments(100.0, 100.0, 0.05, 0.2, 1.0)
    assert abs(r["sum_y"] / r["n"] - e0) < 5 * np.sqrt(v0 / r["n"])
    cv.close()


def test_training_reduces_level_variances(gctx):
    """What the trained network gains: level variances with and without it."""
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.ASIAN)
    cv = mlmc.ControlVariate(gctx, 2, init_seed=1)
    hist = cv.train(gm, gp, M=4, lmax=3, steps=200, batch=4096, lr=3e-3, seed=2)
    assert np.all(np.isfinite(hist)) and hist[-20:].mean() < hist[:20].mean()
    gains = []
    for l in range(4):
        a = gctx.mlmc_level(gm, gp, l, 4, 1 << 16, 77)
        b = gctx.mlmc_level(gm, gp, l, 4, 1 << 16, 77, cv=cv)
        va = a["sum_y2"] / a["n"] - (a["sum_y"] / a["n"]) ** 2
        vb = b["sum_y2"] / b["n"] - (b["sum_y"] / b["n"]) ** 2
        gains.append(va / vb)
    print("variance reduction per level", gains)
    assert gains[0] > 2.0
