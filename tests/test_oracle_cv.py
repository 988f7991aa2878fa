"""Pins for the oracle's learned control variate (CPU only).

The control variate sum_n phi(t_n, X_n) dW_n has mean zero for any phi
evaluated at the left point (the classic control-variate requirement of a
known mean, Sec. 5 "Exploiting Structure"); the network, loss and optimiser
are readings.  Pins: finite-difference gradients, mean zero, the closed-form
level-0 optimum, and Adam's first-step property.
"""
import numpy as np
import pytest
from scipy import integrate, stats

S0, K, R, SIG, T = 100.0, 100.0, 0.05, 0.2, 1.0


def net(orc, in_dim=2, seed=1, bf16=False, scale=1.0):
    p = orc.cv_init(in_dim, 64, seed)
    # non-zero biases so every parameter is exercised
    rng = np.random.default_rng(seed)
    p = p * scale + 0.05 * rng.standard_normal(p.size) * (p == 0)
    return orc.CVNet(p, in_dim, 64, bf16)


def test_param_count_and_init(orc):
    assert orc.cv_nparams(2, 64) == 4417
    assert orc.cv_nparams(3, 64) == 4481
    p = orc.cv_init(2, 64, 1)
    W1, b1 = p[:128], p[128:192]
    W2 = p[192:192 + 4096]
    assert np.all(b1 == 0) and p[-1] == 0
    a2 = np.sqrt(6 / 128)
    assert np.abs(W2).max() <= a2 and np.abs(W2).max() > 0.95 * a2
    assert abs(W2.mean()) < 3 * a2 / np.sqrt(3 * 4096)
    assert np.abs(W1).max() <= np.sqrt(6 / 66)


@pytest.mark.parametrize("kind", [0, 1])
def test_phi_gradient_finite_difference(orc, kind):
    m = orc.model(kind=kind)
    d = 3 if kind else 2
    cv = net(orc, d, seed=3)
    rng = np.random.default_rng(0)
    for (t, S, v) in [(0.0, 100.0, 0.04), (0.3, 91.0, 0.02), (0.77, 123.0, 0.06)]:
        g = orc.cv_phi_grad(m, cv, t, S, v, 1.0)
        idx = np.concatenate([rng.choice(cv.params.size, 80, replace=False),
                              [cv.params.size - 1, 0, 5, 200]])
        for i in idx:
            base = cv.params[i]
            hstep = 1e-6
            cv.params[i] = base + hstep
            fp = orc.cv_phi(m, cv, t, S, v)
            cv.params[i] = base - hstep
            fm = orc.cv_phi(m, cv, t, S, v)
            cv.params[i] = base
            fd = (fp - fm) / (2 * hstep)
            assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_loss_gradient_finite_difference(orc):
    m, p = orc.model(), orc.payoff(kind=1)
    cv = net(orc, 2, seed=5)
    loss, g, var = orc.cv_loss_grad(m, p, 4, 2, 64, seed=9, step=2, cv=cv, nthreads=4)
    assert np.isfinite(loss) and np.all(var > 0)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(cv.params.size, 40, replace=False), [cv.params.size - 1]])
    for i in idx:
        base = cv.params[i]
        hstep = 1e-5
        cv.params[i] = base + hstep
        lp = orc.cv_loss_grad(m, p, 4, 2, 64, 9, 2, cv, 4, want_grad=False)[0]
        cv.params[i] = base - hstep
        lm = orc.cv_loss_grad(m, p, 4, 2, 64, 9, 2, cv, 4, want_grad=False)[0]
        cv.params[i] = base
        fd = (lp - lm) / (2 * hstep)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7, (i, fd, g[i])


@pytest.mark.parametrize("kind,pk", [(0, 1), (1, 0)])
def test_control_variate_has_mean_zero(orc, kind, pk):
    m, p = orc.model(kind=kind), orc.payoff(kind=pk)
    cv = net(orc, 3 if kind else 2, seed=7, scale=3.0)
    l, M, N = 2, 4, 20000
    cf = np.empty(N)
    cc = np.empty(N)
    for s in range(N):
        _, _, cf[s], cc[s] = orc.level_sample(m, p, l, M, 1, s, 0, cv)
    for x in (cf, cc, cf - cc):
        assert abs(x.mean()) < 4.5 * x.std() / np.sqrt(N)
    assert cf.std() > 1.0      # the term is not trivially zero


def _v0_min_by_quadrature():
    disc = np.exp(-R * T)
    pay = lambda z: disc * max(S0 * (1 + R * T + SIG * np.sqrt(T) * z) - K, 0.0)
    w = lambda f: integrate.quad(lambda z: f(z) * stats.norm.pdf(z), -12, 12, points=[-0.25])[0]
    m1, m2 = w(pay), w(lambda z: pay(z) ** 2)
    cov = w(lambda z: pay(z) * np.sqrt(T) * z)      # Cov(P_0, dW)
    c_star = cov / T
    return c_star, (m2 - m1 * m1) - c_star * cov


def test_level0_optimum_closed_form(orc):
    c_star, vmin = _v0_min_by_quadrature()
    assert abs(c_star - 11.390141) < 2e-6 and abs(vmin - 31.371655) < 2e-5
    m, p = orc.model(), orc.payoff()
    # a network that outputs the constant c_star everywhere
    params = np.zeros(orc.cv_nparams(2, 64))
    params[-1] = c_star / orc.cv_out_scale(m)
    cv = orc.CVNet(params)
    r = orc.level(m, p, 0, 4, 200000, seed=3, cv=cv, nthreads=8)
    mean = r["sum_y"] / r["n"]
    var = r["sum_y2"] / r["n"] - mean**2
    assert abs(var / vmin - 1) < 0.03
    e0, _ = orc.level0_call_moments(S0, K, R, SIG, T)
    assert abs(mean - e0) < 4.5 * np.sqrt(vmin / r["n"])


def test_level0_training_reaches_optimum(orc):
    c_star, vmin = _v0_min_by_quadrature()
    m, p = orc.model(), orc.payoff()
    cv = orc.CVNet(orc.cv_init(2, 64, 1))
    m1 = np.zeros_like(cv.params)
    m2 = np.zeros_like(cv.params)
    for step in range(1, 301):
        loss, g, var = orc.cv_loss_grad(m, p, 4, 0, 4096, seed=11, step=step, cv=cv, nthreads=8)
        orc.adam(cv.params, m1, m2, g, lr=1e-2, t=step)
    phi0 = orc.cv_phi(m, cv, 0.0, S0)
    assert abs(phi0 / c_star - 1) < 0.03, phi0
    loss, _, var = orc.cv_loss_grad(m, p, 4, 0, 100000, seed=12, step=0, cv=cv, nthreads=8,
                                    want_grad=False)
    assert var[0] < 1.05 * vmin


def test_adam_first_step_is_lr_times_sign(orc):
    theta = np.array([1.0, -2.0, 3.0, 0.5])
    g = np.array([0.3, -5.0, 1e-3, -2e4])
    m1, m2 = np.zeros(4), np.zeros(4)
    t0 = theta.copy()
    orc.adam(theta, m1, m2, g, lr=0.01, t=1)
    assert np.allclose(t0 - theta, 0.01 * np.sign(g), rtol=1e-4)
    # minimises a quadratic
    x = np.array([5.0, -3.0])
    a, b = np.zeros(2), np.zeros(2)
    for t in range(1, 3001):
        orc.adam(x, a, b, 2 * x, lr=0.05, t=t)
    assert np.abs(x).max() < 1e-2


def test_bf16_emulation_error_bound(orc):
    m = orc.model()
    p64 = net(orc, 2, seed=4)
    p16 = orc.CVNet(p64.params.copy(), 2, 64, True)
    for (t, S) in [(0.0, 100.0), (0.5, 80.0), (0.9, 130.0)]:
        a = orc.cv_phi(m, p64, t, S)
        b = orc.cv_phi(m, p16, t, S)
        # each bf16 rounding is relative <= 2^-9; bound the propagated change
        bound = orc.cv_out_scale(m) * np.abs(p64.params[4352:4416]).sum() * 0.05
        assert 0 < abs(a - b) < bound
