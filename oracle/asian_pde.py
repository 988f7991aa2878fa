"""Continuous arithmetic-average Asian call by Vecer's one-dimensional PDE
(test infrastructure only).

The arithmetic Asian named in Sec. 7.1 has no closed form; this is an
independent characterisation of its continuous-time price, solved on a grid.
With q(t) = (1 - e^{-r(T-t)})/(rT) shares held, a self-financing portfolio X
with X_0 = q(0) S0 - e^{-rT} K ends at X_T = A - K (A the time average of S).
Z = X/S is a martingale under the measure that takes the share as numeraire,
with dZ = sigma (q(t) - Z) dW, so the price is S0 u(0, Z_0), where
    u_t + sigma^2 (q(t) - z)^2 u_zz / 2 = 0,   u(T, z) = max(z, 0).
"""
import math

import numpy as np


def asian_arith_call_pde(S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, nz=4000, nt=2000,
                         zlo=-2.0, zhi=3.0, damp=4):
    """Crank--Nicolson on a uniform z grid, `damp` pairs of half-size implicit
    steps first (Rannacher), u = 0 and u = z at the ends of the grid."""
    from scipy.linalg import solve_banded
    z = np.linspace(zlo, zhi, nz + 1)
    dz = z[1] - z[0]
    zi = z[1:-1]
    u = np.maximum(z, 0.0)

    def q(t):
        return (1.0 - math.exp(-r * (T - t))) / (r * T) if r != 0 else (T - t) / T

    dt = T / nt
    steps = [(dt / 2, 1.0)] * (2 * damp) + [(dt, 0.5)] * (nt - damp)
    t = T
    for k, th in steps:
        tn = t - k
        a_new = 0.5 * sigma**2 * (q(tn) - zi) ** 2 / dz**2
        a_old = 0.5 * sigma**2 * (q(t) - zi) ** 2 / dz**2
        rhs = u[1:-1] + (1 - th) * k * a_old * (u[:-2] - 2 * u[1:-1] + u[2:])
        rhs[-1] += th * k * a_new[-1] * zhi
        ab = np.zeros((3, nz - 1))
        ab[0, 1:] = -th * k * a_new[:-1]
        ab[1, :] = 1 + 2 * th * k * a_new
        ab[2, :-1] = -th * k * a_new[1:]
        u[1:-1] = solve_banded((1, 1), ab, rhs)
        u[0], u[-1] = 0.0, zhi
        t = tn
    z0 = q(0.0) - math.exp(-r * T) * K / S0
    return S0 * float(np.interp(z0, z, u))
