"""ctypes view of the FP64 C oracle (liboracle.so) -- test infrastructure only.

Every function here only marshals arguments; the arithmetic is in the C files
next to this one.  The structures are declared here independently of the GPU
library's header.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB selects another build of the same sources (the sanitizer build)
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

GBM, HESTON = 0, 1
EULER, MILSTEIN = 0, 1
CALL, ASIAN, LOOKBACK, DIGITAL, DIGITAL_COND = 0, 1, 2, 3, 4
STREAM_NORMAL, STREAM_BRIDGE, STREAM_TRAIN_NORMAL, STREAM_TRAIN_BRIDGE = 0, 1, 2, 3
STREAM_STDMC, STREAM_STDMC_BRIDGE, STREAM_INIT, STREAM_LEVEL_DRAW = 4, 5, 6, 7


class Model(C.Structure):
    _fields_ = [("kind", C.c_int), ("S0", C.c_double), ("r", C.c_double),
                ("sigma", C.c_double), ("T", C.c_double), ("kappa", C.c_double),
                ("theta", C.c_double), ("xi", C.c_double), ("rho", C.c_double),
                ("v0", C.c_double), ("scheme", C.c_int), ("antithetic", C.c_int)]


class Payoff(C.Structure):
    _fields_ = [("kind", C.c_int), ("K", C.c_double), ("payout", C.c_double)]


class CVTable(C.Structure):
    _fields_ = [("rows", C.c_int), ("ns", C.c_int), ("nv", C.c_int), ("s_lo", C.c_double),
                ("s_hi", C.c_double), ("v_lo", C.c_double), ("v_hi", C.c_double),
                ("values", C.POINTER(C.c_double))]


class CV(C.Structure):
    _fields_ = [("in_dim", C.c_int), ("hidden", C.c_int),
                ("params", C.POINTER(C.c_double)), ("bf16_emulate", C.c_int),
                ("table", C.POINTER(CVTable))]


class LevelResult(C.Structure):
    _fields_ = [("sum_y", C.c_double), ("sum_y2", C.c_double), ("sum_pf", C.c_double),
                ("sum_pf2", C.c_double), ("sum_pc", C.c_double), ("sum_pc2", C.c_double),
                ("cost", C.c_double), ("n", C.c_uint64), ("n_nonfinite", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RunOpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("M", C.c_int), ("L_min", C.c_int), ("L_max", C.c_int),
                ("n_pilot", C.c_uint64), ("seed", C.c_uint64), ("alpha", C.c_double),
                ("beta", C.c_double), ("nthreads", C.c_int), ("cv", C.POINTER(CV))]


class RGResult(C.Structure):
    _fields_ = [("estimate", C.c_double), ("variance", C.c_double), ("cost", C.c_double),
                ("Lc", C.c_int), ("N", C.c_uint64 * 16), ("p", C.c_double * 16),
                ("sum_y", C.c_double * 16), ("sum_y2", C.c_double * 16),
                ("n_nonfinite", C.c_uint64)]


class RunResult(C.Structure):
    _fields_ = [("estimate", C.c_double), ("L", C.c_int), ("converged", C.c_int),
                ("iterations", C.c_int), ("N", C.c_uint64 * 16), ("sum_y", C.c_double * 16),
                ("sum_y2", C.c_double * 16), ("V", C.c_double * 16), ("E", C.c_double * 16),
                ("C", C.c_double * 16), ("alpha", C.c_double), ("beta", C.c_double),
                ("gamma", C.c_double), ("cost", C.c_double)]


_lib = None


def lib():
    """Load liboracle.so, building it with gcc first if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        dp, u64, i32, d = C.POINTER(C.c_double), C.c_uint64, C.c_int, C.c_double
        u32p = C.POINTER(C.c_uint32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = d
        L.orc_box_muller.argtypes = [C.c_uint32, C.c_uint32, dp, dp]
        L.orc_path_words.argtypes = [u64, i32, u64, i32, C.c_uint32, u32p]
        L.orc_path_normals.argtypes = [u64, i32, u64, i32, i32, i32, dp]
        L.orc_path_uniforms.argtypes = [u64, i32, u64, i32, i32, dp]
        L.orc_level_sample.argtypes = [C.POINTER(Model), C.POINTER(Payoff), i32, i32, u64, u64,
                                       i32, C.POINTER(CV), dp, dp, dp, dp]
        L.orc_path_payoff.argtypes = [C.POINTER(Model), C.POINTER(Payoff), i32, dp, dp]
        L.orc_path_payoff.restype = d
        L.orc_level.argtypes = [C.POINTER(Model), C.POINTER(Payoff), i32, i32, u64, u64, u64,
                                C.POINTER(CV), i32, C.POINTER(LevelResult)]
        L.orc_level_paths.argtypes = [C.POINTER(Model), C.POINTER(Payoff), i32, i32, u64, u64,
                                      u64, C.POINTER(CV), i32, dp, dp]
        L.orc_stdmc.argtypes = [C.POINTER(Model), C.POINTER(Payoff), i32, i32, u64, u64, u64,
                                i32, C.POINTER(LevelResult)]
        L.orc_optimal_n.argtypes = [i32, dp, dp, d, dp]
        L.orc_level_cost.argtypes = [i32, i32, i32]
        L.orc_level_cost.restype = d
        L.orc_mlmc_run.argtypes = [C.POINTER(Model), C.POINTER(Payoff), C.POINTER(RunOpts),
                                   C.POINTER(RunResult)]
        L.orc_fit_rate.argtypes = [i32, dp, i32]
        L.orc_fit_rate.restype = d
        for name, n in [("orc_norm_cdf", 1), ("orc_bs_call", 5), ("orc_bs_digital", 6),
                        ("orc_lookback_float_call", 4), ("orc_geometric_asian_call", 5),
                        ("orc_heston_call", 9)]:
            fn = getattr(L, name)
            fn.argtypes = [d] * n
            fn.restype = d
        L.orc_euler_k0_moments.argtypes = [d, d, d, d, i32, i32, dp]
        L.orc_level0_call_moments.argtypes = [d, d, d, d, d, dp]
        L.orc_cv_nparams.argtypes = [i32, i32]
        L.orc_cv_nparams.restype = C.c_size_t
        L.orc_cv_init.argtypes = [i32, i32, u64, dp]
        L.orc_cv_inputs.argtypes = [C.POINTER(Model), d, d, d, dp]
        L.orc_cv_out_scale.argtypes = [C.POINTER(Model)]
        L.orc_cv_out_scale.restype = d
        L.orc_cv_phi.argtypes = [C.POINTER(Model), C.POINTER(CV), d, d, d]
        L.orc_cv_phi.restype = d
        L.orc_cv_phi_grad.argtypes = [C.POINTER(Model), C.POINTER(CV), d, d, d, d, dp]
        L.orc_cv_table_grid.argtypes = [C.POINTER(Model), C.POINTER(CVTable)]
        L.orc_cv_table_fill.argtypes = [C.POINTER(Model), C.POINTER(CV), C.POINTER(CVTable), dp]
        L.orc_cv_loss_grad.argtypes = [C.POINTER(Model), C.POINTER(Payoff), i32, i32, u64, u64,
                                       u64, C.POINTER(CV), i32, dp, dp]
        L.orc_cv_loss_grad.restype = d
        L.orc_adam.argtypes = [C.c_size_t, dp, dp, dp, dp, d, d, d, d, i32]
        L.orc_rg_probabilities.argtypes = [d, i32, dp, dp]
        L.orc_rg_level_counts.argtypes = [u64, u64, d, i32, C.POINTER(C.c_uint64)]
        L.orc_rhee_glynn.argtypes = [C.POINTER(Model), C.POINTER(Payoff), i32, i32, d, u64, u64,
                                     i32, C.POINTER(RGResult)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u32p(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def model(kind=GBM, S0=100.0, r=0.05, sigma=0.2, T=1.0, kappa=2.0, theta=0.04, xi=0.3,
          rho=-0.7, v0=0.04, scheme=0, antithetic=0):
    return Model(kind, S0, r, sigma, T, kappa, theta, xi, rho, v0, scheme, antithetic)


def payoff(kind=CALL, K=100.0, payout=1.0):
    return Payoff(kind, K, payout)


class CVNet:
    """Holds an FP64 parameter vector and the C view of it.  With a table
    (values shaped [rows, nv, ns] on the grid cv_table_grid gives for the
    model) phi is read from the table instead of the network."""

    def __init__(self, params, in_dim=2, hidden=64, bf16_emulate=False, table=None, grid=None):
        self.params = np.ascontiguousarray(params, dtype=np.float64)
        self.in_dim, self.hidden = in_dim, hidden
        self.c = CV(in_dim, hidden, _dp(self.params), int(bf16_emulate), None)
        self.table = None
        if table is not None:
            self.values = np.ascontiguousarray(table, dtype=np.float64).ravel()
            g = grid
            assert self.values.size == g.rows * g.nv * g.ns
            self.table = CVTable(g.rows, g.ns, g.nv, g.s_lo, g.s_hi, g.v_lo, g.v_hi,
                                 _dp(self.values))
            self.c.table = C.pointer(self.table)

    def ref(self):
        return C.byref(self.c)


def cv_table_grid(m):
    g = CVTable()
    lib().orc_cv_table_grid(C.byref(m), C.byref(g))
    return g


def cv_table_fill(m, cv, grid):
    """The network cv on the grid: array [rows, nv, ns]."""
    out = np.zeros(grid.rows * grid.nv * grid.ns)
    lib().orc_cv_table_fill(C.byref(m), cv.ref(), C.byref(grid), _dp(out))
    return out.reshape(grid.rows, grid.nv, grid.ns)


def _cvref(cv):
    return None if cv is None else cv.ref()


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_u32p(c), _u32p(k), _u32p(out))
    return out


def u01(x):
    return lib().orc_u01(int(x))


def box_muller(a, b):
    z0, z1 = C.c_double(), C.c_double()
    lib().orc_box_muller(int(a), int(b), C.byref(z0), C.byref(z1))
    return z0.value, z1.value


def path_words(seed, level, s, stream, nblocks):
    out = np.zeros(4 * nblocks, np.uint32)
    lib().orc_path_words(seed, level, s, stream, nblocks, _u32p(out))
    return out


def path_normals(seed, level, s, stream, dim, nsteps):
    z = np.zeros(nsteps * dim)
    lib().orc_path_normals(seed, level, s, stream, dim, nsteps, _dp(z))
    return z


def path_uniforms(seed, level, s, stream, nsteps):
    u = np.zeros(nsteps)
    lib().orc_path_uniforms(seed, level, s, stream, nsteps, _dp(u))
    return u


def level_sample(m, p, l, M, seed, s, stream=STREAM_NORMAL, cv=None):
    pf, pc, cf, cc = (C.c_double() for _ in range(4))
    rc = lib().orc_level_sample(C.byref(m), C.byref(p), l, M, seed, s, stream, _cvref(cv),
                                C.byref(pf), C.byref(pc), C.byref(cf), C.byref(cc))
    if rc:
        raise ValueError("orc_level_sample: bad arguments")
    return pf.value, pc.value, cf.value, cc.value


def path_payoff(m, p, dw, u=None):
    dw = np.ascontiguousarray(dw, dtype=np.float64)
    dim = 2 if m.kind == HESTON else 1
    n = dw.size // dim
    uu = np.ascontiguousarray(u if u is not None else np.full(n, 0.5), dtype=np.float64)
    return lib().orc_path_payoff(C.byref(m), C.byref(p), n, _dp(dw), _dp(uu))


def level(m, p, l, M, N, seed, offset=0, cv=None, nthreads=1):
    r = LevelResult()
    rc = lib().orc_level(C.byref(m), C.byref(p), l, M, N, seed, offset, _cvref(cv), nthreads,
                         C.byref(r))
    if rc:
        raise ValueError("orc_level: bad arguments")
    return r.as_dict()


def level_paths(m, p, l, M, N, seed, offset=0, cv=None, nthreads=1):
    pf = np.zeros(N)
    pc = np.zeros(N)
    rc = lib().orc_level_paths(C.byref(m), C.byref(p), l, M, N, seed, offset, _cvref(cv),
                               nthreads, _dp(pf), _dp(pc))
    if rc:
        raise ValueError("orc_level_paths: bad arguments")
    return pf, pc


def stdmc(m, p, L, M, N, seed, offset=0, nthreads=1):
    r = LevelResult()
    rc = lib().orc_stdmc(C.byref(m), C.byref(p), L, M, N, seed, offset, nthreads, C.byref(r))
    if rc:
        raise ValueError("orc_stdmc: bad arguments")
    return r.as_dict()


def optimal_n(V, Cl, eps):
    V = np.ascontiguousarray(V, dtype=np.float64)
    Cl = np.ascontiguousarray(Cl, dtype=np.float64)
    N = np.zeros(V.size)
    lib().orc_optimal_n(V.size - 1, _dp(V), _dp(Cl), eps, _dp(N))
    return N


def level_cost(l, M, antithetic=0):
    return lib().orc_level_cost(l, M, antithetic)


def fit_rate(y, M):
    y = np.ascontiguousarray(y, dtype=np.float64)
    return lib().orc_fit_rate(y.size - 1, _dp(y), M)


def mlmc_run(m, p, eps, M=4, L_min=2, L_max=8, n_pilot=10000, seed=1, alpha=0.0, beta=0.0,
             nthreads=1, cv=None):
    o = RunOpts(eps, M, L_min, L_max, n_pilot, seed, alpha, beta, nthreads,
                None if cv is None else C.pointer(cv.c))
    r = RunResult()
    rc = lib().orc_mlmc_run(C.byref(m), C.byref(p), C.byref(o), C.byref(r))
    if rc:
        raise ValueError("orc_mlmc_run: bad arguments")
    L = r.L
    return {"estimate": r.estimate, "L": L, "converged": bool(r.converged),
            "iterations": r.iterations, "N": list(r.N)[:L + 1], "V": list(r.V)[:L + 1],
            "E": list(r.E)[:L + 1], "C": list(r.C)[:L + 1], "sum_y": list(r.sum_y)[:L + 1],
            "sum_y2": list(r.sum_y2)[:L + 1], "alpha": r.alpha, "beta": r.beta,
            "gamma": r.gamma, "cost": r.cost}


def norm_cdf(x):
    return lib().orc_norm_cdf(x)


def bs_call(S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0):
    return lib().orc_bs_call(S0, K, r, sigma, T)


def bs_digital(S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, payout=1.0):
    return lib().orc_bs_digital(S0, K, r, sigma, T, payout)


def lookback_float_call(S0=100.0, r=0.05, sigma=0.2, T=1.0):
    return lib().orc_lookback_float_call(S0, r, sigma, T)


def geometric_asian_call(S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0):
    return lib().orc_geometric_asian_call(S0, K, r, sigma, T)


def heston_call(S0=100.0, K=100.0, r=0.05, T=1.0, kappa=2.0, theta=0.04, xi=0.3, rho=-0.7,
                v0=0.04):
    return lib().orc_heston_call(S0, K, r, T, kappa, theta, xi, rho, v0)


def euler_k0_moments(S0, r, sigma, T, l, M):
    out = np.zeros(2)
    lib().orc_euler_k0_moments(S0, r, sigma, T, l, M, _dp(out))
    return out[0], out[1]


def level0_call_moments(S0, K, r, sigma, T):
    out = np.zeros(2)
    lib().orc_level0_call_moments(S0, K, r, sigma, T, _dp(out))
    return out[0], out[1]


def cv_nparams(in_dim=2, hidden=64):
    return lib().orc_cv_nparams(in_dim, hidden)


def cv_init(in_dim=2, hidden=64, init_seed=1):
    p = np.zeros(cv_nparams(in_dim, hidden))
    lib().orc_cv_init(in_dim, hidden, init_seed, _dp(p))
    return p


def cv_inputs(m, t, S, v=0.04):
    x = np.zeros(3)
    lib().orc_cv_inputs(C.byref(m), t, S, v, _dp(x))
    return x[: (3 if m.kind == HESTON else 2)]


def cv_out_scale(m):
    return lib().orc_cv_out_scale(C.byref(m))


def cv_phi(m, cv, t, S, v=0.04):
    return lib().orc_cv_phi(C.byref(m), cv.ref(), t, S, v)


def cv_phi_grad(m, cv, t, S, v=0.04, g=1.0):
    grad = np.zeros(cv.params.size)
    lib().orc_cv_phi_grad(C.byref(m), cv.ref(), t, S, v, g, _dp(grad))
    return grad


def cv_loss_grad(m, p, M, lmax, B, seed, step, cv, nthreads=1, want_grad=True):
    grad = np.zeros(cv.params.size) if want_grad else None
    var = np.zeros(lmax + 1)
    loss = lib().orc_cv_loss_grad(C.byref(m), C.byref(p), M, lmax, B, seed, step, cv.ref(),
                                  nthreads, _dp(grad) if want_grad else None, _dp(var))
    return loss, grad, var


def adam(theta, m1, m2, g, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, t=1):
    """In-place Adam step on FP64 numpy arrays."""
    lib().orc_adam(theta.size, _dp(theta), _dp(m1), _dp(m2),
                   _dp(np.ascontiguousarray(g, dtype=np.float64)), lr, b1, b2, eps, t)


def rg_probabilities(q, Lc):
    p, F = np.zeros(Lc + 1), np.zeros(Lc + 1)
    lib().orc_rg_probabilities(q, Lc, _dp(p), _dp(F))
    return p, F


def rg_level_counts(seed, N, q, Lc):
    c = np.zeros(Lc + 1, np.uint64)
    if lib().orc_rg_level_counts(seed, N, q, Lc, c.ctypes.data_as(C.POINTER(C.c_uint64))):
        raise ValueError("orc_rg_level_counts: bad arguments")
    return c


def rhee_glynn(m, p, M, Lc, q, N, seed, nthreads=1):
    r = RGResult()
    if lib().orc_rhee_glynn(C.byref(m), C.byref(p), M, Lc, q, N, seed, nthreads, C.byref(r)):
        raise ValueError("orc_rhee_glynn: bad arguments")
    n = Lc + 1
    return {"estimate": r.estimate, "variance": r.variance, "cost": r.cost, "Lc": r.Lc,
            "N": list(r.N)[:n], "p": list(r.p)[:n], "sum_y": list(r.sum_y)[:n],
            "sum_y2": list(r.sum_y2)[:n], "n_nonfinite": r.n_nonfinite}
