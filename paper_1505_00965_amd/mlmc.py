"""Python binding of libmlmc.so (argument marshalling only).

Every computation runs in the library's HIP kernels.  PyTorch supplies device
memory (tensors passed as d_* pointers) and streams.  If the shared library
is missing or fails to load, every call raises: there is no fallback.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlmc.so")

MLMC_OK, MLMC_ENOTCONV, MLMC_EINVAL, MLMC_ENOMEM, MLMC_EDEVICE, MLMC_ENONFINITE = 0, 1, -1, -2, -3, -4
GBM, HESTON = 0, 1
EULER, MILSTEIN = 0, 1
CALL, ASIAN, LOOKBACK, DIGITAL, DIGITAL_COND = 0, 1, 2, 3, 4
STREAM_NORMAL, STREAM_BRIDGE, STREAM_TRAIN_NORMAL = 0, 1, 2
MAX_LEVELS = 16

EXPORTED = [
    "mlmc_ctx_create", "mlmc_ctx_destroy", "mlmc_set_stream", "mlmc_last_error",
    "mlmc_set_launch", "mlmc_level", "mlmc_level_paths", "mlmc_philox_words", "mlmc_normals",
    "mlmc_stdmc", "mlmc_optimal_n", "mlmc_run", "mlmc_set_timing", "mlmc_kernel_stats",
    "mlmc_levels_batch", "mlmc_set_persistent_launch",
    "mlmc_cv_create", "mlmc_cv_destroy", "mlmc_cv_nparams", "mlmc_cv_get_params",
    "mlmc_cv_set_params", "mlmc_cv_loss_grad", "mlmc_cv_train", "mlmc_autotune",
    "mlmc_autotune_persistent",
    "mlmc_tuned_shape", "mlmc_rhee_glynn", "mlmc_set_timing_mask", "mlmc_level_noalloc",
    "mlmc_cv_set_tabulated", "mlmc_cv_get_table", "mlmc_set_timing_stride", "mlmc_autotune_run",
    "mlmc_set_timing_paused",
]
STAT_SLOTS = 20
STAT_PERSISTENT, STAT_DRIVER, STAT_CV_TRAIN = 16, 17, 18


class MLMCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mlmc status {status}: {msg}")
        self.status = status


class Model(C.Structure):
    _fields_ = [("kind", C.c_int), ("S0", C.c_double), ("r", C.c_double),
                ("sigma", C.c_double), ("T", C.c_double), ("kappa", C.c_double),
                ("theta", C.c_double), ("xi", C.c_double), ("rho", C.c_double),
                ("v0", C.c_double), ("scheme", C.c_int), ("antithetic", C.c_int)]


class Payoff(C.Structure):
    _fields_ = [("kind", C.c_int), ("K", C.c_double), ("payout", C.c_double)]


class LevelResult(C.Structure):
    _fields_ = [("sum_y", C.c_double), ("sum_y2", C.c_double), ("sum_pf", C.c_double),
                ("sum_pf2", C.c_double), ("sum_pc", C.c_double), ("sum_pc2", C.c_double),
                ("cost", C.c_double), ("n", C.c_uint64), ("n_nonfinite", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelStat(C.Structure):
    _fields_ = [("launches", C.c_uint64), ("ms", C.c_double), ("fine_steps", C.c_double),
                ("coarse_steps", C.c_double)]


class RunOpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("M", C.c_int), ("L_min", C.c_int), ("L_max", C.c_int),
                ("n_pilot", C.c_uint64), ("seed", C.c_uint64), ("precision", C.c_int),
                ("persistent", C.c_int), ("alpha", C.c_double), ("beta", C.c_double),
                ("cv", C.c_void_p), ("cv_levels", C.c_int)]


class RGResult(C.Structure):
    _fields_ = [("estimate", C.c_double), ("variance", C.c_double), ("rmse_est", C.c_double),
                ("cost", C.c_double), ("wall_s", C.c_double), ("L_cap", C.c_int),
                ("N", C.c_uint64 * MAX_LEVELS), ("p", C.c_double * MAX_LEVELS),
                ("sum_y", C.c_double * MAX_LEVELS), ("sum_y2", C.c_double * MAX_LEVELS),
                ("n_nonfinite", C.c_uint64)]


class RunResult(C.Structure):
    L16 = MAX_LEVELS
    _fields_ = [("estimate", C.c_double), ("rmse_est", C.c_double), ("wall_s", C.c_double),
                ("L", C.c_int), ("converged", C.c_int), ("iterations", C.c_int),
                ("N", C.c_uint64 * L16), ("E", C.c_double * L16), ("V", C.c_double * L16),
                ("C", C.c_double * L16), ("sum_y", C.c_double * L16),
                ("sum_y2", C.c_double * L16), ("alpha", C.c_double), ("beta", C.c_double),
                ("gamma", C.c_double), ("cost", C.c_double), ("n_nonfinite", C.c_uint64)]

    def as_dict(self):
        n = self.L + 1
        # slicing a ctypes array yields a list of Python numbers
        return {"estimate": self.estimate, "rmse_est": self.rmse_est, "wall_s": self.wall_s,
                "L": self.L, "converged": bool(self.converged), "iterations": self.iterations,
                "alpha": self.alpha, "beta": self.beta, "gamma": self.gamma, "cost": self.cost,
                "n_nonfinite": self.n_nonfinite, "N": self.N[:n], "E": self.E[:n],
                "V": self.V[:n], "C": self.C[:n], "sum_y": self.sum_y[:n],
                "sum_y2": self.sum_y2[:n]}


_lib = None


def lib():
    """Load libmlmc.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # PyTorch ships its own HIP runtime under the same soname as the system
    # one.  Loading torch first makes the library bind to that copy, so the
    # process has one HIP runtime and torch's device pointers and stream
    # handles are valid in the library; loaded the other way round the two
    # runtimes coexist and torch no longer sees the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, u64, i32, d, u32 = C.c_void_p, C.c_uint64, C.c_int, C.c_double, C.c_uint32
    M_, P_ = C.POINTER(Model), C.POINTER(Payoff)
    L.mlmc_ctx_create.argtypes = [i32, C.POINTER(vp)]
    L.mlmc_ctx_destroy.argtypes = [vp]
    L.mlmc_set_stream.argtypes = [vp, vp]
    L.mlmc_last_error.argtypes = [vp]
    L.mlmc_last_error.restype = C.c_char_p
    L.mlmc_set_launch.argtypes = [vp, i32, i32]
    L.mlmc_level.argtypes = [vp, M_, P_, i32, i32, u64, u64, u64, i32, vp, C.POINTER(LevelResult)]
    L.mlmc_level_paths.argtypes = [vp, M_, P_, i32, i32, u64, u64, u64, i32, vp, vp, vp,
                                   C.POINTER(LevelResult)]
    L.mlmc_philox_words.argtypes = [vp, u64, i32, u64, u32, u32, u64, vp]
    L.mlmc_normals.argtypes = [vp, u64, i32, u64, u32, i32, i32, u64, i32, vp]
    L.mlmc_stdmc.argtypes = [vp, M_, P_, i32, i32, u64, u64, u64, i32, C.POINTER(LevelResult)]
    L.mlmc_rhee_glynn.argtypes = [vp, M_, P_, i32, i32, d, u64, u64, i32, C.POINTER(RGResult)]
    L.mlmc_optimal_n.argtypes = [vp, i32, C.POINTER(d), C.POINTER(d), d, C.POINTER(d)]
    L.mlmc_run.argtypes = [vp, M_, P_, C.POINTER(RunOpts), C.POINTER(RunResult)]
    L.mlmc_levels_batch.argtypes = [vp, M_, P_, i32, i32, i32, C.POINTER(u64), C.POINTER(u64),
                                    u64, C.POINTER(LevelResult)]
    L.mlmc_set_persistent_launch.argtypes = [vp, i32, i32, i32]
    L.mlmc_cv_create.argtypes = [vp, i32, i32, u64, C.POINTER(vp)]
    L.mlmc_cv_destroy.argtypes = [vp]
    L.mlmc_cv_nparams.argtypes = [vp]
    L.mlmc_cv_get_params.argtypes = [vp, C.POINTER(C.c_float), C.c_size_t]
    L.mlmc_cv_set_params.argtypes = [vp, C.POINTER(C.c_float), C.c_size_t]
    L.mlmc_cv_loss_grad.argtypes = [vp, M_, P_, i32, i32, u64, u64, u64, C.POINTER(C.c_float),
                                    C.POINTER(d), C.POINTER(d)]
    L.mlmc_cv_train.argtypes = [vp, M_, P_, i32, i32, i32, u64, d, u64, C.POINTER(C.c_float)]
    L.mlmc_cv_set_tabulated.argtypes = [vp, i32]
    L.mlmc_cv_get_table.argtypes = [vp, M_, C.POINTER(C.c_float), C.c_size_t, C.POINTER(i32)]
    L.mlmc_autotune.argtypes = [vp, M_, P_, i32, i32, C.c_char_p]
    L.mlmc_autotune_persistent.argtypes = [vp, M_, P_, i32, i32, i32, C.c_char_p,
                                           C.POINTER(C.c_int)]
    L.mlmc_tuned_shape.argtypes = [vp, M_, P_, i32, i32, i32, C.POINTER(i32), C.POINTER(i32)]
    L.mlmc_set_timing.argtypes = [vp, i32]
    L.mlmc_set_timing_mask.argtypes = [vp, u32]
    L.mlmc_set_timing_stride.argtypes = [vp, u32]
    L.mlmc_set_timing_paused.argtypes = [vp, i32]
    L.mlmc_autotune_run.argtypes = [vp, M_, P_, C.POINTER(RunOpts), C.c_char_p, C.POINTER(i32)]
    L.mlmc_kernel_stats.argtypes = [vp, C.POINTER(KernelStat)]
    L.mlmc_level_noalloc.argtypes = [M_, P_, i32, i32, u64, u64, u64, i32, vp, vp, C.c_char_p,
                                     C.c_size_t]
    for name in EXPORTED:
        if name != "mlmc_last_error":
            getattr(L, name).restype = i32
    L.mlmc_cv_nparams.restype = C.c_size_t
    _lib = L
    return L


def model(kind=GBM, S0=100.0, r=0.05, sigma=0.2, T=1.0, kappa=2.0, theta=0.04, xi=0.3,
          rho=-0.7, v0=0.04, scheme=0, antithetic=0):
    return Model(kind, S0, r, sigma, T, kappa, theta, xi, rho, v0, scheme, antithetic)


def payoff(kind=CALL, K=100.0, payout=1.0):
    return Payoff(kind, K, payout)


def _ptr(t):
    """Device pointer of a torch tensor (or an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def mlmc_level_noalloc(m, p, l, M, N, seed, d_out, path_offset=0, precision=32, stream=None):
    """mlmc_level's sums with no context and no allocation, enqueued on
    `stream` (a torch stream or raw handle; None = the null stream) of the
    current device; d_out: a device tensor of at least 72 bytes (e.g. 9
    float64) that receives the mlmc_level_result.  Does not synchronise."""
    L = lib()
    h = None if stream is None else getattr(stream, "cuda_stream", stream)
    err = C.create_string_buffer(256)
    st = L.mlmc_level_noalloc(C.byref(m), C.byref(p), l, M, N, seed, path_offset, precision, h,
                              _ptr(d_out), err, len(err))
    if st != MLMC_OK:
        raise MLMCError(st, err.value.decode())


def level_result_from(t):
    """Decode the 72-byte mlmc_level_result held in a device tensor."""
    raw = t.detach().cpu().contiguous().view(-1).numpy().tobytes()[:C.sizeof(LevelResult)]
    r = LevelResult.from_buffer_copy(raw)
    return r.as_dict()


class Context:
    """Owns an mlmc_ctx on one device; methods mirror the C entry points."""

    def __init__(self, device=0):
        self._lib = lib()
        h = C.c_void_p()
        st = self._lib.mlmc_ctx_create(device, C.byref(h))
        if st != MLMC_OK:
            raise MLMCError(st, f"mlmc_ctx_create(device={device}) failed")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            self._lib.mlmc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st, allow=(MLMC_OK,)):
        if st not in allow:
            raise MLMCError(st, self._lib.mlmc_last_error(self.h).decode())
        return st

    def last_error(self):
        return self._lib.mlmc_last_error(self.h).decode()

    def set_stream(self, stream):
        """stream: a torch.cuda.Stream, a raw hipStream_t int, or None."""
        raw = None if stream is None else getattr(stream, "cuda_stream", stream)
        self._check(self._lib.mlmc_set_stream(self.h, raw))

    def set_timing(self, on=True):
        self._check(self._lib.mlmc_set_timing(self.h, int(on)))

    def set_timing_slots(self, slots):
        """Time only the given statistics slots (levels 0..15, STAT_*)."""
        mask = 0
        for s in slots:
            mask |= 1 << int(s)
        self._check(self._lib.mlmc_set_timing_mask(self.h, mask))

    def set_timing_stride(self, stride=1):
        """Time one launch in `stride` of each timed slot."""
        self._check(self._lib.mlmc_set_timing_stride(self.h, int(stride)))

    def set_timing_paused(self, paused=True):
        """Stamp nothing while paused (mask, stride count and statistics kept)."""
        self._check(self._lib.mlmc_set_timing_paused(self.h, int(bool(paused))))

    def kernel_stats(self):
        """Per-slot {launches, ms, fine_steps, coarse_steps} (slots 0..15 = level)."""
        arr = (KernelStat * STAT_SLOTS)()
        self._check(self._lib.mlmc_kernel_stats(self.h, arr))
        return [{k: getattr(a, k) for k, _ in KernelStat._fields_} for a in arr]

    def autotune(self, m, p, M=4, precision=32, cache_path=None):
        self._check(self._lib.mlmc_autotune(self.h, C.byref(m), C.byref(p), M, precision,
                                            cache_path.encode() if cache_path else None))

    def autotune_persistent(self, m, payoffs, M=4, L=8, cache_path=None):
        """Tune the persistent form's launch shape; returns (block, ppt, blocks_per_cu)."""
        npay = len(payoffs)
        P = (Payoff * npay)(*payoffs)
        shape = (C.c_int * 3)()
        self._check(self._lib.mlmc_autotune_persistent(
            self.h, C.byref(m), P, npay, M, L, cache_path.encode() if cache_path else None, shape))
        return tuple(shape)

    def autotune_run(self, m, p, eps, M=4, L_min=2, L_max=8, n_pilot=10000, seed=1, precision=32,
                     alpha=0.0, beta=0.0, cache_path=None):
        """Tune the device-planned run's launch shape on this run configuration;
        returns (block, ppt, blocks_per_cu)."""
        o = RunOpts(eps, M, L_min, L_max, n_pilot, seed, precision, 1, alpha, beta, None, 0)
        shape = (C.c_int * 3)()
        self._check(self._lib.mlmc_autotune_run(
            self.h, C.byref(m), C.byref(p), C.byref(o),
            cache_path.encode() if cache_path else None, shape))
        return tuple(shape)

    def tuned_shape(self, m, p, l, M=4, precision=32):
        b, q = C.c_int(), C.c_int()
        self._check(self._lib.mlmc_tuned_shape(self.h, C.byref(m), C.byref(p), l, M, precision,
                                               C.byref(b), C.byref(q)))
        return b.value, q.value

    def set_launch(self, block=0, ppt=0):
        self._check(self._lib.mlmc_set_launch(self.h, block, ppt))

    def mlmc_level(self, m, p, l, M, N, seed, path_offset=0, precision=32, cv=None,
                   allow_nonfinite=False):
        r = LevelResult()
        allow = (MLMC_OK, MLMC_ENONFINITE) if allow_nonfinite else (MLMC_OK,)
        self._check(self._lib.mlmc_level(self.h, C.byref(m), C.byref(p), l, M, N, seed,
                                         path_offset, precision, _cvh(cv), C.byref(r)), allow)
        return r.as_dict()

    def mlmc_level_paths(self, m, p, l, M, N, seed, d_pf, d_pc, path_offset=0, precision=32,
                         cv=None, allow_nonfinite=False):
        r = LevelResult()
        allow = (MLMC_OK, MLMC_ENONFINITE) if allow_nonfinite else (MLMC_OK,)
        self._check(self._lib.mlmc_level_paths(self.h, C.byref(m), C.byref(p), l, M, N, seed,
                                               path_offset, precision, _cvh(cv), _ptr(d_pf),
                                               _ptr(d_pc), C.byref(r)), allow)
        return r.as_dict()

    def mlmc_philox_words(self, seed, level, s0, stream, nblocks, npaths, d_out):
        self._check(self._lib.mlmc_philox_words(self.h, seed, level, s0, stream, nblocks, npaths,
                                                _ptr(d_out)))

    def mlmc_normals(self, seed, level, s0, stream, dim, nsteps, npaths, precision, d_out):
        self._check(self._lib.mlmc_normals(self.h, seed, level, s0, stream, dim, nsteps, npaths,
                                           precision, _ptr(d_out)))

    def mlmc_rhee_glynn(self, m, p, M, L_cap, q, N, seed, precision=32):
        r = RGResult()
        self._check(self._lib.mlmc_rhee_glynn(self.h, C.byref(m), C.byref(p), M, L_cap, q, N, seed,
                                              precision, C.byref(r)))
        n = L_cap + 1
        return {"estimate": r.estimate, "variance": r.variance, "rmse_est": r.rmse_est,
                "cost": r.cost, "wall_s": r.wall_s, "L_cap": r.L_cap, "N": list(r.N)[:n],
                "p": list(r.p)[:n], "sum_y": list(r.sum_y)[:n], "sum_y2": list(r.sum_y2)[:n],
                "n_nonfinite": r.n_nonfinite}

    def mlmc_stdmc(self, m, p, L, M, N, seed, path_offset=0, precision=32):
        r = LevelResult()
        self._check(self._lib.mlmc_stdmc(self.h, C.byref(m), C.byref(p), L, M, N, seed,
                                         path_offset, precision, C.byref(r)))
        return r.as_dict()

    def mlmc_levels_batch(self, m, payoffs, M, L, N, seed, offsets=None, allow_nonfinite=False):
        """payoffs: list of Payoff; N[k][l]; returns results[k][l] dicts."""
        npay = len(payoffs)
        P = (Payoff * npay)(*payoffs)
        flat = [int(N[k][l]) for k in range(npay) for l in range(L + 1)]
        Na = (C.c_uint64 * len(flat))(*flat)
        Oa = None
        if offsets is not None:
            of = [int(offsets[k][l]) for k in range(npay) for l in range(L + 1)]
            Oa = (C.c_uint64 * len(of))(*of)
        R = (LevelResult * len(flat))()
        allow = (MLMC_OK, MLMC_ENONFINITE) if allow_nonfinite else (MLMC_OK,)
        self._check(self._lib.mlmc_levels_batch(self.h, C.byref(m), P, npay, M, L, Na, Oa, seed, R),
                    allow)
        return [[R[k * (L + 1) + l].as_dict() for l in range(L + 1)] for k in range(npay)]

    def set_persistent_launch(self, block=0, ppt=0, blocks_per_cu=0):
        self._check(self._lib.mlmc_set_persistent_launch(self.h, block, ppt, blocks_per_cu))

    def mlmc_optimal_n(self, V, Cl, eps):
        L = len(V) - 1
        Va = (C.c_double * (L + 1))(*V)
        Ca = (C.c_double * (L + 1))(*Cl)
        Na = (C.c_double * (L + 1))()
        self._check(self._lib.mlmc_optimal_n(self.h, L, Va, Ca, eps, Na))
        return list(Na)

    def mlmc_run(self, m, p, eps, M=4, L_min=2, L_max=8, n_pilot=10000, seed=1, precision=32,
                 persistent=False, alpha=0.0, beta=0.0, cv=None, cv_levels=0,
                 allow_notconv=False):
        o = RunOpts(eps, M, L_min, L_max, n_pilot, seed, precision, int(persistent), alpha, beta,
                    _cvh(cv), cv_levels)
        r = RunResult()
        allow = (MLMC_OK, MLMC_ENOTCONV) if allow_notconv else (MLMC_OK,)
        self._check(self._lib.mlmc_run(self.h, C.byref(m), C.byref(p), C.byref(o), C.byref(r)),
                    allow)
        return r.as_dict()


def _cvh(cv):
    if cv is None:
        return None
    return cv.h


class ControlVariate:
    """An mlmc_cv network on a Context (parameters live on the device)."""

    def __init__(self, ctx, in_dim=2, hidden=64, init_seed=1):
        self.ctx = ctx
        self._lib = ctx._lib
        h = C.c_void_p()
        ctx._check(self._lib.mlmc_cv_create(ctx.h, in_dim, hidden, init_seed, C.byref(h)))
        self.h = h
        self.in_dim = in_dim

    def close(self):
        if self.h:
            self._lib.mlmc_cv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nparams(self):
        return int(self._lib.mlmc_cv_nparams(self.h))

    def get_params(self):
        import numpy as np
        out = np.zeros(self.nparams, dtype=np.float32)
        self.ctx._check(self._lib.mlmc_cv_get_params(
            self.h, out.ctypes.data_as(C.POINTER(C.c_float)), out.size))
        return out

    def loss_grad(self, m, p, M, lmax, batch, seed, step):
        """(loss, grad[nparams] float32, var[lmax+1]) of one training batch."""
        import numpy as np
        g = np.zeros(self.nparams, dtype=np.float32)
        var = (C.c_double * (lmax + 1))()
        loss = C.c_double()
        self.ctx._check(self._lib.mlmc_cv_loss_grad(
            self.h, C.byref(m), C.byref(p), M, lmax, batch, seed, step,
            g.ctypes.data_as(C.POINTER(C.c_float)), var, C.byref(loss)))
        return loss.value, g, list(var)

    def train(self, m, p, M=4, lmax=3, steps=2000, batch=16384, lr=1e-3, seed=1):
        """Adam training on the device; returns the loss history (float32)."""
        import numpy as np
        hist = np.zeros(max(steps, 1), dtype=np.float32)
        self.ctx._check(self._lib.mlmc_cv_train(
            self.h, C.byref(m), C.byref(p), M, lmax, steps, batch, lr, seed,
            hist.ctypes.data_as(C.POINTER(C.c_float))))
        return hist[:steps]

    def set_tabulated(self, on=True):
        """Estimation samplers read phi from its table (True) or evaluate the
        network (False)."""
        self.ctx._check(self._lib.mlmc_cv_set_tabulated(self.h, int(bool(on))))

    def get_table(self, m):
        """The table of the tabulated form for model m: array [R, nv, ns]."""
        import numpy as np
        dims = (C.c_int * 3)()
        self.ctx._check(self._lib.mlmc_cv_get_table(self.h, C.byref(m), None, 0, dims))
        out = np.zeros(dims[0] * dims[1] * dims[2], dtype=np.float32)
        self.ctx._check(self._lib.mlmc_cv_get_table(
            self.h, C.byref(m), out.ctypes.data_as(C.POINTER(C.c_float)), out.size, dims))
        return out.reshape(dims[0], dims[1], dims[2])

    def set_params(self, values):
        import numpy as np
        v = np.ascontiguousarray(values, dtype=np.float32)
        self.ctx._check(self._lib.mlmc_cv_set_params(
            self.h, v.ctypes.data_as(C.POINTER(C.c_float)), v.size))
