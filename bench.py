"""Benchmark: adaptive MLMC on one MI355X, fine path-steps per second.

One step = one complete adaptive MLMC estimate (every level sampled by the
HIP level sampler, the fp64 driver update on the device) of the GBM European
call (S0=100, r=0.05, sigma=0.2, T=1, K=100), M=4, fp32 paths with fp64 sums,
one level per launch.  The target RMSE defaults to 2e-5*S0: with it the driver
reaches about 10^8 samples at level 0, the scale that workload is described
at (its listed RMSEs of 2e-3..5e-4*S0 need only 1.4e4..2.2e5 there).

value = fine path steps computed by all steps / wall time of the K timed
steps.  The JSON line also carries the roofline of the dominant kernel, timed
with HIP events on the launch stream, the CPU oracle timed on a bounded sample
of the same workload, and seconds to RMSE 1e-3*S0.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "seconds to RMSE 1e-3·S0 (learned-CV vs plain MLMC); fine path-steps/s"
UNIT = "fine path-steps/s"

# Algorithmic vector-ALU operations of the GBM call sampler, M = 4: per fine
# step, a quarter Philox4x32-10 call (10 rounds of 2 32x32->64 products and 2
# three-input xors: 10), half a Box-Muller pair with sqrt(h) folded into its
# radius (6.5), the Euler step (2 fma), coarse increment sum and a quarter
# coarse step (1.5); per sample, payoffs and fp64 sums.
OPS_PER_FINE_STEP = 20.0
# level 0: the one step plus payoff (3) and Y, Y^2 sums (3) is the method's
# count, 24.5; the fp32 call kernel folds the step and the strike into one fma
# and executes 22.5 of them.  The roofline counts what the kernel executes.
OPS_PER_SAMPLE_L0_METHOD = 24.5
OPS_PER_SAMPLE_L0 = 22.5
OPS_PER_SAMPLE = 11.0         # levels >= 1: two payoffs, difference, sums
FP32_PEAK_FLOPS = 157.3e12    # MI355X fp32 vector peak (an fma counts 2, packed fp32 2x)


def algorithmic_ops(level, fine_steps, samples):
    if level == 0:
        return OPS_PER_SAMPLE_L0 * samples
    return OPS_PER_FINE_STEP * fine_steps + OPS_PER_SAMPLE * samples
# MI355X vector ALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9


def profile_field(kernel_label, field):
    """A figure from the committed rocprofv3 summaries (profiles/*.md) of this
    kernel, or None if the kernel sources changed since they were taken."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in ("philox.hpp", "sampler.hpp", "sampler_impl.hpp", "reduce.hpp", "level.hip",
              "level.hpp", "level_kernels.hpp", "level_gbm.hip", "../build.py"):
        with open(os.path.join(ROOT, "paper_1505_00965_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    digest = h.hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        fields = {}
        for line in open(path):
            if ":" in line and not line.startswith(("|", "#", "-", " ")):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        if (fields.get("kernel") == kernel_label and fields.get("kernel_sources_sha256") == digest
                and field in fields):
            return float(fields[field])
    return None


def measured_traffic(kernel_label):
    """HBM bytes per launch (FETCH_SIZE/WRITE_SIZE summary)."""
    return profile_field(kernel_label, "traffic_bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--eps", type=float, default=2e-5, help="target RMSE in units of S0")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU work for the oracle baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tta", action="store_true", help="skip seconds-to-RMSE runs")
    ap.add_argument("--cv-steps", type=int, default=2000,
                    help="Adam steps for the control-variate networks (0: plain only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 256 MiB device copy first (scales HBM byte counters)")
    ap.add_argument("--persistent", type=int, default=0,
                    help="1: each driver iteration is one graph launch of the persistent kernel")
    # kernel profiling mode (for rocprofv3 counter runs): only repeated
    # launches of one level's sampler, with the tuned shape, then one JSON line
    ap.add_argument("--profile-level", type=int, default=None,
                    help="profile mode: time only mlmc_level launches at this level (M=4)")
    ap.add_argument("--profile-samples", type=float, default=0,
                    help="samples per profiled launch (0: the adaptive run's N_l at RMSE 2e-5*S0)")
    ap.add_argument("--profile-launches", type=int, default=5)
    ap.add_argument("--profile-model", choices=("gbm", "heston"), default="gbm")
    ap.add_argument("--profile-payoff", choices=("call", "asian", "lookback", "digital"),
                    default="call")
    ap.add_argument("--profile-cv", action="store_true",
                    help="profile the control-variate sampler (and one training gradient per "
                         "launch) with a network trained for 50 steps")
    ap.add_argument("--profile-cv-tab", action="store_true",
                    help="with --profile-cv: the tabulated network in the sampler")
    return ap.parse_args()


# samples per level of the adaptive run at RMSE 2e-5*S0 (seed 1)
ADAPTIVE_N = [200141355, 14852584, 3713146, 928287, 232072]


def profile_mode(args):
    """Launch one level's sampler `launches` times (the last launches of the
    run are these: counter runs take them by kernel name from the end)."""
    import torch
    from paper_1505_00965_amd import mlmc, workloads as W
    ctx = mlmc.Context(0)
    ctx.set_stream(torch.cuda.current_stream())
    md = W.GBM_MODEL if args.profile_model == "gbm" else W.HESTON_MODEL
    m, p = mlmc.model(**md), mlmc.payoff(**W.PAYOFFS[args.profile_payoff])
    l, M = args.profile_level, 4
    N = int(args.profile_samples) or (ADAPTIVE_N[l] if l < len(ADAPTIVE_N) else 1 << 16)
    cv = None
    if args.profile_cv:
        cv = mlmc.ControlVariate(ctx, 3 if args.profile_model == "heston" else 2, init_seed=1)
        cv.train(m, p, M=M, lmax=3, steps=50, batch=16384, lr=1e-3, seed=2)
        cv.set_tabulated(args.profile_cv_tab)
    else:
        ctx.autotune(m, p, M=M, precision=32)
    torch.cuda.synchronize()
    ctx.set_timing_slots([l])
    t0 = time.perf_counter()
    for r in range(args.profile_launches):
        ctx.mlmc_level(m, p, l, M, N, 1 + r, cv=cv)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.kernel_stats()[l]
    ctx.set_timing(False)
    grads = 0
    if cv is not None:
        for r in range(args.profile_launches):
            cv.loss_grad(m, p, M, 3, 16384, 7, r)
            grads += 1
        torch.cuda.synchronize()
    nf = M**l
    out = {"mode": "profile", "model": args.profile_model, "payoff": args.profile_payoff,
           "level": l, "M": M, "samples_per_launch": N, "launches": args.profile_launches,
           "fine_steps_per_launch": N * nf, "avg_launch_ms": st["ms"] / max(st["launches"], 1),
           "wall_s": wall, "cv": bool(cv), "cv_gradients": grads,
           "tuned_shape": None if cv else ctx.tuned_shape(m, p, l, M=M)}
    if cv is not None:
        cv.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def fine_steps_of(res, M):
    return float(sum(n * M**l for l, n in enumerate(res["N"])))


def host_info():
    """Host cores and CPU model of the machine the oracle runs on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    affinity = len(os.sched_getaffinity(0))
    # the host share of one GPU: the box sets OMP_NUM_THREADS to it (16)
    share = int(os.environ.get("OMP_NUM_THREADS") or affinity)
    return {"nproc": os.cpu_count(), "affinity": affinity, "threads": max(1, min(affinity, share)),
            "cpu_model": model}


def oracle_rate(oracle, om, op, N, M, threads, budget_s):
    """Fine path-steps/s of the oracle on passes over levels 0..L with counts
    N_l (scaled down when a pass does not fit), run until the budget is used.

    One untimed call first (thread start-up, first touch), then a probe: a
    pass over the same levels at a small scale, grown until it takes >= 0.2 s
    (the levels' per-sample costs differ, so the probe has the run's mix); its
    rate sizes the first pass, the rate measured so far every later one."""
    costs = [M**l + (M ** (l - 1) if l else 0) for l in range(len(N))]
    total = sum(n * c for n, c in zip(N, costs))
    oracle.level(om, op, 1, M, 1000, 97, nthreads=threads)
    scale = min(1.0, 2e5 / total)
    while True:
        t0 = time.perf_counter()
        steps = 0.0
        for l, nl in enumerate(N):
            nn = max(1, int(nl * scale))
            oracle.level(om, op, l, M, nn, 98, nthreads=threads)
            steps += nn * costs[l]
        dt = time.perf_counter() - t0
        if dt >= 0.2 or scale >= 1.0:
            break
        scale = min(1.0, scale * min(10.0, max(2.0, 0.25 / max(dt, 1e-6))))
    rate = steps / dt
    fine = steps = 0.0
    passes, scales = 0, []
    t0 = time.perf_counter()
    while passes < 1000:
        left = budget_s - (time.perf_counter() - t0)
        if left <= 0.05 * budget_s:
            break
        scale = min(1.0, left * rate / total)
        for l, nl in enumerate(N):
            nn = max(1, int(nl * scale))
            oracle.level(om, op, l, M, nn, 1 + passes, nthreads=threads)
            fine += nn * M**l
            steps += nn * costs[l]
        passes += 1
        scales.append(scale)
        rate = steps / (time.perf_counter() - t0)
    dt = time.perf_counter() - t0
    return {"fine_steps_per_s": fine / dt, "fine_steps": fine, "seconds": dt, "passes": passes,
            "scales": [round(x, 4) for x in scales[:3]] + (["..."] if len(scales) > 3 else [])}


def cpu_baseline(ref_run, M, budget_s):
    """The oracle, as it stands, on a bounded sample of the same levels: on
    the host threads one GPU gets and on one thread."""
    import oracle
    from paper_1505_00965_amd import workloads as W
    om, op = oracle.model(**W.GBM_MODEL), oracle.payoff(**W.CALL)
    info = host_info()
    N = list(ref_run["N"])
    many = oracle_rate(oracle, om, op, N, M, info["threads"], 0.7 * budget_s)
    one = oracle_rate(oracle, om, op, N, M, 1, 0.3 * budget_s)
    return {"value": many["fine_steps_per_s"], "unit": UNIT, "cores": info["threads"],
            "kind": "oracle",
            "sample": (f"levels 0..{len(N) - 1} of one adaptive run (its N_l, scaled to the time "
                       f"budget), {many['passes']} pass(es), {many['fine_steps']:.3g} fine path "
                       f"steps in {many['seconds']:.1f} s, fp64"),
            "single_thread": {"value": one["fine_steps_per_s"], "passes": one["passes"],
                              "fine_steps": one["fine_steps"], "seconds": one["seconds"]},
            "scales": many["scales"], "nproc": info["nproc"], "affinity": info["affinity"],
            "cpu_model": info["cpu_model"]}


def reference_prices():
    """Continuous-time prices the accuracy runs are measured against
    (tests/golden/prices.json, written from the oracle's closed forms)."""
    with open(os.path.join(ROOT, "tests", "golden", "prices.json")) as f:
        return {k: v["value"] for k, v in json.load(f).items()}


def seeds_runs(ctx, m, p, eps, M, cv, seeds, exact, cv_levels=0):
    """Runs over the seeds: median wall seconds, empirical RMSE against the
    continuous price, and the median run."""
    import statistics
    runs = [ctx.mlmc_run(m, p, eps, M=M, seed=s, precision=32, cv=cv, cv_levels=cv_levels)
            for s in seeds]
    rmse = (sum((r["estimate"] - exact) ** 2 for r in runs) / len(runs)) ** 0.5
    mid = sorted(runs, key=lambda r: r["wall_s"])[len(runs) // 2]
    return statistics.median(r["wall_s"] for r in runs), rmse, mid


def time_to_accuracy(ctx, mlmc, W, args, seeds=range(1, 33)):
    """Seconds to RMSE eps, plain MLMC vs the learned control variate, for
    the GBM arithmetic Asian and the Heston call, eps in {1e-3, 5e-4} S0,
    32 seeds each; the empirical RMSE of the estimates against the
    continuous-time price is reported beside the median time.

    The network is trained once per model (Adam, lr 1e-3, batch 16384 samples
    per level on levels 0..3, i.e. 65536 per step) on the training streams.
    A trained network is reused across estimates, so the estimation times
    exclude training; `with_training_s` adds it to one estimate.
    """
    import torch
    ref = reference_prices()
    out = {}
    cases = (("gbm_asian", W.GBM_MODEL, W.ASIAN, 2, ref["gbm_asian"]),
             ("heston_call", W.HESTON_MODEL, W.CALL, 3, ref["heston_call"]))
    for name, md, pd, d, exact in cases:
        m, p = mlmc.model(**md), mlmc.payoff(**pd)
        entry = {"reference_price": exact, "seeds": len(seeds)}
        cv = None
        if args.cv_steps > 0:
            cv = mlmc.ControlVariate(ctx, d, init_seed=1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hist = cv.train(m, p, M=4, lmax=3, steps=args.cv_steps, batch=16384, lr=1e-3, seed=2)
            torch.cuda.synchronize()
            entry["train_s"] = time.perf_counter() - t0
            entry["train_steps"] = args.cv_steps
            entry["loss_first_last"] = [float(hist[0]), float(hist[-1])]
        for eps in (1e-3, 5e-4):
            key = f"eps_{eps:g}_S0"
            tp, ep, rp = seeds_runs(ctx, m, p, eps * W.S0, 4, None, seeds, exact)
            e = {"target_rmse": eps * W.S0, "plain_s": tp, "plain_rmse": ep, "plain_cost": rp["cost"],
                 "plain_N": rp["N"], "plain_V": [round(v, 6) for v in rp["V"]]}
            if cv is not None:
                tc, ec, rc = seeds_runs(ctx, m, p, eps * W.S0, 4, cv, seeds, exact)
                e.update({"cv_s": tc, "cv_rmse": ec, "cv_cost": rc["cost"], "cv_N": rc["N"],
                          "cv_V": [round(v, 6) for v in rc["V"]], "speedup": tp / tc,
                          "cv_with_training_s": tc + entry["train_s"]})
                # the network on level 0 only: one evaluation per launch
                t0, e0, r0 = seeds_runs(ctx, m, p, eps * W.S0, 4, cv, seeds, exact, cv_levels=1)
                e.update({"cv_level0_s": t0, "cv_level0_rmse": e0, "cv_level0_cost": r0["cost"],
                          "cv_level0_N": r0["N"], "speedup_level0": tp / t0,
                          "cv_level0_with_training_s": t0 + entry["train_s"]})
                # the tabulated network on every level (built once per
                # parameter change, interpolated by the samplers)
                cv.set_tabulated(True)
                tt, et, rt = seeds_runs(ctx, m, p, eps * W.S0, 4, cv, seeds, exact)
                cv.set_tabulated(False)
                e.update({"cv_tab_s": tt, "cv_tab_rmse": et, "cv_tab_cost": rt["cost"],
                          "cv_tab_N": rt["N"], "cv_tab_V": [round(v, 6) for v in rt["V"]],
                          "speedup_tab": tp / tt, "cv_tab_with_training_s": tt + entry["train_s"]})
            entry[key] = e
        if cv is not None:
            cv.close()
        out[name] = entry
    return out


def persistent_batch(ctx, mlmc, W, reps=3):
    """All levels 0..8 of four payoffs (N_l = 2^26 4^-l) in one graph-replayed
    persistent launch with the autotuned shape (and the default one), against
    the sum of the 36 per-level launches."""
    import torch
    gm = mlmc.model(**W.GBM_MODEL)
    names = ("call", "asian", "lookback", "digital")
    pays = [mlmc.payoff(**W.PAYOFFS[n]) for n in names]
    L = 8
    N = [[W.persistent_n(l) for l in range(L + 1)] for _ in pays]
    fine = sum(N[0][l] * 4**l for l in range(L + 1)) * len(pays)

    def time_batch():
        ctx.mlmc_levels_batch(gm, pays, 4, L, N, seed=1)          # capture + warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(reps):
            ctx.mlmc_levels_batch(gm, pays, 4, L, N, seed=1 + r)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    ctx.set_persistent_launch(0, 0, 0)
    t_default = time_batch()
    # the persistent form's autotuner on this batch's payoffs and levels
    t0 = time.perf_counter()
    shape = ctx.autotune_persistent(gm, pays, M=4, L=L)
    t_tune = time.perf_counter() - t0
    t_batch = time_batch()
    t0 = time.perf_counter()
    for r in range(reps):
        for p in pays:
            for l in range(L + 1):
                ctx.mlmc_level(gm, p, l, 4, N[0][l], 1 + r)
    torch.cuda.synchronize()
    t_levels = (time.perf_counter() - t0) / reps
    # the tail: level 8 (1024 paths of 65536 steps) of each payoff as one launch
    tail = {}
    for name, p in zip(names, pays):
        ctx.set_timing_slots([L])
        for r in range(reps):
            ctx.mlmc_level(gm, p, L, 4, N[0][L], 1 + r)
        st = ctx.kernel_stats()[L]
        ctx.set_timing(False)
        tail[name] = 1e3 * st["ms"] / st["launches"]
    return {"workload": "GBM call/Asian/lookback/digital, M=4, levels 0..8, N_l = 2^26 4^-l",
            "fine_path_steps": fine, "persistent_ms": 1e3 * t_batch,
            "autotuned_shape": {"block": shape[0], "ppt": shape[1], "blocks_per_cu": shape[2],
                                "tuning_s": t_tune},
            "persistent_ms_default_shape": 1e3 * t_default,
            "per_level_launches_ms": 1e3 * t_levels,
            "persistent_fine_steps_per_s": fine / t_batch,
            "per_level_fine_steps_per_s": fine / t_levels,
            "level8_launch_us": tail}


def accuracy_targets(ctx, mlmc, W, seeds=range(1, 33)):
    """The configurations' own accuracy targets, 32 seeds each: the adaptive
    GBM call (M = 4, eps in {2e-3, 1e-3, 5e-4} S0, against Black--Scholes)
    and the Heston call (M = 4, full-truncation Euler, eps = 1e-3 S0, against
    the characteristic-function price); median wall seconds and the
    empirical RMSE of the estimates."""
    ref = reference_prices()
    out = {"workload": "M=4, pilot 1e4, L_min 2, fp32 paths, 32 seeds",
           "black_scholes": ref["gbm_call"], "heston_price": ref["heston_call"]}
    cases = [("gbm_call", W.GBM_MODEL, eps) for eps in (2e-3, 1e-3, 5e-4)]
    cases.append(("heston_call", W.HESTON_MODEL, 1e-3))
    for name, md, eps in cases:
        m, p = mlmc.model(**md), mlmc.payoff(**W.CALL)
        t, rmse, mid = seeds_runs(ctx, m, p, eps * W.S0, 4, None, seeds, ref[name])
        key = f"eps_{eps:g}_S0" if name == "gbm_call" else f"{name}_eps_{eps:g}_S0"
        out[key] = {"median_s": t, "rmse": rmse, "target_rmse": eps * W.S0, "L": mid["L"],
                    "N_median_run": mid["N"]}
    return out


def fp64_error(ctx, mlmc, W, N_l, M=4, cap=1 << 20):
    """Error against fp64 of the benchmark's levels: the same samples (seed 1,
    the first min(N_l, 2^20) of each level) with fp32 and with fp64 paths;
    per-level difference of the means and its sum (the telescoped estimate)."""
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    levels, total = [], 0.0
    for l, n_l in enumerate(N_l):
        n = int(min(n_l, cap))
        a = ctx.mlmc_level(gm, gp, l, M, n, 1, precision=32)
        b = ctx.mlmc_level(gm, gp, l, M, n, 1, precision=64)
        d = a["sum_y"] / n - b["sum_y"] / n
        total += d
        levels.append({"level": l, "samples": n, "mean_fp64": b["sum_y"] / n,
                       "fp32_minus_fp64": d})
    return {"levels": levels, "telescoped_fp32_minus_fp64": total}


def fig3(ctx, mlmc, W):
    """The paper's Sec. 6 experiment on the GPU: N_l per level and eps^2 x cost
    and time for adaptive MLMC and standard Monte Carlo, call and digital."""
    from paper_1505_00965_amd import complexity
    out = {"workload": "GBM r=0.05 sigma=0.25 S0=100 T=1, K=100, M=2, fp32 paths, "
                       "eps (absolute) " + ", ".join(f"{e:g}" for e in W.FIG3_EPS)}
    for name, pay in (("call", W.FIG3_CALL), ("digital", W.FIG3_DIGITAL)):
        recs = complexity.sweep(ctx, mlmc.model(**W.FIG3_MODEL), mlmc.payoff(**pay), W.FIG3_EPS,
                                **W.FIG3_RUN)
        keep = ("eps", "L", "N", "estimate", "eps2_mlmc_cost", "eps2_std_cost", "mlmc_s",
                "std_s", "std_scaled")
        out[name] = {"runs": [{k: r[k] for k in keep} for r in recs],
                     "shape_checks": {what: ok for what, ok in
                                      complexity.shape_checks(recs, pay["kind"])}}
    # the same sweep with the Milstein scheme (Sec. 5's remark: beta = 2 >
    # gamma = 1, so eps^2 x cost stays bounded) and with its antithetic twin
    for name, extra in (("call_milstein", dict(scheme=1)),
                        ("call_milstein_antithetic", dict(scheme=1, antithetic=1))):
        m = mlmc.model(**dict(W.FIG3_MODEL, **extra))
        recs = complexity.sweep(ctx, m, mlmc.payoff(**W.FIG3_CALL), W.FIG3_EPS, run_stdmc=False,
                                **W.FIG3_RUN)
        e2 = [r["eps2_mlmc_cost"] for r in recs]
        out[name] = {"runs": [{k: r[k] for k in ("eps", "L", "N", "estimate", "eps2_mlmc_cost",
                                                  "mlmc_s")} for r in recs],
                     "eps2_cost_max_over_min": max(e2) / min(e2)}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library runs no cross-GPU work "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1505_00965_amd import mlmc, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    if args.copy_calibration:
        # a copy of known size: 256 MiB read + 256 MiB written
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.profile_level is not None:
        return profile_mode(args)
    ctx = mlmc.Context(0)
    stream = torch.cuda.current_stream()
    ctx.set_stream(stream)
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    M = 4
    eps = args.eps * W.S0

    def step(seed):
        return ctx.mlmc_run(gm, gp, eps, M=M, L_min=2, L_max=9, n_pilot=10000, seed=seed,
                            precision=32, persistent=bool(args.persistent))

    for i in range(args.warmup):
        step(1 + i % max(args.steps, 1))   # same seeds, hence launch sizes, as timed steps
    # context: the same steps with the default launch shapes, before tuning
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(1 + i)
    torch.cuda.synchronize()
    dt_default = time.perf_counter() - t0
    # the launch-shape autotuner for this model, payoff and M (three level
    # classes, block x samples per lane, measured on this device); every
    # later launch takes the tuned shapes
    tune = {}
    t0 = time.perf_counter()
    if args.persistent:
        tune["persistent"] = ctx.autotune_persistent(gm, [gp], M=M, L=4)
    else:
        ctx.autotune(gm, gp, M=M, precision=32)
        tune.update({f"level_{l}": ctx.tuned_shape(gm, gp, l, M=M) for l in (0, 1, 3)})
    tune["tuning_s"] = time.perf_counter() - t0
    for i in range(args.warmup):
        step(1 + i % max(args.steps, 1))
    # Which kernel dominates: every slot timed over the same steps, untimed
    # by the clock.  The timed region then stamps only that kernel's launches
    # (each stamped launch costs the host ~10 us more than a plain one).
    ctx.set_timing(True)
    for i in range(args.steps):
        step(1 + i)
    all_slots = ctx.kernel_stats()
    ctx.set_timing(False)
    dom = mlmc.STAT_PERSISTENT if args.persistent else max(range(16), key=lambda l: all_slots[l]["ms"])
    ctx.set_timing_slots([dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step(1 + i) for i in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = ctx.kernel_stats()
    ctx.set_timing(False)
    # context: the same steps with no kernel stamped (a stamped launch costs
    # the host ~10 us of event handling); `value` stays the timed region's
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(1 + i)
    torch.cuda.synchronize()
    dt_unstamped = time.perf_counter() - t0

    fine = sum(fine_steps_of(r, M) for r in runs)
    value = fine / dt
    roofline = None
    if args.persistent:
        # one graph launch (plan, persistent sampler, driver update) per iteration
        s = stats[mlmc.STAT_PERSISTENT]
        if s["launches"]:
            avg_ms = s["ms"] / s["launches"]
            samples = sum(sum(r["N"]) for r in runs) / s["launches"]
            ops_per_launch = (OPS_PER_FINE_STEP * s["fine_steps"] / s["launches"]
                              + OPS_PER_SAMPLE * samples)
            achieved = ops_per_launch / (avg_ms * 1e-3)
            roofline = {"bound": "alu", "achieved": achieved / 1e12,
                        "peak": VALU_PEAK_OPS / 1e12, "unit": "Top/s",
                        "frac": achieved / VALU_PEAK_OPS, "traffic": None,
                        "kernel": "persistent_kernel<GBM,M=4> graph (plan + sampler + update)",
                        "ops_per_launch": ops_per_launch, "avg_launch_ms": avg_ms,
                        "launches": s["launches"]}
    else:
        # dominant kernel: the level whose launches took the most time
        lv = dom
        s = stats[lv]
        if s["launches"]:
            avg_ms = s["ms"] / s["launches"]
            samples = s["fine_steps"] / M**lv
            ops_per_launch = algorithmic_ops(lv, s["fine_steps"], samples) / s["launches"]
            achieved = ops_per_launch / (avg_ms * 1e-3)
            label = ("short_level_kernel<GBM,call,fp32,n_f=1>" if lv == 0
                     else f"level_kernel<GBM,call,fp32,M=4> at level {lv}")
            samples_per_s = samples / s["launches"] / (avg_ms * 1e-3)
            roofline = {"bound": "alu", "achieved": achieved / 1e12,
                        "peak": VALU_PEAK_OPS / 1e12, "unit": "Top/s",
                        "frac": achieved / VALU_PEAK_OPS, "traffic": measured_traffic(label),
                        "kernel": label,
                        # the target (half the vector-ALU peak) is judged by `frac`:
                        # executed operations per sample over the issue peak
                        "ops_per_sample": {"executed": OPS_PER_SAMPLE_L0 if lv == 0 else None,
                                           "method": OPS_PER_SAMPLE_L0_METHOD if lv == 0 else None},
                        "frac_method_ops": (achieved / VALU_PEAK_OPS * OPS_PER_SAMPLE_L0_METHOD
                                            / OPS_PER_SAMPLE_L0 if lv == 0 else None),
                        "ops_per_launch": ops_per_launch, "avg_launch_ms": avg_ms,
                        "launches": s["launches"],
                        "fine_steps_per_launch": s["fine_steps"] / s["launches"]}
            # from the committed counter summaries of this kernel (profiles/):
            # issued vector instructions x 4 cycles over SIMD cycles
            # (SQ_INSTS_VALU, GRBM_GUI_ACTIVE); this run's rate against the
            # ceiling those instructions allow; fp32 FLOPs (an fma counts 2,
            # SQ_INSTS_VALU_FLOPS_FP32 + _TRANS) per second over the fp32 peak
            roofline["valu_issue_frac_counters"] = profile_field(label, "valu_issue_frac")
            ipsamp = profile_field(label, "valu_insts_per_sample")
            roofline["valu_insts_per_sample"] = ipsamp
            roofline["slot_ceiling_frac"] = (samples_per_s * ipsamp / VALU_PEAK_OPS
                                             if ipsamp else None)
            fps = profile_field(label, "fp32_flops_per_sample")
            roofline["fp32_flops_per_sample"] = fps
            roofline["fp32_flop_frac"] = samples_per_s * fps / FP32_PEAK_FLOPS if fps else None

    line = {"metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
            "ms_per_step_unstamped": 1e3 * dt_unstamped / args.steps,
            "ms_per_step_default_shapes": 1e3 * dt_default / args.steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"adaptive MLMC, GBM European call S0=100 r=0.05 sigma=0.2 "
                                   f"T=1 K=100, M=4, RMSE {args.eps:g}*S0, fp32 paths fp64 sums, "
                                   + ("one graph launch per driver iteration" if args.persistent
                                      else "one level per launch"),
                       "levels": runs[-1]["L"] + 1, "N_l": runs[-1]["N"],
                       "estimate": runs[-1]["estimate"], "tuned_shapes": tune},
            "roofline": roofline}

    if not args.persistent and not args.no_tta:
        # the same estimates with every driver iteration as one graph launch
        # (plan, persistent all-levels sampler, driver update), in the shape
        # the persistent form's tuner picks for this payoff and depth
        t0 = time.perf_counter()
        pshape = ctx.autotune_persistent(gm, [gp], M=M, L=runs[-1]["L"])
        ptune_s = time.perf_counter() - t0
        for i in range(args.warmup):
            ctx.mlmc_run(gm, gp, eps, M=M, L_min=2, L_max=9, n_pilot=10000,
                         seed=1 + i % max(args.steps, 1), precision=32, persistent=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gr = [ctx.mlmc_run(gm, gp, eps, M=M, L_min=2, L_max=9, n_pilot=10000, seed=1 + i,
                           precision=32, persistent=True) for i in range(args.steps)]
        torch.cuda.synchronize()
        dtg = time.perf_counter() - t0
        line["adaptive_graph_form"] = {
            "ms_per_step": 1e3 * dtg / args.steps,
            "tuned_shape": {"block": pshape[0], "ppt": pshape[1], "blocks_per_cu": pshape[2],
                            "tuning_s": ptune_s},
            "fine_path_steps_per_s": sum(fine_steps_of(r, M) for r in gr) / dtg,
            "same_N_l": all(a["N"] == b["N"] for a, b in zip(runs, gr))}
    if not args.no_tta:
        line["persistent_batch"] = persistent_batch(ctx, mlmc, W)
        line["seconds_to_rmse"] = time_to_accuracy(ctx, mlmc, W, args)
        line["accuracy_targets"] = accuracy_targets(ctx, mlmc, W)
        line["fp64_error"] = fp64_error(ctx, mlmc, W, runs[-1]["N"])
        line["fig3"] = fig3(ctx, mlmc, W)

    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(runs[-1], M, args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
