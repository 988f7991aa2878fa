"""Benchmark: adaptive MLMC on one MI355X, fine path-steps per second.

One step = one complete adaptive MLMC estimate (every level sampled on the
GPU, the fp64 driver update on the device) of the GBM European call (S0=100,
r=0.05, sigma=0.2, T=1, K=100), M=4, fp32 paths with fp64 sums.  By default
the estimate runs device-planned: per driver iteration one launch of the
all-levels sampler and one of the update-and-plan block, enqueued by the host
one iteration ahead (--form per-level: one launch per level and iteration,
with the host reading each update before it launches).  The target RMSE
defaults to 2e-5*S0: with it the driver reaches about 10^8 samples at level
0, the scale that workload is described at (its listed RMSEs of
2e-3..5e-4*S0 need only 1.4e4..2.2e5 there).

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


# The sources each profiled kernel is compiled from: a committed counter
# summary is used only while their digest is the one it was taken with.
# The digest covers them and the compile flags.
KERNEL_SOURCES = {
    "level": ("philox.hpp", "sampler.hpp", "sampler_impl.hpp", "reduce.hpp", "level.hip",
              "level.hpp", "level_kernels.hpp", "level_gbm.hip"),
    "persistent": ("philox.hpp", "sampler.hpp", "sampler_impl.hpp", "reduce.hpp", "level.hpp",
                   "driver.hpp", "driver_dev.hpp", "cv.hpp", "cv_tab.hpp", "persistent.hpp",
                   "persistent.hip", "persistent_gbm.hip"),
}


def kernel_sources_digest(kernel_label):
    import hashlib
    from paper_1505_00965_amd import build
    h = hashlib.sha256()
    family = "persistent" if kernel_label.startswith("persistent") else "level"
    for f in KERNEL_SOURCES[family]:
        with open(os.path.join(ROOT, "paper_1505_00965_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    flags = [f for f in build.COMMON if not f.startswith("-I") and "include" not in f]
    h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]


def profile_field(kernel_label, field):
    """A figure from the committed rocprofv3 summaries (profiles/*.md) of this
    kernel, or None if the kernel sources changed since they were taken."""
    import glob
    digest = kernel_sources_digest(kernel_label)
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
    ap.add_argument("--stamp-every", type=int, default=5,
                    help="timed region: stamp every launch of the dominant kernel in one "
                         "estimate in this many (the others run unstamped)")
    ap.add_argument("--form", choices=("planned", "per-level"), default="planned",
                    help="planned: per driver iteration one all-levels sampler launch and one "
                         "update-and-plan launch, enqueued ahead by the host; per-level: one "
                         "launch per level and iteration")
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
    ap.add_argument("--profile-run", type=int, default=0,
                    help="profile mode: this many device-planned adaptive estimates of the "
                         "benchmark workload (after tuning), then one JSON line")
    ap.add_argument("--planned-shape", default="",
                    help="with --profile-run: block,ppt,blocks_per_cu of the persistent sampler "
                         "instead of the run tuner's choice")
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


def profile_run_mode(args):
    """The benchmark's device-planned estimates, `profile_run` of them after
    the tuners and a warm-up, untimed (counter runs take the last
    `sampler_launches` persistent-sampler dispatches)."""
    import torch
    from paper_1505_00965_amd import mlmc, workloads as W
    ctx = mlmc.Context(0)
    ctx.set_stream(torch.cuda.current_stream())
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    M, eps = 4, args.eps * W.S0
    run_kw = dict(M=M, L_min=2, L_max=9, n_pilot=10000, precision=32)
    ctx.autotune(gm, gp, M=M, precision=32)
    if args.planned_shape:
        shape = tuple(int(x) for x in args.planned_shape.split(","))
        ctx.set_persistent_launch(*shape)
    else:
        shape = ctx.autotune_run(gm, gp, eps, seed=1, **run_kw)
    for i in range(2):
        ctx.mlmc_run(gm, gp, eps, seed=1 + i, persistent=True, **run_kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [ctx.mlmc_run(gm, gp, eps, seed=1 + i, persistent=True, **run_kw)
            for i in range(args.profile_run)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"mode": "profile-run", "runs": len(runs), "eps": args.eps,
           "sampler_launches": sum(r["iterations"] + 1 for r in runs),
           "fine_steps": sum(fine_steps_of(r, M) for r in runs),
           "samples": float(sum(sum(r["N"]) for r in runs)), "ops": run_ops(runs, M),
           "shape": list(shape), "wall_s": wall,
           "kernel": f"persistent_kernel<GBM,M=4,ppt={shape[1]},call>"}
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


def seeds_runs(ctx, m, p, eps, M, cv, seeds, exact, cv_levels=0, persistent=False):
    """Runs over the seeds: median wall seconds, empirical RMSE against the
    continuous price, and the median run."""
    import statistics
    runs = [ctx.mlmc_run(m, p, eps, M=M, seed=s, precision=32, cv=cv, cv_levels=cv_levels,
                         persistent=persistent)
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
            # plain MLMC device-planned (the control variate runs per level),
            # in the shape the run tuner picks for this configuration
            ctx.autotune_run(m, p, eps * W.S0, M=4, seed=1)
            tq, eq, _ = seeds_runs(ctx, m, p, eps * W.S0, 4, None, seeds, exact, persistent=True)
            e.update({"plain_planned_s": tq, "plain_planned_rmse": eq})
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
                # the tabulated network in the device-planned form (the
                # persistent shape as tuned for the plain run above)
                ctx.autotune_run(m, p, eps * W.S0, M=4, seed=1)
                tqc, eqc, rqc = seeds_runs(ctx, m, p, eps * W.S0, 4, cv, seeds, exact,
                                           persistent=True)
                cv.set_tabulated(False)
                e.update({"cv_tab_s": tt, "cv_tab_rmse": et, "cv_tab_cost": rt["cost"],
                          "cv_tab_N": rt["N"], "cv_tab_V": [round(v, 6) for v in rt["V"]],
                          "speedup_tab": tp / tt, "cv_tab_with_training_s": tt + entry["train_s"],
                          "cv_tab_planned_s": tqc, "cv_tab_planned_rmse": eqc,
                          "speedup_tab_planned_vs_plain_planned": e["plain_planned_s"] / tqc})
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


def level_rates(ctx, gm, gp, M, all_slots, steps, target_fine=1 << 30, reps=3):
    """Each level's launches in the adaptive run (every slot timed) against the
    same level's sampler saturated: one launch of about 2^30 fine steps."""
    out = {}
    for l in range(16):
        s = all_slots[l]
        if not s["launches"]:
            continue
        N = max(target_fine // M**l, 1 << 14)
        ctx.set_timing_slots([l])
        for r in range(reps):
            ctx.mlmc_level(gm, gp, l, M, N, 1000 + r)
        st = ctx.kernel_stats()[l]
        ctx.set_timing(False)
        run_rate = s["fine_steps"] / (s["ms"] * 1e-3)
        sat_rate = st["fine_steps"] / (st["ms"] * 1e-3)
        out[f"level_{l}"] = {"launches_per_step": s["launches"] / steps,
                             "avg_launch_us": 1e3 * s["ms"] / s["launches"],
                             "samples_per_launch": s["fine_steps"] / M**l / s["launches"],
                             "fine_steps_per_s": run_rate,
                             "saturated_samples_per_launch": N,
                             "saturated_fine_steps_per_s": sat_rate,
                             "frac_of_saturated": run_rate / sat_rate}
    return out


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
        ctx.autotune_run(m, p, eps * W.S0, M=4, seed=1)
        tq, rq, _ = seeds_runs(ctx, m, p, eps * W.S0, 4, None, seeds, ref[name], persistent=True)
        key = f"eps_{eps:g}_S0" if name == "gbm_call" else f"{name}_eps_{eps:g}_S0"
        out[key] = {"median_s": t, "rmse": rmse, "target_rmse": eps * W.S0, "L": mid["L"],
                    "N_median_run": mid["N"], "planned_median_s": tq, "planned_rmse": rq}
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


def per_level_roofline(stats, lv, M, label):
    """Roofline of one level's sampler from stamped launches (per-level form)."""
    s = stats[lv]
    if not s["launches"]:
        return None
    avg_ms = s["ms"] / s["launches"]
    samples = s["fine_steps"] / M**lv
    ops_per_launch = algorithmic_ops(lv, s["fine_steps"], samples) / s["launches"]
    achieved = ops_per_launch / (avg_ms * 1e-3)
    samples_per_s = samples / s["launches"] / (avg_ms * 1e-3)
    r = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
         "unit": "Top/s", "frac": achieved / VALU_PEAK_OPS,
         "traffic": measured_traffic(label), "kernel": label,
         "ops_per_sample": {"executed": OPS_PER_SAMPLE_L0 if lv == 0 else None,
                            "method": OPS_PER_SAMPLE_L0_METHOD if lv == 0 else None},
         "frac_method_ops": (achieved / VALU_PEAK_OPS * OPS_PER_SAMPLE_L0_METHOD
                             / OPS_PER_SAMPLE_L0 if lv == 0 else None),
         "ops_per_launch": ops_per_launch, "avg_launch_ms": avg_ms, "launches": s["launches"],
         "fine_steps_per_launch": s["fine_steps"] / s["launches"]}
    # from the committed counter summaries of this kernel (profiles/):
    # issued vector instructions x 4 cycles over SIMD cycles; this run's rate
    # against the ceiling those instructions allow; fp32 FLOPs over the peak
    r["valu_issue_frac_counters"] = profile_field(label, "valu_issue_frac")
    ipsamp = profile_field(label, "valu_insts_per_sample")
    r["valu_insts_per_sample"] = ipsamp
    r["slot_ceiling_frac"] = samples_per_s * ipsamp / VALU_PEAK_OPS if ipsamp else None
    fps = profile_field(label, "fp32_flops_per_sample")
    r["fp32_flops_per_sample"] = fps
    r["fp32_flop_frac"] = samples_per_s * fps / FP32_PEAK_FLOPS if fps else None
    return r


def run_ops(runs, M):
    """Algorithmic vector-ALU operations of the runs' samples (all levels)."""
    ops = 0.0
    for r in runs:
        for l, n in enumerate(r["N"]):
            ops += algorithmic_ops(l, n * M**l, n)
    return ops


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
    if args.profile_run:
        return profile_run_mode(args)
    ctx = mlmc.Context(0)
    stream = torch.cuda.current_stream()
    ctx.set_stream(stream)
    gm, gp = mlmc.model(**W.GBM_MODEL), mlmc.payoff(**W.CALL)
    M = 4
    eps = args.eps * W.S0
    planned = args.form == "planned"
    run_kw = dict(M=M, L_min=2, L_max=9, n_pilot=10000, precision=32)

    def step(seed, persistent=planned):
        return ctx.mlmc_run(gm, gp, eps, seed=seed, persistent=persistent, **run_kw)

    def timed_pass(persistent=planned, stamp_every=0):
        """The K steps by the clock; with stamp_every k, the timing (set up
        by the caller) is paused for all but every k-th estimate."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = []
        for i in range(args.steps):
            if stamp_every:
                ctx.set_timing_paused(i % stamp_every != 0)
            rs.append(step(1 + i, persistent))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if stamp_every:
            ctx.set_timing_paused(False)
        return rs, dt

    def warm(persistent=planned):
        for i in range(args.warmup):
            step(1 + i % max(args.steps, 1), persistent)   # the timed steps' seeds, hence sizes

    warm()
    # context: the same steps with the default launch shapes, before tuning
    _, dt_default = timed_pass()
    # launch-shape autotuners: the per-level sampler's shape per level (block
    # x samples per lane, on this device) and, for the device-planned form,
    # the persistent sampler's shape timed on this run configuration itself
    tune = {}
    t0 = time.perf_counter()
    ctx.autotune(gm, gp, M=M, precision=32)
    tune.update({f"level_{l}": ctx.tuned_shape(gm, gp, l, M=M) for l in range(7)})
    if planned:
        tune["planned_run"] = ctx.autotune_run(gm, gp, eps, seed=1, **run_kw)
    tune["tuning_s"] = time.perf_counter() - t0
    warm()
    # Which kernel dominates: every slot timed over the same steps, untimed
    # by the clock.  The timed region then stamps that kernel only, and only
    # in every --stamp-every-th estimate (a stamped launch costs ~10 us of
    # queue time more than a plain one), every launch of those estimates, so
    # the stamped launches are whole runs whose work is known.
    ctx.set_timing(True)
    all_runs = [step(1 + i) for i in range(args.steps)]
    all_slots = ctx.kernel_stats()
    ctx.set_timing(False)
    dom = mlmc.STAT_PERSISTENT if planned else max(range(16), key=lambda l: all_slots[l]["ms"])
    ctx.set_timing_slots([dom])
    runs, dt = timed_pass(stamp_every=args.stamp_every)
    stats = ctx.kernel_stats()
    ctx.set_timing(False)
    stamped_runs = runs[::args.stamp_every]
    # context: the same steps with no kernel stamped
    _, dt_unstamped = timed_pass()

    fine = sum(fine_steps_of(r, M) for r in runs)
    value = fine / dt
    roofline = None
    s = stats[dom]
    if planned and s["launches"]:
        # the device-planned form: one persistent all-levels sampler launch
        # per driver iteration (and the empty one queued past the last
        # update).  The host sees only whole runs: the operations of the
        # stamped runs over their stamped sampler launches (all of them).
        launches = sum(r["iterations"] + 1 for r in stamped_runs)
        assert launches == s["launches"], (launches, s["launches"])
        ops = run_ops(stamped_runs, M)
        avg_ms = s["ms"] / s["launches"]
        achieved = ops / launches / (avg_ms * 1e-3)
        all_launches = sum(r["iterations"] + 1 for r in runs)
        shape = tune.get("planned_run") or (256, 1, 4)
        label = f"persistent_kernel<GBM,M=4,ppt={shape[1]},call>"
        a = all_slots[dom]
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                    "unit": "Top/s", "frac": achieved / VALU_PEAK_OPS,
                    "traffic": measured_traffic(label), "kernel": label,
                    "launch_shape": {"block": shape[0], "ppt": shape[1], "blocks_per_cu": shape[2]},
                    "ops_per_launch": ops / launches, "avg_launch_ms": avg_ms,
                    "launches": s["launches"], "launches_in_timed_region": all_launches,
                    "stamped_estimates": len(stamped_runs), "stamp_every": args.stamp_every,
                    # every sampler launch of the same steps stamped (the
                    # all-slots pass): the stamped runs' cross-check
                    "avg_launch_ms_all_stamped": a["ms"] / a["launches"] if a["launches"] else None,
                    "ops_per_launch_all": run_ops(runs, M) / all_launches,
                    "share_of_step": all_launches * avg_ms * 1e-3 / dt}
        # from the committed counter summary of this kernel (profiles/): its
        # issue fraction under the counters, this run's rate against the
        # ceiling its instructions per fine step allow, and its fp32 FLOPs
        # over the fp32 peak
        fine_per_s = sum(fine_steps_of(r, M) for r in stamped_runs) / launches / (avg_ms * 1e-3)
        roofline["valu_issue_frac_counters"] = profile_field(label, "valu_issue_frac")
        ipf = profile_field(label, "valu_insts_per_fine_step")
        roofline["valu_insts_per_fine_step"] = ipf
        roofline["slot_ceiling_frac"] = fine_per_s * ipf / VALU_PEAK_OPS if ipf else None
        fpf = profile_field(label, "fp32_flops_per_fine_step")
        roofline["fp32_flops_per_fine_step"] = fpf
        roofline["fp32_flop_frac"] = fine_per_s * fpf / FP32_PEAK_FLOPS if fpf else None
    elif s["launches"]:
        label = ("short_level_kernel<GBM,call,fp32,n_f=1>" if dom == 0
                 else f"level_kernel<GBM,call,fp32,M=4> at level {dom}")
        roofline = per_level_roofline(stats, dom, M, label)
        roofline["launches_in_timed_region"] = all_slots[dom]["launches"]
        roofline["stamped_estimates"] = len(stamped_runs)
        roofline["stamp_every"] = args.stamp_every

    upd = all_slots[mlmc.STAT_DRIVER]
    line = {"metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
            "ms_per_step_unstamped": 1e3 * dt_unstamped / args.steps,
            "ms_per_step_default_shapes": 1e3 * dt_default / args.steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"adaptive MLMC, GBM European call S0=100 r=0.05 sigma=0.2 "
                                   f"T=1 K=100, M=4, RMSE {args.eps:g}*S0, fp32 paths fp64 sums, "
                                   + ("device-planned: per driver iteration one all-levels "
                                      "sampler launch and one update-and-plan launch, enqueued "
                                      "ahead of the host" if planned
                                      else "one level per launch"),
                       "levels": runs[-1]["L"] + 1, "N_l": runs[-1]["N"],
                       "iterations": runs[-1]["iterations"],
                       "estimate": runs[-1]["estimate"], "tuned_shapes": tune},
            "roofline": roofline,
            "update_kernel_us": 1e3 * upd["ms"] / upd["launches"] if upd["launches"] else None}

    if planned:
        # context: the per-level form of the same estimates (one launch per
        # level and iteration, the tuned per-level shapes), its per-level
        # rates against each level saturated, and its dominant kernel
        warm(False)
        pl_runs, pl_dt = timed_pass(False)
        ctx.set_timing(True)
        for i in range(args.steps):
            step(1 + i, False)
        pl_slots = ctx.kernel_stats()
        ctx.set_timing(False)
        ctx.set_timing_slots([0])
        timed_pass(False, stamp_every=args.stamp_every)
        pl_stats = ctx.kernel_stats()
        ctx.set_timing(False)
        line["per_level_form"] = {
            "ms_per_step": 1e3 * pl_dt / args.steps,
            "fine_path_steps_per_s": sum(fine_steps_of(r, M) for r in pl_runs) / pl_dt,
            "same_N_l": all(a["N"] == b["N"] for a, b in zip(runs, pl_runs)),
            "level0_roofline": per_level_roofline(pl_stats, 0, M,
                                                  "short_level_kernel<GBM,call,fp32,n_f=1>"),
            "per_level": level_rates(ctx, gm, gp, M, pl_slots, args.steps)}
    else:
        line["per_level"] = level_rates(ctx, gm, gp, M, all_slots, args.steps)
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
