"""Complexity sweep of Sec. 6 (Fig. 3): adaptive MLMC against standard Monte
Carlo over a list of accuracy requests, both run on the GPU.

For every eps the adaptive driver (``mlmc_run``) picks L and the N_l; its
cost is sum_l N_l C_l path steps (C_0 = 1, C_l = M^l + M^(l-1)), the cost
measure of Sec. 3 (generator calls) applied to the coupled pairs.

The standard Monte Carlo comparator of Sec. 3 (eq. for a_M) is the uncoupled
sampler on the finest grid of that MLMC run, h_L = M^-L T, so that both
estimators carry the same discretisation bias; its sampling variance gets the
same half of the mean-square budget as the MLMC run's, so it needs
N = ceil(2 V[P_L] / eps^2) paths of M^L steps.  V[P_L] is measured by a pilot
of the uncoupled sampler (generator streams 4/5, never shared with the MLMC
run), then the comparator is run in full and timed.  The returned records
hold what Fig. 3 plots: N_l per level, and eps^2 times cost and time for
both methods.
"""
import math
import time


def _level_cost(l, M):
    return 1.0 if l == 0 else float(M ** l + M ** (l - 1))


def sweep(ctx, model, payoff, eps_list, M=2, L_min=2, L_max=12, n_pilot=10000, seed=1,
          precision=32, var_pilot=1 << 16, run_stdmc=True, std_cost=True, max_std_steps=2e11):
    """One record per eps (largest first, as in Fig. 3).

    model / payoff: ``mlmc.model(...)`` / ``mlmc.payoff(...)`` structures.
    std_cost: estimate the comparator's cost from a variance pilot;
    run_stdmc: also run and time the comparator.  max_std_steps caps the
    standard Monte Carlo run (path steps); a capped comparator is timed on
    the cap and its time scaled up, which the record states
    (``std_scaled``).  With an antithetic model there is no comparator.
    """
    if model.antithetic:
        run_stdmc = std_cost = False
    # one untimed run first: the first launch of a kernel variant loads its code
    ctx.mlmc_run(model, payoff, max(eps_list), M=M, L_min=L_min, L_max=L_max, n_pilot=n_pilot,
                 seed=seed + 999, precision=precision)
    out = []
    for i, eps in enumerate(sorted(eps_list, reverse=True)):
        run_seed = seed + 1000 * i
        r = ctx.mlmc_run(model, payoff, eps, M=M, L_min=L_min, L_max=L_max, n_pilot=n_pilot,
                         seed=run_seed, precision=precision)
        L = r["L"]
        cost = sum(n * _level_cost(l, M) for l, n in enumerate(r["N"][:L + 1]))
        rec = {"eps": eps, "L": L, "N": list(r["N"][:L + 1]), "V": list(r["V"][:L + 1]),
               "estimate": r["estimate"], "mlmc_cost": cost, "mlmc_s": r["wall_s"],
               "eps2_mlmc_cost": eps * eps * cost, "eps2_mlmc_s": eps * eps * r["wall_s"]}
        if not run_stdmc and not std_cost:
            out.append(rec)
            continue
        # variance of the finest-grid payoff, from an independent pilot
        p = ctx.mlmc_stdmc(model, payoff, L, M, var_pilot, run_seed, precision=precision)
        mean = p["sum_pf"] / p["n"]
        var = max(p["sum_pf2"] / p["n"] - mean * mean, 0.0)
        n_std = max(2, math.ceil(2.0 * var / (eps * eps)))
        steps = float(M ** L)
        rec.update({"V_PL": var, "std_N": n_std, "std_cost": n_std * steps,
                    "eps2_std_cost": eps * eps * n_std * steps})
        if run_stdmc:
            n_run = min(n_std, max(2, int(max_std_steps / steps)))
            t0 = time.perf_counter()     # mlmc_stdmc returns after its results are in
            s = ctx.mlmc_stdmc(model, payoff, L, M, n_run, run_seed, path_offset=var_pilot,
                               precision=precision)
            dt = time.perf_counter() - t0
            rec.update({"std_estimate": s["sum_pf"] / s["n"],
                        "std_s": dt * n_std / n_run, "std_scaled": n_run < n_std,
                        "eps2_std_s": eps * eps * dt * n_std / n_run})
        out.append(rec)
    return out


def shape_checks(records, payoff_kind):
    """The qualitative claims of Sec. 6 about Fig. 3, as (name, passed) pairs."""
    checks = []
    for r in records:
        n = r["N"]
        checks.append((f"eps={r['eps']:g}: N_l non-increasing in l",
                       all(n[l + 1] <= n[l] for l in range(len(n) - 1))))
    Ls = [r["L"] for r in records]                # eps decreasing
    if payoff_kind == 0:
        checks.append(("levels are added as eps falls",
                       all(b >= a for a, b in zip(Ls, Ls[1:])) and Ls[-1] > Ls[0]))
    else:
        # the digital's level differences decay slowly (beta = 1/2) and its
        # bias test sees noisy means, so one run per eps gives a trend only
        checks.append(("more levels at the smallest eps than at the largest", Ls[-1] > Ls[0]))
    checks.append(("standard MC costs more at every eps",
                   all(r["std_cost"] > r["mlmc_cost"] for r in records)))
    e2s = [r["eps2_std_cost"] for r in records]
    checks.append(("eps^2 x standard MC cost grows as eps falls", e2s[-1] > 2.0 * e2s[0]))
    e2m = [r["eps2_mlmc_cost"] for r in records]
    if payoff_kind == 0:
        # Euler with a Lipschitz payoff: beta = gamma = 1, cost ~ eps^-2 (log eps)^2
        checks.append(("eps^2 x MLMC cost roughly flat (call)",
                       max(e2m) / min(e2m) < (e2s[-1] / e2s[0])))
    return checks
