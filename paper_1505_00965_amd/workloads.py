"""Named workload presets: model and payoff parameters, sizes and seeds.

Plain data only (no arithmetic of the method); shared by the tests, the smoke
check and the benchmark so that the GPU library and the CPU oracle are fed
identical inputs.  Random numbers are not stored anywhere: each side draws
them from its own Philox4x32-10 implementation.
"""

S0, R, SIGMA, T = 100.0, 0.05, 0.2, 1.0
HESTON = dict(kappa=2.0, theta=0.04, xi=0.3, rho=-0.7, v0=0.04)

GBM_MODEL = dict(kind=0, S0=S0, r=R, sigma=SIGMA, T=T, **HESTON)
HESTON_MODEL = dict(kind=1, S0=S0, r=R, sigma=SIGMA, T=T, **HESTON)
# the paper's Sec. 6 experiment uses sigma = 0.25
PAPER_GBM_MODEL = dict(kind=0, S0=S0, r=R, sigma=0.25, T=T, **HESTON)

CALL = dict(kind=0, K=100.0, payout=1.0)
ASIAN = dict(kind=1, K=100.0, payout=1.0)
LOOKBACK = dict(kind=2, K=100.0, payout=1.0)
DIGITAL = dict(kind=3, K=100.0, payout=1.0)
DIGITAL_COND = dict(kind=4, K=100.0, payout=1.0)
PAYOFFS = {"call": CALL, "asian": ASIAN, "lookback": LOOKBACK, "digital": DIGITAL}

# Sec. 6 experiment (Fig. 3): GBM with sigma = 0.25, European call and digital
# call (payout 100, h(100) = half the payout), K = 100, T = 1; the accuracy
# requests eps (absolute) and the refinement factor M = 2 the paper suggests
# thinking of; n_pilot = 1000 and L_min = 2 are readings (not stated).
FIG3_MODEL = PAPER_GBM_MODEL
FIG3_CALL = dict(kind=0, K=100.0, payout=1.0)
FIG3_DIGITAL = dict(kind=3, K=100.0, payout=100.0)
FIG3_EPS = [0.1, 0.05, 0.02, 0.01, 0.005]
FIG3_RUN = dict(M=2, L_min=2, L_max=12, n_pilot=1000)

# Parity set: GBM call, M=2, levels 0..5, 20000 samples per level, seed 1, fp64.
PARITY_SET = dict(M=2, levels=list(range(6)), N=20000, seed=1, precision=64)
# Adaptive driver: GBM call, M=4, eps in units of S0.
DRIVER_EPS = [2e-3, 1e-3, 5e-4]
# Throughput sweep: N_l = 2^(32-2l) for l <= 5, 2^22 above (fp32, M=4).
def throughput_n(l):
    return 2 ** (32 - 2 * l) if l <= 5 else 2 ** 22
# MLMC-shaped persistent batch: N_l = 2^26 4^-l, levels 0..8, four payoffs.
def persistent_n(l):
    return 2 ** 26 // 4 ** l
