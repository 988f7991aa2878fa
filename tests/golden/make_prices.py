"""Write tests/golden/prices.json: reference prices for the benchmark's
accuracy runs, computed by the oracle's closed forms only.

    python tests/golden/make_prices.py

Parameters: S0 = K = 100, r = 0.05, T = 1; GBM sigma = 0.2; Heston kappa = 2,
theta = 0.04, xi = 0.3, rho = -0.7, v0 = 0.04.  All prices discounted.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def main():
    prices = {
        "gbm_call": {"value": oracle.bs_call(),
                     "source": "Black-Scholes European call (oracle closed form)"},
        "gbm_digital": {"value": oracle.bs_digital(),
                        "source": "Black-Scholes cash-or-nothing call, payout 1 (oracle closed form)"},
        "gbm_lookback": {"value": oracle.lookback_float_call(),
                         "source": "Goldman-Sosin-Gatto floating-strike lookback call, continuous "
                                   "monitoring (oracle closed form)"},
        "gbm_asian": {"value": oracle.asian_arith_call_pde(),
                      "source": "continuous arithmetic-average Asian call, Vecer PDE by "
                                "Crank-Nicolson (oracle asian_pde module)"},
        "gbm_geometric_asian": {"value": oracle.geometric_asian_call(),
                                "source": "continuous geometric-average Asian call (oracle closed "
                                          "form); a lower bound of the arithmetic one"},
        "heston_call": {"value": oracle.heston_call(),
                        "source": "Heston European call, characteristic-function formula (oracle "
                                  "closed form)"},
    }
    with open(os.path.join(HERE, "prices.json"), "w") as f:
        json.dump(prices, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
