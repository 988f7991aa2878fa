"""tests/golden/prices.json (reference prices the benchmark's accuracy runs
compare with) is what tests/golden/make_prices.py writes from the oracle."""
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def test_golden_prices_are_the_oracles(orc):
    g = json.load(open(os.path.join(HERE, "golden", "prices.json")))
    want = {"gbm_call": orc.bs_call(), "gbm_digital": orc.bs_digital(),
            "gbm_lookback": orc.lookback_float_call(), "gbm_asian": orc.asian_arith_call_pde(),
            "gbm_geometric_asian": orc.geometric_asian_call(), "heston_call": orc.heston_call()}
    assert set(g) == set(want)
    for k, v in want.items():
        assert abs(g[k]["value"] - v) <= 1e-12 * abs(v), k
