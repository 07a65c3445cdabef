"""The operation counts of App. B against the totals printed in Table 1."""
import json
import os

import numpy as np

from oracle import accounting as acc

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_table1_update_and_prediction():
    t = GOLD["table1_operations"]
    m = t["m"]
    u = t["update_one_domain"]
    ops = acc.update_operations(m, u["n"], u["p"])
    assert ops == 7645288
    assert round(ops / 1e6, 2) == round(u["printed"] / 1e6, 2)
    for case in t["prediction"]:
        ops = acc.prediction_operations(m, case["n"])
        assert ops == 4 * m * case["n"]
        assert round(ops / 1e6, 2) == round(case["printed"] / 1e6, 2)


def test_table3_rows_sum_to_printed_total():
    rng = np.random.default_rng(0)
    for _ in range(20):
        m, n, p, gam = (int(v) for v in rng.integers(2, 300, 4))
        assert sum(acc.update_rows(m, n, p, gam)) == acc.update_multiplications(m, n, p, gam)
