"""Pins of the operation counter (oracle/opcount.py) and of the FP64 table the benchmark takes from it.

The counter is checked on expressions whose operation count is known by inspection, on the rules
that define it (an untaken np.where branch, a product with a literal 0 or 1, a reused subexpression),
and on the logarithmic mean of the oracle, whose series form is counted by hand from its formula.
bench.ORACLE_OPS must equal the counter's output for every workload it lists."""
import numpy as np
import pytest

import bench
from oracle import gas as G
from oracle import opcount as OC


def test_counts_of_plain_expressions():
    a, b, c = OC.Op(1.5), OC.Op(2.0), OC.Op(-0.5)
    assert OC.count(a * b + c)["flop"] == 2
    assert OC.count((a + b) / c)["flop"] == 2
    assert OC.count(np.sqrt(np.array([a], dtype=object))[0] * b)["flop"] == 2
    s = a + b
    k = OC.count(s * s + s)          # s is computed once
    assert k["add"] == 2 and k["mul"] == 1 and k["flop"] == 3
    assert OC.count(-a * abs(b))["flop"] == 1     # sign operations are free


def test_literal_zeros_and_ones_and_untaken_branches_cost_nothing():
    a, b = OC.Op(3.0), OC.Op(4.0)
    assert OC.count(0.0 * a + 1.0 * b)["flop"] == 0
    assert OC.count((a * 0.0) / b, b * 1)["flop"] == 0
    x = OC.wrap([1.0, 2.0])
    y = np.where(np.array([True, False]), x * x, x + x)
    k = OC.count(y)
    assert k["mul"] == 1 and k["add"] == 1        # one element of each branch is used


def test_log_mean_series_form_count():
    """(a+b)/(2(1 + z^2/3 + z^4/5 + z^6/7)), z = (a-b)/(a+b), as the oracle writes it: z (a-b, a+b,
    a division: 3); z2 (1); z2/3 (1); z2*z2/5 (a product and a division: 2); z2*z2*z2/7 (two
    products and a division: 3); three sums; 2*(...) (1); the numerator a+b again (1); the final
    division (1): 16."""
    with OC.counting_numpy():
        a, b = OC.wrap([1.0]), OC.wrap([1.0 + 1e-6])
        k = OC.count(G.log_mean(a, b))
    assert k["flop"] == 16 and k.get("log", 0) == 0


def test_direct_form_is_counted_when_taken():
    with OC.counting_numpy():
        k = OC.count(G.log_mean(OC.wrap([1.0]), OC.wrap([2.0])))
    assert k["log"] == 1                           # log1p, no series terms
    assert k["flop"] < 10


@pytest.mark.parametrize("key", sorted(bench.ORACLE_OPS))
def test_bench_table_is_the_counters_output(key):
    p, viscous = key
    r = OC.unit_counts(p, viscous=viscous)
    assert bench.ORACLE_OPS[key] == (r["pair"]["flop"], r["rest_per_element"]["flop"])
