"""Pin: the memory-optimised tableaux derived in exact arithmetic from the
standard Heun-3, classic RK4 and Cash-Karp tableaux equal the values printed
in App. A (tests/golden/modified_tableaux.txt)."""
import os
from fractions import Fraction

import pytest

from oracle import tableau

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "modified_tableaux.txt")


def _read_golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            meth, kind, row, vals = line.split()
            vals = [Fraction(v) for v in vals.split(",")]
            out.setdefault(meth, {"a*": {}, "b*": None})
            if kind == "a*":
                out[meth]["a*"][int(row)] = vals
            else:
                out[meth]["b*"] = vals
    return out


@pytest.mark.parametrize("name,fn", [("RKHE3", tableau.heun3), ("RK4", tableau.rk4), ("RKCK", tableau.cash_karp5)])
def test_derived_tableau_equals_printed(name, fn):
    gold = _read_golden()[name]
    a_star, b_star = tableau.modified_tableau(*fn())
    assert len(a_star) == len(gold["a*"])
    for i, row in enumerate(a_star, start=1):
        assert row == gold["a*"][i]
    assert b_star == gold["b*"]


def test_standard_tableaux_are_consistent():
    """Row sums give c_i, and b sums to one (first-order condition)."""
    for fn in (tableau.heun3, tableau.rk4, tableau.cash_karp5):
        A, b = fn()
        assert sum(b) == 1
        for i, row in enumerate(A):
            assert sum(row[:i]) == sum(row)
