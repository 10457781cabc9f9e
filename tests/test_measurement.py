"""The measurement helpers against the paper's own numbers: aggregating two
kernels' issue-slot utilisation over their back-to-back run, weighted by their
elapsed times, reproduces the Native column of the paper's Table II from its
Table I (tests/golden/paper_issue_slot_tables.txt) within 3 points for all 16
pairs on both GPUs (the paper weighs by elapsed cycles, which differ slightly
from the printed milliseconds)."""
import os

import pytest

from paper_2007_01277_amd import rocprof_summary as RS

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_issue_slot_tables.txt")


def _tables():
    t1, t2 = {}, {}
    for ln in open(GOLD):
        f = ln.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "T1":
            t1[f[1]] = tuple(map(float, f[2:6]))
        else:
            t2[f[1]] = tuple(map(float, f[2:4]))
    return t1, t2


T1, T2 = _tables()


@pytest.mark.parametrize("pair", sorted(T2))
def test_time_weighted_issue_slots_reproduce_table_ii_native(pair):
    a, b = pair.split("+")
    for g in (0, 1):  # 1080 Ti, V100
        agg = RS.time_weighted([T1[a][2 + g], T1[b][2 + g]], [T1[a][g], T1[b][g]])
        assert abs(agg - T2[pair][g]) <= 3.0, (pair, g, agg, T2[pair][g])


def test_time_weighted_basics():
    assert RS.time_weighted([50.0, 50.0], [1.0, 3.0]) == 50.0
    assert RS.time_weighted([100.0, 0.0], [1.0, 3.0]) == 25.0
