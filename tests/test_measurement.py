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


def test_alone_average_leaves_out_concurrent_launches(tmp_path):
    # A runs alone twice (10 and 30 ns); B overlaps C (two streams) and once runs alone
    rows = [("A", 0, 10), ("B", 20, 40), ("C", 30, 50), ("A", 60, 90), ("B", 100, 104)]
    f = tmp_path / "trace.csv"
    f.write_text("Kernel_Name,Start_Timestamp,End_Timestamp\n" +
                 "".join(f"{n},{s},{e}\n" for n, s, e in rows))
    assert RS.alone_avg_ns(str(f), "A") == 20.0
    assert RS.alone_avg_ns(str(f), "B") == 4.0
    with pytest.raises(SystemExit):
        RS.alone_avg_ns(str(f), "C")


def test_alone_by_grid_groups_dispatches_by_grid(tmp_path):
    rows = [("K", 0, 10, 64), ("K", 20, 50, 128), ("J", 40, 60, 64), ("K", 70, 80, 64), ("K", 90, 96, 128)]
    f = tmp_path / "trace.csv"
    f.write_text("Kernel_Name,Start_Timestamp,End_Timestamp,Grid_Size_X\n" +
                 "".join(f"{n},{s},{e},{g}\n" for n, s, e, g in rows))
    res = RS.alone_by_grid_us(str(f), "K")
    assert res == {64: (2, 0.01, 0.01), 128: (1, 0.006, 0.006)}


def test_clock_rows_derive_clock_and_issue_rate(tmp_path):
    """GRBM_GUI_ACTIVE summed over 8 XCDs over a 1 ms dispatch of 2.4e6 cycles
    per XCD is 2.4 GHz; 0.25 instructions per SIMD per cycle over 1024 SIMDs
    is 0.25 * 1024 * 2.4e6 VALU instructions.  A 10 us dispatch is left out."""
    hdr = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value,Start_Timestamp,End_Timestamp\n"
    rows = [
        "1,kern,GRBM_GUI_ACTIVE,%d,0,1000000" % (8 * 2400000),
        "1,kern,SQ_INSTS_VALU,%d,0,1000000" % int(0.25 * 1024 * 2400000),
        "2,kern,GRBM_GUI_ACTIVE,%d,2000000,3000000" % (8 * 2200000),
        "2,kern,SQ_INSTS_VALU,%d,2000000,3000000" % int(0.25 * 1024 * 2200000),
        "3,short,GRBM_GUI_ACTIVE,999999,5000000,5010000",
    ]
    (tmp_path / "pmc_counter_collection.csv").write_text(hdr + "\n".join(rows) + "\n")
    res = RS.clock_rows(str(tmp_path))
    assert set(res) == {"kern"}
    n, ghz, ipc = res["kern"]
    assert n == 2 and ghz == pytest.approx(2.3) and ipc == pytest.approx(0.25)
