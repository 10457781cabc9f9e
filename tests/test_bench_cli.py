"""Host-side checks of bench.py: the one-GPU contract and the counter records
that the bench line reports only while they match the kernel sources."""
import json
import os
import subprocess
import sys

import bench
from paper_2007_01277_amd import rocprof_summary as RS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profile_records_are_used_only_for_the_current_kernel_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"fused_x": {"csrc_hash": RS.csrc_hash(), "hbm_bytes_per_launch": 123, "VALUBusy": 50.0,
                       "native_VALUBusy": 40.0},
           "fused_old": {"csrc_hash": "0" * 16, "hbm_bytes_per_launch": 7, "VALUBusy": 1.0}}
    (prof / "traffic.json").write_text(json.dumps(rec))
    (prof / "counters.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profiles("fused_x") == 123
    assert bench.valu_busy_from_profiles("fused_x") == 50.0
    assert bench.valu_busy_from_profiles("fused_x", native=True) == 40.0
    assert bench.traffic_from_profiles("fused_old") is None
    assert bench.valu_busy_from_profiles("fused_old") is None
    assert bench.traffic_from_profiles("missing") is None


def test_alu_roofline_constants():
    # 256 CUs x 64 lanes x 2.4 GHz, and eight VALU instructions per int_mix round
    assert abs(bench.INT_PEAK_TOPS - 39.3216) < 1e-9
    assert bench.OPS_PER_ROUND == 8
    assert bench.HBM_PEAK_GBS == 8000


def test_ratio_sweep_sets():
    from paper_2007_01277_amd import ratio_sweep as RSW
    assert RSW.parse_sets("paper,memmem") == {"data", "crypto", "memmem"}
    assert RSW.parse_sets("crypto") == {"crypto"}
    assert RSW.parse_sets("data, memmem") == {"data", "memmem"}
    import pytest
    with pytest.raises(SystemExit):
        RSW.parse_sets("hashes")
