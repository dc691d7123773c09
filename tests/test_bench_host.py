"""Host-side logic of bench.py (CPU only): the one-GPU rule and the lookup
of measured HBM traffic, which must go null once a kernel's source or the
persistent-plan shape no longer matches the counters' run."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.fixture
def records(tmp_path, monkeypatch):
    src = bench.KERNEL_SOURCES["k_tile_round"]
    rec = {"reg3_maxcut": {"k_tile_round": {"hbm_bytes_per_launch": 1234, "source_sha256": bench.source_sha256(src),
                                            "tile": "1,1024,1,0,3"}},
           "torus1m_maxcut": {"k_pga_step": {"hbm_bytes_per_launch": 99, "source_sha256": "0" * 64}}}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    return rec


def test_traffic_found_for_the_same_source_and_shape(records):
    assert bench.measured_traffic("reg3_maxcut", "k_tile_round", "1,1024,1,0,3") == 1234
    assert bench.measured_traffic("reg3_maxcut", "k_tile_round") == 1234


def test_traffic_null_for_another_shape(records):
    assert bench.measured_traffic("reg3_maxcut", "k_tile_round", "16,1024,4,0,0") is None


def test_traffic_null_once_the_source_changed(records):
    assert bench.measured_traffic("torus1m_maxcut", "k_pga_step") is None


def test_traffic_null_without_a_record(records):
    assert bench.measured_traffic("er1m_mis", "k_pga_step") is None


def test_committed_records_name_known_kernels():
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as f:
        recs = json.load(f)
    for wl, kernels in recs.items():
        for k, rec in kernels.items():
            assert bench.KERNEL_SOURCES[k] == rec["source"]
            assert rec["hbm_bytes_per_launch"] > 0
            # a warm-up run fills the tuning cache, then the counter run
            assert rec["command_fetch"].startswith("cd /tmp && export TMPDIR=/tmp")
            assert " && rocprofv3 --pmc FETCH_SIZE -d " in rec["command_fetch"]
            assert " && rocprofv3 --pmc WRITE_SIZE -d " in rec["command_write"]
            if k == "k_tile_round":
                assert len(rec["tile"].split(",")) == 6
