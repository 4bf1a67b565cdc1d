"""Host-side checks of bench.py (no GPU): the one-GPU guard and the HBM
traffic figure it reads from the committed counter summary."""
import hashlib
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

TRAFFIC = os.path.join(ROOT, "profiles", "k_sym_forces_n100000_traffic.json")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_summary_is_of_the_current_pair_kernel():
    # the bench reports the counters' traffic only while pairs.hip is the
    # source they were taken on; the committed summary must be that source's
    d = json.load(open(TRAFFIC))
    src = open(os.path.join(ROOT, "paper_2609_24722_amd", "csrc", "pairs.hip"), "rb").read()
    assert d["pairs_hip_sha256"] == hashlib.sha256(src).hexdigest()
    assert bench.traffic_from_profiles() == d["traffic_bytes_per_launch"]


def test_traffic_summary_arithmetic():
    # counters in KiB per dispatch, each scaled by what the same counter read
    # for a plain copy of known size (bytes read and written once each)
    d = json.load(open(TRAFFIC))
    probe = d["copy_probe_bytes"]
    assert d["fetch_scale"] == pytest.approx(probe / (d["copy_probe_fetch_kib"] * 1024), rel=1e-12)
    assert d["write_scale"] == pytest.approx(probe / (d["copy_probe_write_kib"] * 1024), rel=1e-12)
    rd = d["fetch_kib_per_dispatch"] * 1024 * d["fetch_scale"]
    wr = d["write_kib_per_dispatch"] * 1024 * d["write_scale"]
    assert d["read_bytes_per_launch"] == pytest.approx(rd, rel=1e-12)
    assert d["write_bytes_per_launch"] == pytest.approx(wr, rel=1e-12)
    assert d["traffic_bytes_per_launch"] == pytest.approx(rd + wr, rel=1e-12)


def test_traffic_is_null_once_the_kernel_changes(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_2609_24722_amd" / "csrc").mkdir(parents=True)
    shutil.copy(TRAFFIC, tmp_path / "profiles")
    src = open(os.path.join(ROOT, "paper_2609_24722_amd", "csrc", "pairs.hip"), "rb").read()
    (tmp_path / "paper_2609_24722_amd" / "csrc" / "pairs.hip").write_bytes(src + b"\n// edited\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profiles() is None
    (tmp_path / "paper_2609_24722_amd" / "csrc" / "pairs.hip").write_bytes(src)
    assert bench.traffic_from_profiles() is not None
