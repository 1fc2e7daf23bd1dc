"""Host logic of bench.py (CPU only): the one-GPU guard and the rule that the
HBM traffic figure comes only from a counter summary of the current kernels."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def write_summary(path, sha, hbm="9.5e+08"):
    with open(path, "w") as fh:
        fh.write("# rocprofv3 --pmc summary\n# command: x\n")
        fh.write(f"hbm_bytes_per_launch: {hbm}\n")
        fh.write(f"kernel_source_sha256: {sha}\n")


@pytest.fixture
def profiles(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    return tmp_path


def test_traffic_read_when_hash_matches(profiles):
    write_summary(profiles / "k_stream_w_counters.txt", bench.kernel_source_hash(), "9.5e+08")
    assert bench.read_traffic("w") == pytest.approx(9.5e8)


def test_traffic_null_when_kernel_changed(profiles):
    write_summary(profiles / "k_stream_w_counters.txt", "0" * 64)
    assert bench.read_traffic("w") is None


def test_traffic_null_when_missing_or_malformed(profiles):
    assert bench.read_traffic("absent") is None
    write_summary(profiles / "k_stream_w_counters.txt", bench.kernel_source_hash(), "not-a-number")
    assert bench.read_traffic("w") is None


def test_committed_counter_summary_parses():
    """The committed Mach-3 summary holds the fields bench.py reads."""
    path = os.path.join(ROOT, "profiles", "k_stream_shock_m3_fp32_counters.txt")
    kv = dict(line.split(":", 1) for line in open(path) if ":" in line and not line.startswith("#"))
    assert float(kv["hbm_bytes_per_launch"]) > 0
    assert len(kv["kernel_source_sha256"].strip()) == 64


def test_bytes_per_update():
    assert bench.bytes_per_update("fp32") == 8
    assert bench.bytes_per_update("fp64") == 16
