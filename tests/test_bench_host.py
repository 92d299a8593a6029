"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic byte
counts of a round's phases, the roofline record and the traffic summaries'
source-hash gate."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_no_timed_steps_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "0"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "--steps" in r.stderr


def test_phase_bytes_by_hand():
    st = {"boundary": 2, "active_pins": 5, "candidates": 1, "approved": 1, "moved_pins": 3,
          "touched_nets": 4, "touched_pins": 9}
    # n/8 + 16 per active vertex + (12 + 4 ceil(k/32)) per active incidence + 16 per candidate
    assert bench.select_bytes(st, 64, 16) == 8 + 32 + 5 * 16 + 16
    assert bench.select_bytes(st, 64, 64) == 8 + 32 + 5 * 20 + 16
    assert bench.approve_bytes(st, 64, 16) == 32 + 20 + 60
    assert bench.finalize_bytes(st, 64, 16) == 32 + 36 + 8


def test_roofline_record():
    r = bench.roofline_of("x", 8e9, 1000.0)       # 8 GB in one second
    assert r["achieved"] == pytest.approx(8.0)
    assert r["frac"] == pytest.approx(8.0 / bench.HBM_PEAK_GBS)
    assert r["unit"] == "GB/s" and r["bound"] == "hbm"


def _profile(tmp_path, sources, digest, value=123456):
    text = ("select_traffic_bytes_per_launch: %d\nselect_sources: %s\n"
            "select_sources_sha256: %s\n" % (value, sources, digest))
    (tmp_path / "p.md").write_text(text)


def test_traffic_gate(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    rel = "paper_2010_10272_amd/csrc/hg_lp.hip"
    digest = hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest()
    _profile(tmp_path, rel, digest)
    assert bench.measured_traffic("p.md", "select") == 123456.0
    _profile(tmp_path, rel, "0" * 64)                 # sources changed since the counters
    assert bench.measured_traffic("p.md", "select") is None
    _profile(tmp_path, "no/such/file.hip", digest)
    assert bench.measured_traffic("p.md", "select") is None
    assert bench.measured_traffic("missing.md", "select") is None
    assert bench.measured_traffic("p.md", "approve") is None


@pytest.mark.parametrize("profile", ["plain_vlsi_traffic.md", "plain_sparse_matrix_traffic.md"])
def test_committed_traffic_summaries_parse(profile):
    """Each committed summary records the three phases' bytes and their
    sources; the figures are positive wherever the hash still matches."""
    text = open(os.path.join(ROOT, "profiles", profile)).read()
    for prefix in ("select", "approve", "finalize"):
        assert prefix + "_traffic_bytes_per_launch:" in text
        assert prefix + "_sources_sha256:" in text
        v = bench.measured_traffic(profile, prefix)
        assert v is None or v > 0
