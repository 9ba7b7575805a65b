"""Host-side parts of bench.py (no GPU): the one-GPU contract, the byte model
the oracle's rate is quoted on, the traffic record's guards and the
comment-blind source hash."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_byte_model():
    # fused pipeline: 186 half-spectrum fields per MHD step, 93 per NS step
    sc64 = 512 * 512 * 257 * 16.0
    assert bench.model_step_bytes(512, 6) == pytest.approx(186 * sc64)
    assert bench.model_step_bytes(512, 3) == pytest.approx(93 * sc64)
    assert bench.model_step_bytes(256, 3, real_bytes=4) == pytest.approx(93 * 256 * 256 * 129 * 8.0)


def test_code_only_ignores_comments_and_spacing():
    a = "int x = 1; // one\n/* block\n comment */ int y;"
    b = "int x = 1;\n\n   int y;  // another"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only("int x = 1;") != bench._code_only("int x = 2;")


def test_traffic_guards(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"mhd512/f32/x_prod": {"kernel": "k", "bytes_per_launch": 123.0,
                                 "src_hash": bench.src_hash(), "pipe": 4}}
    (prof / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "src_hash", lambda: rec["mhd512/f32/x_prod"]["src_hash"])
    assert bench.load_traffic("x_prod", "mhd512", "f32", {"pipe": 4}) == 123.0
    # taken in another slab setting, for another kind, or from other sources: no figure
    assert bench.load_traffic("x_prod", "mhd512", "f32", {"pipe": 0}) is None
    assert bench.load_traffic("y_inv", "mhd512", "f32", {"pipe": 4}) is None
    monkeypatch.setattr(bench, "src_hash", lambda: "other")
    assert bench.load_traffic("x_prod", "mhd512", "f32", {"pipe": 4}) is None


def test_host_info_fields():
    info = bench.host_info()
    assert info["nproc"] >= 1 and "MemTotal_GB" in info


def test_pipe_slabs():
    # in order or over three helper streams: 2^pipe; two chains: 2^(pipe - 3);
    # never more slabs than planes
    assert [bench.pipe_slabs(v, 512) for v in range(10)] == [1, 2, 4, 8, 16, 32, 64, 16, 32, 64]
    assert bench.pipe_slabs(6, 24) == 24 and bench.pipe_slabs(9, 24) == 24
