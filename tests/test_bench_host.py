"""Host-side logic of bench.py (no GPU): the single-GPU guard, the code
digest that ties counter figures to kernel code, and the traffic lookup."""
import json
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
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "single-GPU" in msg["error"]


def test_code_digest_ignores_comments_not_code(tmp_path):
    a, b, c = tmp_path / "a.hip", tmp_path / "b.hip", tmp_path / "c.hip"
    a.write_text("int f(int x) {\n    return x + 1;\n}\n")
    b.write_text("// header\n/* block\n   comment */\nint f(int x) {  // trailing\n\n"
                 "    return x + 1;   \n}\n")
    c.write_text("int f(int x) {\n    return x + 2;\n}\n")
    assert bench.code_digest(str(a)) == bench.code_digest(str(b))
    assert bench.code_digest(str(a)) != bench.code_digest(str(c))


def test_counter_traffic_only_for_the_counted_code(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("__global__ void k() {}\n")
    prof = tmp_path / "counters.md"
    prof.write_text(f"figures\n\ntraffic: nn_bytes=123456 code_sha256={bench.code_digest(str(src))}\n")
    monkeypatch.setattr(bench, "GEMM_SOURCE", str(src))
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(prof))
    assert bench.counter_traffic() == 123456
    src.write_text("__global__ void k() { int x = 0; }\n")   # the kernel changed
    assert bench.counter_traffic() is None
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(tmp_path / "missing.md"))
    assert bench.counter_traffic() is None


def test_committed_counters_name_a_digest():
    text = open(bench.COUNTERS_FILE).read()
    assert "traffic: nn_bytes=" in text and "code_sha256=" in text
