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
    assert "one GPU only" in msg["error"]


def test_code_digest_ignores_comments_not_code(tmp_path):
    a, b, c = tmp_path / "a.hip", tmp_path / "b.hip", tmp_path / "c.hip"
    a.write_text("int f(int x) {\n    return x + 1;\n}\n")
    b.write_text("// header\n/* block\n   comment */\nint f(int x) {  // trailing\n\n"
                 "    return x + 1;   \n}\n")
    c.write_text("int f(int x) {\n    return x + 2;\n}\n")
    assert bench.code_digest(str(a)) == bench.code_digest(str(b))
    assert bench.code_digest(str(a)) != bench.code_digest(str(c))


def test_counter_traffic_only_for_the_counted_code(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2112_07552_amd" / "csrc"
    profiles = tmp_path / "profiles"
    csrc.mkdir(parents=True)
    profiles.mkdir()
    src = csrc / "k.hip"
    src.write_text("__global__ void k() {}\n")
    (profiles / "counters.md").write_text(
        f"figures\n\ntraffic: gemm=123456 code_sha256={bench.code_digest(str(src))}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("counters.md", "gemm", "k.hip") == 123456
    assert bench.counter_traffic("counters.md", "other", "k.hip") is None
    src.write_text("__global__ void k() { int x = 0; }\n")   # the kernel changed
    assert bench.counter_traffic("counters.md", "gemm", "k.hip") is None
    assert bench.counter_traffic("missing.md", "gemm", "k.hip") is None


def test_launch_stats_average_and_rate():
    launches = [(2.0, 4e12, 8, 8, 8, 2), (4.0, 8e12, 8, 8, 8, 4)]
    st = bench.launch_stats(launches, 1e12, "tops")
    assert st["launches"] == 2 and st["avg_ms"] == 3.0
    assert st["avg_ops_per_launch"] == 6e12
    assert abs(st["achieved_tops"] - 12e12 / 6e-3 / 1e12) < 1e-9
    assert st["shapes_m_n_k_planes"] == [[8, 8, 8, 2], [8, 8, 8, 4]]
    assert bench.launch_stats([], 1e12, "tops") is None
