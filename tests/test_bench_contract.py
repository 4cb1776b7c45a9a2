"""CPU checks of the benchmark script's contract: one GPU only, and the
helper that finds when a method reaches a target."""

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_first_below_counts_iterations_done():
    trace = np.array([10.0, 7.0, 5.0, 5.0, 2.0])
    assert bench.first_below(trace, 10.0) == 0
    assert bench.first_below(trace, 5.0) == 2
    assert bench.first_below(trace, 4.0) == 4
    assert bench.first_below(trace, 1.0) is None


def test_code_digest_ignores_comments_and_spacing(tmp_path):
    a, b, c = tmp_path / "a.hip", tmp_path / "b.hip", tmp_path / "c.hip"
    a.write_text("int f(int x) {\n  return x + 1;  // one more\n}\n")
    b.write_text("/* a note */ int f(int x)\n{ return x + 1; }\n")
    c.write_text("int f(int x) { return x + 2; }\n")
    assert bench.code_digest([str(a)]) == bench.code_digest([str(b)])
    assert bench.code_digest([str(a)]) != bench.code_digest([str(c)])
