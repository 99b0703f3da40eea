"""The contraction's split-count rule (host logic, no GPU): tests/c/split_rule.cpp builds
against the library's own header and checks the straggler-round cases of the o=48
v=768 naux=2304 ladder and the rule's properties over a sweep of launch shapes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_split_rule(tmp_path):
    exe = tmp_path / "split_rule"
    cmd = ["hipcc", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "split_rule.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "split rule ok" in run.stdout
