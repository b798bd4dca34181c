"""Admission control of the sort server, on the CPU (host code only)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_admission_and_arena(tmp_path):
    exe = tmp_path / "check"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Xlinker", "--no-as-needed",
                           "-I", os.path.join(ROOT, "paper_1403_2056_amd", "csrc"),
                           os.path.join(ROOT, "tests", "serving_host_check.cpp"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ALL OK" in out.stdout
