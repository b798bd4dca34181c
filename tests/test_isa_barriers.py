"""The HIP kernels compile for gfx950 with every barrier-carrying loop closed
by a lane-uniform back edge (see isa_barriers.py)."""
import os
import shutil
import subprocess

import pytest

from tests import isa_barriers

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("/opt/rocm/bin/hipcc") is None, reason="hipcc not installed")
def test_no_barrier_in_lane_divergent_loop(tmp_path):
    from paper_1403_2056_amd import build
    out = tmp_path / "ssort.s"
    cmd = [build.HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", build.INCLUDE, "-I", build.CSRC, "-S", "--cuda-device-only", "-o", str(out),
           os.path.join(build.CSRC, "ssort_api.hip")]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    lines = out.read_text().splitlines()
    kernels = list(isa_barriers.kernels(lines))
    assert len(kernels) >= 10
    bad = {k: b for k, body in kernels if (b := isa_barriers.check(body))}
    assert not bad, bad
    names = " ".join(k for k, _ in kernels)
    assert "k_worker" in names
