"""bench.py's command-line contract on the host (no GPU needed): more than one
GPU is refused with a JSON message and a non-zero status before anything
touches a device."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    for n in (2, 8):
        p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                           capture_output=True, text=True, timeout=120, cwd=ROOT)
        assert p.returncode != 0
        line = json.loads(p.stdout.strip().splitlines()[-1])
        assert line["n_gpus"] == n
        assert "one GPU" in line["error"]
