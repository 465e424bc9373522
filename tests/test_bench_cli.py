"""The benchmark's command line, checked on the host: it measures one GPU and
says so for any other count, before it touches a device."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n), "--steps", "1",
                        "--warmup", "0"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = r.stdout + r.stderr
    assert f"--gpus {n}" in msg and "one GPU" in msg
