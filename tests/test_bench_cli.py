"""bench.py's command-line contract on the CPU: a request for more than one
GPU is refused with a JSON message and a non-zero status, before any device
work."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1",
                        "--warmup", "0"], capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    line = [l for l in r.stdout.splitlines() if l.strip().startswith("{")][-1]
    msg = json.loads(line)
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
