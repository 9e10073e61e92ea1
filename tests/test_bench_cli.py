"""Host-side behaviour of bench.py that needs no GPU: it refuses more than
one GPU with an explanation, and its oracle-only child (the one-thread CPU
baseline) prints one JSON record with the fields the baseline reports."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_oracle_only_record():
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--oracle-only", "--cpu-n", "64",
                        "--cpu-seconds", "0.2"], capture_output=True, text=True, timeout=300, env=env, check=True)
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["kind"] == "oracle" and rec["unit"] == "cell-updates/s" and rec["cores"] == 1
    assert rec["value"] > 0 and "64^2" in rec["sample"]
