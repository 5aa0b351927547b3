"""CPU checks of bench.py's contract that need no GPU: it refuses more than one GPU with a
message (there is no multi-GPU path), and its CPU baseline is the oracle timed on a bounded
sample, reported with the fields the result line carries.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import kfbi_inputs as KI


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_cpu_baseline_fields():
    import bench
    cb = bench.cpu_baseline(KI.WORKLOADS["sphere32"].with_N(16), 20, calib_N=16)
    assert cb["kind"] == "oracle" and cb["unit"] == "evals/s"
    assert cb["value"] > 0 and cb["cores"] >= 1
    assert "Schur-complement applications" in cb["sample"]
    c = cb["calibration"]
    assert c["factor"] > 0 and abs(cb["value"] * c["factor"] - cb["extrapolated_value"]) < 1e-9 * cb["extrapolated_value"]
