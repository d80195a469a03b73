"""Host-side parts of the bench.py contract (no GPU): it refuses more than one GPU with
a message, and the committed counter summary it reads is well formed."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_counter_summary_is_well_formed():
    path = os.path.join(ROOT, "profiles", "traffic_batched_pair_6x18x18x18.txt")
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    assert float(vals["fwd_pair_hbm_bytes_per_launch"]) > 0
    assert float(vals["bwd_pair_hbm_bytes_per_launch"]) > 0
    assert len(vals["kernel_source_sha256_16"]) == 16
