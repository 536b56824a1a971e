"""bench.py on the host (no GPU): the one-GPU contract and the helpers that
need no device."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in res.stderr and "--gpus 2" in res.stderr
    assert res.stdout.strip() == ""


def test_roofline_constants_and_traffic_record():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.HBM_PEAK_GBS == 8000.0
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    rec = json.load(open(os.path.join(ROOT, "profiles", "step_kernel_hbm_traffic.json")))
    for key in ("turbulent:0", "turbulent:1"):
        e = rec[key]
        # measured bytes per launch are at least the algorithmic ones, and the
        # record says which kernel source it was taken on
        assert e["bytes_per_launch"] >= e["algorithmic_read"] + e["algorithmic_write"]
        assert len(e["source_hash"]) == 16
    # the bench reports the counter bytes only for the source they were taken on
    t = bench.measured_traffic("turbulent", 0)
    assert t is None or t == rec["turbulent:0"]["bytes_per_launch"]
