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


def test_record_traffic_scales_counters_by_the_copy_calibration(tmp_path, monkeypatch):
    """bench.py --record-traffic (host only): per-dispatch FETCH_SIZE and
    WRITE_SIZE of the step kernel, each scaled by what it reads for the
    2 GiB copy, written under the current kernel-source hash; other kernels
    and counters in the files are ignored."""
    sys.path.insert(0, ROOT)
    import bench
    hdr = '"Kernel_Name","Counter_Name","Counter_Value"\n'

    def write(folder, rows):
        os.makedirs(tmp_path / folder)
        with open(tmp_path / folder / "c_counter_collection.csv", "w") as f:
            f.write(hdr + "".join(f'"{k}","{c}",{v}\n' for k, c, v in rows))
    gib2 = 2048 * 1024  # KiB in 2 GiB
    write("copyf", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", gib2 / 2), ("k_other", "FETCH_SIZE", 1.0)])
    write("copyw", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", gib2)])
    step = "void lbm::k_step<float, 512, false>(lbm::Geom, ...)"
    write("fetch0", [(step, "FETCH_SIZE", 1000.0), (step, "FETCH_SIZE", 3000.0),
                     ("void lbm::k_stream_copy<float, 512>(...)", "FETCH_SIZE", 99.0)])
    write("write0", [(step, "WRITE_SIZE", 500.0)])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    src = os.path.join(ROOT, "paper_2405_12082_amd", "csrc")
    os.makedirs(tmp_path / "paper_2405_12082_amd")
    os.symlink(src, tmp_path / "paper_2405_12082_amd" / "csrc")
    rec = bench.record_traffic(str(tmp_path), "laminar", 0)
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0 and rec["dispatches"] == 2
    assert rec["read_bytes"] == 2000 * 1024 * 2 and rec["write_bytes"] == 500 * 1024
    assert rec["bytes_per_launch"] == rec["read_bytes"] + rec["write_bytes"]
    assert rec["algorithmic_read"] == 15168 * 27 * 4  # the laminar pipe's fluid nodes, FP32
    stored = json.load(open(tmp_path / "profiles" / "step_kernel_hbm_traffic.json"))["laminar:0"]
    assert stored == rec and stored["source_hash"] == bench.kernel_source_hash()
