"""Precision of the storage forms against the FP64 reference, per result
(needs an MI355X).  The 64x64x256 precision pipe (R = 30) runs 5000 steps in
FP64 (reference, tied to the FP64 oracle at step 100), FP32 and FP16 storage.
Errors: relative max norms (velocity; mean and rms profiles over the second
half, sampled every 100 steps) and absolute differences (skewness,
flatness); the FP64 run's FP64 sums (mass, momentum, energy) meet the
oracle's at rounding level.

Stated accuracy, asserted below:
 * velocity after 100 steps within the storage's own precision: 1e-5 for
   FP32 (the velocity target of the laminar case), 1e-3 for FP16 (deviations
   with 11 significant bits); at most linear growth after that (10x at 1000
   steps: the FP32 drift is linear in the steps);
 * the statistics, for both storage forms, at the resolution of a profile
   figure: mean within 0.5%, rms within 2% of the profile's maximum,
   skewness within 0.05 and flatness within 0.1 (absolute).
FP16 meets them because it stores each value relative to its column's
initial equilibrium (the codec in include/lbm.h); stored relative to the
lattice weights alone it missed them by 10-50x (rms 23%, skewness 1.1,
flatness 2.4)."""
import sys

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

VELOCITY = {"fp32": (1e-5, 1e-4), "fp16": (1e-3, 1e-2)}
STATISTICS = {"mean_profile": 5e-3, "rms_profile": 2e-2, "skewness_profile_abs": 0.05, "flatness_profile_abs": 0.1}


def test_storage_precision_per_result(oracle_mod):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    r = bench.run_precision()
    print({k: v for k, v in r.items() if k != "reference_profiles"}, flush=True)
    sys.stdout.flush()
    assert r["fp64_gpu_vs_oracle_velocity"]["step_100"] < 3e-7  # through the FP32 export
    sums = r["fp64_gpu_vs_oracle_sums"]  # FP64 throughout: rounding level
    assert sums["mass"] < 1e-12 and sums["momentum"] < 1e-10 and sums["energy"] < 1e-10
    for name, (v100, v1000) in VELOCITY.items():
        res = r[name]
        assert res["state_finite"], name
        assert res["velocity_step_100"] < v100, (name, res)
        assert res["velocity_step_1000"] < v1000, (name, res)
        for key, bound in STATISTICS.items():
            assert res[key] < bound, (name, key, res)
