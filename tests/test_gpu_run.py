"""Long runs (paper_2405_12082_amd.run): sampling schedule and
radial statistics against u_z taken directly from the stepped state (needs
an MI355X)."""
import numpy as np
import pytest

import lbm_inputs as LI

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_12082_amd as P
    P.lib()
    return P


def test_run_statistics_match_sampled_velocity(P):
    from paper_2405_12082_amd import run
    lines = []
    res = run.run("precision_ref", 400, 200, every=100, progress=200, log=lines.append)
    assert res["samples"] == 3 and len(lines) == 2
    prof = res["profiles"]
    cfg = LI.preset("precision_ref")
    p = P.Pipe(cfg, LI.preset_amplitudes(cfg))
    nx, ny, nz = LI.dims_of(cfg)
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = np.hypot(xx - 0.5 * (nx - 1), yy - 0.5 * (ny - 1))
    fluid = r < cfg["radius"]
    nb = len(prof["r"])
    idx = np.minimum(r.astype(int), nb - 1)
    s1 = np.zeros(nb)
    cnt = np.zeros(nb)
    for target in (200, 300, 400):
        p.step(target - p.step_index)
        uz = p.moments()[1][0, 2].cpu().numpy().astype(np.float64)  # [nz][ny][nx]
        for b in range(nb):
            sel = fluid & (idx == b)
            s1[b] += uz[:, sel].sum()
            cnt[b] += nz * sel.sum()
    mean = np.where(cnt > 0, s1 / np.maximum(cnt, 1), 0.0)
    np.testing.assert_allclose(prof["count"], cnt)
    np.testing.assert_allclose(prof["mean"], mean, rtol=1e-6, atol=1e-9)
    nu = (cfg["tau"] - 0.5) / 3.0
    np.testing.assert_allclose(prof["y_plus"], (cfg["radius"] - np.asarray(prof["r"])) * cfg["u_tau"] / nu)


def test_run_records_the_dominant_mode_series(P):
    """Modes every 20 steps from step 200 (11 samples): the series equals the
    dominant modes found by sampling a second pipe at the same steps, and the
    statistics are those of the host functions on that series."""
    from paper_2405_12082_amd import run, structures as H
    res = run.run("precision_ref", 400, 200, every=100, progress=200, log=lambda s: None, modes_every=20,
                  modes_from=200, ntheta=256, mmax=10)
    m = res["modes"]
    assert len(m["series"]) == 11
    cfg = LI.preset("precision_ref")
    p = P.Pipe(cfg, LI.preset_amplitudes(cfg))
    ref = []
    for target in range(200, 401, 20):
        p.step(target - p.step_index)
        _, _, dom = p.ring_spectrum(p.ring_sample(0.78 * cfg["radius"], 256), 10)
        ref.append(int(dom.cpu()[0]))
    assert m["series"] == ref
    if min(ref) >= 1:
        np.testing.assert_allclose(m["transition_matrix"], H.transition_matrix(ref, 10))


def test_run_save_resume_continues_bitwise(P, tmp_path):
    """400 steps in one process equal 200 steps, an archive, and 200 more
    resumed from it: the state bitwise, the sample count and mode series
    exactly, the statistics to FP64 rounding (the resumed run adds the
    archived sums on the host)."""
    from paper_2405_12082_amd import run
    kw = dict(every=100, progress=200, log=lambda s: None, modes_every=20, modes_from=200, ntheta=256, mmax=10)
    whole = run.run("precision_ref", 400, 100, save=str(tmp_path / "whole.npz"), **kw)
    run.run("precision_ref", 200, 100, save=str(tmp_path / "half.npz"), out_path=str(tmp_path / "part.json"),
            partial_every=100, **dict(kw, progress=100))
    import json
    part = json.load(open(tmp_path / "part.json"))  # written at step 100 (the last one is the caller's)
    assert part["steps_done"] == 100 and part["samples"] == 1 and len(part["profiles"]["mean"]) > 0
    resumed = run.run("precision_ref", 400, 100, resume=str(tmp_path / "half.npz"),
                      save=str(tmp_path / "resumed.npz"), **kw)
    with pytest.raises(ValueError, match="another configuration"):
        run.run("precision_ref", 400, 100, resume=str(tmp_path / "half.npz"), **dict(kw, every=50))
    a, b = np.load(tmp_path / "whole.npz"), np.load(tmp_path / "resumed.npz")
    assert int(a["step"]) == int(b["step"]) == 400
    assert np.array_equal(a["state"], b["state"])
    assert resumed["samples"] == whole["samples"] == 4
    assert resumed["modes"]["series"] == whole["modes"]["series"]
    np.testing.assert_allclose(b["profile"], a["profile"], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(resumed["modes"]["mean_spectrum"], whole["modes"]["mean_spectrum"], rtol=1e-12)
    for key in ("mean", "rms"):
        np.testing.assert_allclose(resumed["profiles"][key], whole["profiles"][key], rtol=1e-10, atol=1e-15)


def test_run_fp16_spinup_hands_over_the_state(P):
    """An FP16 spin-up of 210 steps (not a multiple of the sampling
    interval), then FP32: the handed-over state is the FP16 run's (the first
    FP32 diagnostics equal the FP16 run's mass to FP32 rounding of the
    export), the sampling steps are still reached, and the run stays finite
    with its mass kept."""
    from paper_2405_12082_amd import run
    lines = []
    res = run.run("precision_ref", 400, 300, every=100, progress=100, log=lines.append,
                  spinup_steps=210, spinup_storage=1)
    import json
    recs = [json.loads(s) for s in lines]
    spin = [r for r in recs if "spinup_step" in r]
    main = [r for r in recs if "step" in r]
    assert [r["spinup_step"] for r in spin] == [100, 200, 210]
    assert [r["step"] for r in main] == [300, 400]
    assert all(r["non_finite"] == 0 for r in recs)
    assert abs(main[0]["mass"] - spin[-1]["mass"]) < 1e-6
    assert res["samples"] == 2
