"""Long runs of a pipe preset with turbulence statistics.

    python -m paper_2405_12082_amd.run --preset paper --steps 300000 \\
        --stats-from 200000 --every 100 --out run.json

Steps the pipe with graph replays of ``every`` steps, accumulates the FP64
per-column power sums of u_z at every ``every``-th step from ``stats_from``
on (Eq. (urmsformula): pooled over time, azimuth and z per radial bin), and
prints one JSON progress line per ``progress`` steps (mass, mean streamwise
velocity, energy, throughput).  The result holds the radial profiles of
mean, rms, skewness and flatness of u_z, also in wall units (y+ = (R - r)
u*/nu, U+ = U/u*), with the run's parameters.  The paper's own run is 30
T^LET with statistics over the last 10 T^LET, sampled every 100 steps
(Section II.B).  With ``--modes-every`` the dominant azimuthal mode of the
correlation on r = 0.78 R (Section II.C) is found on the GPU every that many
steps; the series, its transition matrix, the Chapman-Kolmogorov test, the
self mode correlation and Taylor lengths (Section III; the paper samples
every 20 steps over the last 10 T^LET) go into the result.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def run(preset: str, steps: int, stats_from: int, every: int = 100, progress: int = 10000,
        storage: int = 0, wall: int | None = None, log=print, modes_every: int = 0, modes_from: int = 0,
        r0_frac: float = 0.78, ntheta: int = 1024, mmax: int = 10) -> dict:
    import math

    import torch

    import lbm_inputs as LI
    from . import structures as H
    from .pipe import Pipe, radial_profiles

    cfg = LI.preset(preset)
    cfg["storage"] = storage
    if wall is not None:
        cfg["wall"] = wall
    amps = LI.preset_amplitudes(cfg)
    if every < 2 or every % 2:
        raise ValueError("every must be an even number >= 2 (graph replays of that many steps)")
    if modes_every and (modes_every < 2 or modes_every % 2):
        raise ValueError("modes_every must be an even number >= 2")
    # one graph length for the whole run: a divisor of every sampling interval
    chunk = math.gcd(every, modes_every) if modes_every else every
    p = Pipe(cfg, amps)
    nf = p.n_fluid
    nu = (cfg["tau"] - 0.5) / 3.0
    p.profile_reset()
    samples = 0
    r0 = r0_frac * cfg["radius"]
    ring = None
    dominant, spec_sum = [], None
    t0 = time.perf_counter()
    last_t, last_n = t0, 0
    n = 0
    while n < steps:
        k = min(chunk, steps - n)
        if k == chunk:
            p.step_graph(k, chunk)
        else:
            p.step(k)
        n += k
        if n >= stats_from and n % every == 0:
            p.profile_accumulate()
            samples += 1
        if modes_every and n >= modes_from and n % modes_every == 0:
            ring = p.ring_sample(r0, ntheta, out=ring)
            _, mean, dom = p.ring_spectrum(ring, mmax)
            dominant.append(dom)
            spec_sum = mean if spec_sum is None else spec_sum + mean
        if n % progress == 0 or n == steps:
            d = p.diagnostics()[0]
            torch.cuda.synchronize()
            now = time.perf_counter()
            rec = {"step": n, "elapsed_s": round(now - t0, 1),
                   "mlups": round(nf * (n - last_n) / max(now - last_t, 1e-9) / 1e6, 1),
                   "mass": d[0] / nf, "mean_uz": d[3] / d[0], "energy": float(p.energy()[0]),
                   "non_finite": int(d[4]), "samples": samples}
            log(json.dumps(rec))
            last_t, last_n = now, n
            if d[4] != 0 or not np.isfinite(d[0]):
                raise FloatingPointError(f"non-finite populations at step {n}")
    prof = radial_profiles(p.profile_read()[0], cfg) if samples else None
    out = {"preset": preset, "steps": steps, "stats_from": stats_from, "every": every, "samples": samples,
           "storage": storage, "wall": cfg["wall"], "fluid_nodes": nf,
           "params": {k: cfg[k] for k in ("nx", "ny", "nz", "radius", "tau", "accel_z", "u_tau", "period",
                                          "force_off_step", "n_modes")},
           "amplitudes": np.asarray(amps).tolist(), "wall_time_s": round(time.perf_counter() - t0, 1)}
    if dominant:
        series = torch.stack(dominant).cpu().numpy()[:, 0]  # first pipe
        out["modes"] = {
            "every": modes_every, "from": modes_from, "r0": r0, "ntheta": ntheta, "mmax": mmax,
            "series": series.tolist(),
            "mean_spectrum": (spec_sum[0] / len(dominant)).cpu().numpy().tolist()}
    if dominant and series.min() >= 1:  # 0: a ring without fluctuations
        u_conv = float(np.interp(r0, prof["r"], prof["mean"])) if prof is not None else float("nan")
        out["modes"].update({
            "occupation": np.bincount(series, minlength=mmax + 1)[1:].tolist(),
            "transition_matrix": H.transition_matrix(series, mmax).tolist(),
            "ck": [{"order": d, "eigenvalues": lam.tolist(), "markov_prediction": pred.tolist()}
                   for d, lam, pred in H.ck_test(series, mmax)],
            "self_correlation_mean": H.self_correlation(series, mmax, min(200, len(series) // 4))[1].tolist(),
            "streamwise_lengths": {str(k): v for k, v in
                                   H.streamwise_lengths(series, mmax, modes_every, u_conv).items()},
        })
    if prof is not None:
        ut = cfg["u_tau"]
        prof = {k: np.asarray(v).tolist() for k, v in prof.items()}
        prof["y_plus"] = ((cfg["radius"] - np.asarray(prof["r"])) * ut / nu).tolist()
        prof["U_plus"] = (np.asarray(prof["mean"]) / ut).tolist()
        prof["rms_plus"] = (np.asarray(prof["rms"]) / ut).tolist()
        out["profiles"] = prof
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--preset", default="paper")
    ap.add_argument("--steps", type=int, required=True)
    ap.add_argument("--stats-from", type=int, default=None, help="first step of the statistics (default steps/2)")
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--progress", type=int, default=10000)
    ap.add_argument("--storage", type=int, default=0)
    ap.add_argument("--wall", type=int, default=None)
    ap.add_argument("--modes-every", type=int, default=0, help="dominant azimuthal mode every this many steps")
    ap.add_argument("--modes-from", type=int, default=None, help="first step of the mode series (default: stats)")
    ap.add_argument("--r0-frac", type=float, default=0.78)
    ap.add_argument("--ntheta", type=int, default=1024)
    ap.add_argument("--mmax", type=int, default=10)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    stats_from = a.stats_from if a.stats_from is not None else a.steps // 2
    res = run(a.preset, a.steps, stats_from, a.every, a.progress, a.storage, a.wall,
              log=lambda s: print(s, flush=True), modes_every=a.modes_every,
              modes_from=a.modes_from if a.modes_from is not None else stats_from, r0_frac=a.r0_frac,
              ntheta=a.ntheta, mmax=a.mmax)
    text = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    else:
        print(text, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
