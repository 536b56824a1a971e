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

``--spinup-steps S --spinup-storage 1`` runs the first S steps in FP16
storage (half the bytes per step) and hands the state to the main storage
through the dense populations; ``--save PATH`` writes, at the end of the run,
the state, its step, the statistics gathered so far (the host copy of the
per-column power sums and their sample count) and the mode series to a
NumPy archive, and ``--resume PATH`` continues a run from one (same preset,
storage and sampling), so a long run can span several processes; the state
continues bitwise.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def _series(dominant) -> np.ndarray:
    """The first pipe's dominant modes: ints (resumed) and device tensors [batch]."""
    return np.array([d if isinstance(d, int) else int(d[0].item()) for d in dominant], dtype=np.int64)


def _write(path, result):
    """Write a result JSON atomically (a partial one stays readable if the run
    is stopped while writing the next)."""
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write(json.dumps(result))
    os.replace(tmp, path)


def _fingerprint(cfg, every, modes_every, r0_frac, ntheta, mmax) -> str:
    """What a resumed run must share with the archived one: the
    configuration and the sampling."""
    return json.dumps({"cfg": {k: cfg[k] for k in sorted(cfg)}, "every": every, "modes_every": modes_every,
                       "r0_frac": r0_frac, "ntheta": ntheta, "mmax": mmax}, sort_keys=True, default=str)


def _save(path, p, samples, profile, dominant, spec_sum, spec_n, fingerprint):
    """Archive of a run in progress (see the module notes)."""
    blob, step = p.save()
    np.savez(path, state=blob.cpu().numpy(), step=step, samples=samples, profile=profile,
             dominant=_series(dominant), spec_sum=np.zeros(0) if spec_sum is None else spec_sum.cpu().numpy(),
             spec_n=spec_n, fingerprint=np.array(fingerprint))


def run(preset: str, steps: int, stats_from: int, every: int = 100, progress: int = 10000,
        storage: int = 0, wall: int | None = None, log=print, modes_every: int = 0, modes_from: int = 0,
        r0_frac: float = 0.78, ntheta: int = 1024, mmax: int = 10, spinup_steps: int = 0,
        spinup_storage: int | None = None, save: str | None = None, resume: str | None = None,
        out_path: str | None = None, partial_every: int = 0) -> dict:
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
    t0 = time.perf_counter()
    p = Pipe(cfg, amps)
    nf = p.n_fluid
    nu = (cfg["tau"] - 0.5) / 3.0
    p.profile_reset()
    samples = 0
    r0 = r0_frac * cfg["radius"]
    ring = None
    dominant, spec_sum, spec_n = [], None, 0
    prof_host = None  # statistics of earlier processes (resume)
    n = 0
    fingerprint = _fingerprint(cfg, every, modes_every, r0_frac, ntheta, mmax)
    if resume:
        arc = np.load(resume)
        if str(arc["fingerprint"]) != fingerprint:
            raise ValueError(f"{resume}: archived with another configuration or sampling")
        blob = torch.from_numpy(arc["state"]).to(p.device)
        if blob.numel() != p.state_bytes:
            raise ValueError(f"{resume}: the state does not match this configuration")
        n = int(arc["step"])
        p.load(blob, n)
        samples = int(arc["samples"])
        prof_host = arc["profile"]
        dominant = [int(v) for v in arc["dominant"]]
        spec_n = int(arc["spec_n"])
        spec_sum = torch.from_numpy(arc["spec_sum"]).to(p.device) if spec_n else None
        del blob
        log(json.dumps({"resumed": resume, "step": n, "samples": samples, "modes": len(dominant)}))
    elif spinup_steps and spinup_storage is not None and spinup_storage != storage:
        # the first steps in another storage, then the state through the dense populations
        q = Pipe(dict(cfg, storage=spinup_storage), amps)
        while n < spinup_steps:
            k = min(chunk - n % chunk, spinup_steps - n)  # whole chunks from chunk multiples on
            q.step_graph(k, chunk) if k == chunk else q.step(k)
            n += k
            if n % progress == 0 or n == spinup_steps:
                d = q.diagnostics()[0]
                log(json.dumps({"spinup_step": n, "storage": spinup_storage,
                                "elapsed_s": round(time.perf_counter() - t0, 1), "mass": d[0] / nf,
                                "mean_uz": d[3] / d[0], "non_finite": int(d[4])}))
                if d[4] != 0:
                    raise FloatingPointError(f"non-finite populations at spin-up step {n}")
        g = q.populations()
        del q
        torch.cuda.empty_cache()
        p.set_populations(g, n)
        del g
        torch.cuda.empty_cache()

    def summary(n_done):
        """The result so far (also written every partial_every steps)."""
        acc = p.profile_read()
        if prof_host is not None:
            acc = acc + prof_host
        prof = radial_profiles(acc[0], cfg) if samples else None
        out = {"preset": preset, "steps": steps, "steps_done": n_done, "stats_from": stats_from, "every": every,
               "samples": samples, "storage": storage, "spinup_steps": spinup_steps, "spinup_storage": spinup_storage,
               "wall": cfg["wall"], "fluid_nodes": nf,
               "params": {k: cfg[k] for k in ("nx", "ny", "nz", "radius", "tau", "accel_z", "u_tau", "period",
                                              "force_off_step", "n_modes")},
               "amplitudes": np.asarray(amps).tolist(), "wall_time_s": round(time.perf_counter() - t0, 1)}
        series = _series(dominant) if dominant else None
        if dominant:
            out["modes"] = {
                "every": modes_every, "from": modes_from, "r0": r0, "ntheta": ntheta, "mmax": mmax,
                "series": series.tolist(), "mean_spectrum": (spec_sum.cpu().numpy() / spec_n).tolist()}
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

    last_t, last_n = time.perf_counter(), n
    while n < steps:
        # steps up to the next multiple of chunk (a spin-up or an archive may
        # end between two), so that every sampling step is reached
        k = min(chunk - n % chunk, steps - n)
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
            dominant.append(dom)  # device tensors until the end of the run
            spec_sum = mean[0] if spec_sum is None else spec_sum + mean[0]  # first pipe
            spec_n += 1
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
            if out_path and partial_every and n % partial_every == 0 and n < steps:
                _write(out_path, summary(n))
            last_t = time.perf_counter()
    if save:
        acc = p.profile_read()
        _save(save, p, samples, acc if prof_host is None else acc + prof_host, dominant, spec_sum, spec_n,
              fingerprint)
    return summary(n)


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
    ap.add_argument("--spinup-steps", type=int, default=0, help="first steps in --spinup-storage")
    ap.add_argument("--spinup-storage", type=int, default=None, help="storage of the spin-up (1: FP16)")
    ap.add_argument("--save", default=None, help="archive the run's state and statistics at its end (.npz)")
    ap.add_argument("--resume", default=None, help="continue from an archive written by --save")
    ap.add_argument("--out", default=None)
    ap.add_argument("--partial-every", type=int, default=0,
                    help="also write the result so far to --out every this many steps")
    a = ap.parse_args(argv)
    stats_from = a.stats_from if a.stats_from is not None else a.steps // 2
    res = run(a.preset, a.steps, stats_from, a.every, a.progress, a.storage, a.wall,
              log=lambda s: print(s, flush=True), modes_every=a.modes_every,
              modes_from=a.modes_from if a.modes_from is not None else stats_from, r0_frac=a.r0_frac,
              ntheta=a.ntheta, mmax=a.mmax, spinup_steps=a.spinup_steps, spinup_storage=a.spinup_storage,
              save=a.save, resume=a.resume, out_path=a.out, partial_every=a.partial_every)
    if a.out:
        _write(a.out, res)
    else:
        print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
