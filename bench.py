"""Benchmark of the fused D3Q27 MRT stream-collide step on one MI355X.

Workload (default): the turbulent pipe 192x192x1152, R = 90, Re_tau ~ 181
shape (u* = 0.00388), log-law start, trigger force with 12 seeded amplitudes
active for steps < 5000, FP32 deviation storage, halfway bounce-back.  One
"step" is one time step of the whole pipe: the fused stream-collide kernel,
plus the FP64 velocity-statistics sampling every 100 steps.

Prints one JSON line: MLUPS (fluid-node updates per second / 1e6), the HBM
roofline of the step kernel (216 algorithmic bytes per fluid-node update,
timed with HIP events on the library's stream), and the FP64 oracle timed on
the host cores over a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SAMPLE_EVERY = 100


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lbm_device.h", "lbm_kernels.hip"):
        h.update(open(os.path.join(ROOT, "paper_2405_12082_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload, storage):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "step_kernel_hbm_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = rec.get(f"{workload}:{storage}")
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def _oracle_rate(cfg, amps, nz, seconds):
    """MLUPS of the FP64 oracle on a z-slab of nz planes of the pipe."""
    from oracle import oracle as O
    c = dict(cfg)
    c["nz"] = nz
    p = O.Pipe(O.make_config(**c), amps)
    p.step(1)
    nf = p.n_fluid
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < seconds:
        p.step(2)
        steps += 2
    dt = time.perf_counter() - t0
    return nf * steps / dt / 1e6, steps, nf, dt, O.num_threads()


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_single_thread(cfg, amps, seconds=4.0):
    """The FP64 oracle on one thread: a child process with OMP_NUM_THREADS=1
    (the oracle's thread count is fixed when its library loads) on a 4-plane
    slab.  Called before this process touches the GPU."""
    import subprocess
    code = ("import json, sys; sys.path.insert(0, sys.argv[1]); import bench; "
            "r = bench._oracle_rate(json.loads(sys.argv[2]), json.loads(sys.argv[3]), 4, float(sys.argv[4])); "
            "print(json.dumps(r))")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        res = subprocess.run([sys.executable, "-c", code, ROOT, json.dumps(cfg),
                              json.dumps(None if amps is None else [float(a) for a in amps]), str(seconds)],
                             env=env, capture_output=True, text=True, timeout=120)
        r1 = json.loads(res.stdout.strip().splitlines()[-1])
        return {"value": r1[0], "threads": r1[4],
                "sample": f"{cfg['nx']}x{cfg['ny']}x4 slab, {r1[1]} steps, {r1[3]:.1f} s"}
    except (subprocess.SubprocessError, ValueError, IndexError) as e:
        return {"error": str(e)[:200]}


def cpu_baseline(cfg, amps, seconds=12.0, single=None):
    """The FP64 oracle (as it stands) on a z-slab of the same pipe: same
    cross-section, parameters and forcing, nz = 48, on all host threads;
    ``single``: the one-thread figure of cpu_single_thread."""
    rate, steps, nf, dt, threads = _oracle_rate(cfg, amps, 48, seconds)
    out = {"value": rate, "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"{cfg['nx']}x{cfg['ny']}x48 slab of the same pipe (R={cfg['radius']}), "
                     f"{steps} steps, {nf} fluid nodes, {dt:.1f} s",
           "cpu_model": _cpu_model()}
    if single is not None:
        out["single_thread"] = single
    return out


def _events(stream):
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    return a, b


def leg_fp16(steps=500, storage=1, pattern=0, wall=0, preset="turbulent", fused=None):
    """The turbulent pipe with FP16 scaled-deviation storage (108 B per update)."""
    import torch
    import lbm_inputs as LI
    import paper_2405_12082_amd as P
    cfg = LI.preset(preset)
    cfg["storage"] = storage
    cfg["pattern"] = pattern
    cfg["wall"] = wall
    amps = LI.preset_amplitudes(cfg)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        p = P.Pipe(cfg, amps, stream=stream)
        if fused:
            p.set_fused(*fused)
        p.step(20)
        a, b = _events(stream)
        a.record(stream)
        p.step(steps)
        b.record(stream)
        b.synchronize()
        ms = a.elapsed_time(b) / steps
        ok = bool(p.diagnostics()[0, 4] == 0)
    nf = p.n_fluid
    bpu = int(p.layout.bytes_per_update)
    del p
    torch.cuda.empty_cache()
    gbs = nf * bpu / (ms * 1e-3) / 1e9
    return {"value": round(nf / (ms * 1e-3) / 1e6, 1), "unit": "MLUPS", "ms_per_step": round(ms, 4),
            "bytes_per_update": bpu, "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "steps": steps, "state_finite": ok}


def leg_aa(steps=500):
    """The turbulent pipe in FP32 with the AA pattern: one buffer updated in
    place (half the state memory; same results as two buffers)."""
    r = leg_fp16(steps, storage=0, pattern=1)
    r["pattern"] = "AA (in place)"
    return r


def leg_two_step(steps=200, zchunk=32, xcd_remap=1):
    """The turbulent pipe in FP32 with two time steps per launch (temporal
    blocking: step n on a tile and its halo ring into LDS, step n+1 from
    there; the state crosses HBM once per two steps, 108 algorithmic bytes
    per update).  Same states as single steps, bitwise."""
    r = leg_fp16(steps, storage=0, fused=(2, zchunk, xcd_remap))
    r["bytes_per_update"] = 108
    gbs = r["value"] * 1e6 * 108 / 1e9
    r["achieved_gbs"] = round(gbs, 1)
    r["frac"] = round(gbs / HBM_PEAK_GBS, 4)
    r["launch"] = {"steps_per_launch": 2, "zchunk": zchunk, "xcd_remap": xcd_remap}
    return r


def leg_bouzidi(steps=500):
    """The turbulent pipe in FP32 with the interpolated wall of Eqs.
    (fbc1)/(fbc2) instead of the halfway bounce-back."""
    r = leg_fp16(steps, storage=0, pattern=0, wall=1)
    r["wall"] = "interpolated (Bouzidi)"
    return r


def leg_paper(steps=300, ntheta=1024, mmax=10, reps=50):
    """The paper's own pipe, 300x300x600 (R = 149.5), FP32, with its wall
    (the interpolation of Eqs. (fbc1)/(fbc2)) and its k_theta = 2 trigger;
    plus the cost of one coherent-structure sample (Section II.C: u_z on
    r = 0.78 R at every plane, transform of the azimuthal correlation,
    dominant mode)."""
    import torch
    import lbm_inputs as LI
    import paper_2405_12082_amd as P
    r = leg_fp16(steps, storage=0, pattern=0, wall=1, preset="paper")
    r["workload"] = "paper pipe 300x300x600 R=149.5, interpolated wall"
    cfg = LI.preset("paper")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        p = P.Pipe(cfg, LI.preset_amplitudes(cfg), stream=stream)
        p.step(200)
        ring = p.ring_sample(0.78 * cfg["radius"], ntheta)
        p.ring_spectrum(ring, mmax)
        a, b = _events(stream)
        a.record(stream)
        for _ in range(reps):
            p.ring_sample(0.78 * cfg["radius"], ntheta, out=ring)
            _, _, dom = p.ring_spectrum(ring, mmax)
        b.record(stream)
        b.synchronize()
        ms = a.elapsed_time(b) / reps
        del p
        torch.cuda.empty_cache()
    r["structure_sample"] = {"ms": round(ms, 4), "ntheta": ntheta, "planes": cfg["nz"], "mmax": mmax,
                             "per_step_equivalent": round(ms / r["ms_per_step"], 4)}
    return r


def leg_turbulent_stats(steps=20000, stats_from=10000):
    """The turbulent pipe's full run (20,000 steps, trigger force for the
    first 5,000) with the u_z statistics over the second half, sampled every
    100 steps: rms, skewness and flatness profiles (Eq. (urmsformula)), in
    wall units, at a few radii."""
    import numpy as np
    from paper_2405_12082_amd import run
    res = run.run("turbulent", steps, stats_from, every=100, progress=steps, log=lambda s: None)
    p = res["profiles"]
    yp = np.asarray(p["y_plus"])
    pick = [int(np.argmin(np.abs(yp - y))) for y in (5.0, 15.0, 30.0, 60.0, 120.0)] + [0]
    prof = {k: [round(float(np.asarray(p[k])[i]), 4) for i in pick]
            for k in ("y_plus", "U_plus", "rms_plus", "skewness", "flatness")}
    nf = res["fluid_nodes"]
    return {"steps": steps, "stats_window": [stats_from, steps], "samples": res["samples"],
            "wall_time_s": res["wall_time_s"], "mlups_whole_run": round(nf * steps / res["wall_time_s"] / 1e6, 1),
            "profiles_at": prof}


def leg_batched(steps=200, graph_k=50):
    """64 independent pipes 64x64x256 (R = 30) with their own seeded forcing:
    one context, autotuned launch geometry and step order, graph replay;
    against the same pipes run one after another as single-pipe contexts."""
    import torch
    import lbm_inputs as LI
    import paper_2405_12082_amd as P
    from paper_2405_12082_amd import autotune
    cfg = LI.preset("batched")
    amps = LI.preset_amplitudes(cfg)
    B = cfg["batch"]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        # launch geometry and buffer pattern (two buffers / AA in place)
        tune = autotune.choose_pattern(cfg, amps, steps=10, stream=stream)
        p = P.Pipe(dict(cfg, pattern=tune["pattern"]), amps, stream=stream)
        p.set_launch(**tune["best"])
        p.step_graph(2 * graph_k, graph_k)  # capture + warm
        a, b = _events(stream)
        a.record(stream)
        p.step_graph(steps, graph_k)
        b.record(stream)
        b.synchronize()
        ms_batched = a.elapsed_time(b) / steps
        # the same steps as one persistent cooperative launch (grid barrier per step)
        p.step_persistent(2)
        a, b = _events(stream)
        a.record(stream)
        p.step_persistent(steps)
        b.record(stream)
        b.synchronize()
        ms_persistent = a.elapsed_time(b) / steps
        # replays of a graph holding one persistent launch of graph_k steps
        p.step_persistent_graph(2 * graph_k, graph_k)  # capture + warm
        a, b = _events(stream)
        a.record(stream)
        p.step_persistent_graph(steps, graph_k)
        b.record(stream)
        b.synchronize()
        ms_pgraph = a.elapsed_time(b) / steps
        nf = p.n_fluid
        ok = bool((p.diagnostics()[:, 4] == 0).all())
        del p
        torch.cuda.empty_cache()
        # sequential single-pipe launches (eager, default geometry)
        c1 = dict(cfg, batch=1)
        singles = [P.Pipe(c1, amps[i:i + 1], stream=stream) for i in range(B)]
        for q in singles:
            q.step(2)
        a, b = _events(stream)
        a.record(stream)
        for q in singles:
            q.step(steps)
        b.record(stream)
        b.synchronize()
        ms_seq = a.elapsed_time(b) / steps
        del singles
        torch.cuda.empty_cache()
    return {"value": round(B * nf / (ms_batched * 1e-3) / 1e6, 1), "unit": "MLUPS (aggregate)",
            "ms_per_step": round(ms_batched, 4), "pipes": B, "fluid_nodes_per_pipe": nf,
            "launch": tune["best"], "pattern": ["two buffers", "AA"][tune["pattern"]],
            "autotune_ms_by_pattern": {["two buffers", "AA"][q]: round(v, 4) for q, v in tune["by_pattern"].items()},
            "graph_steps": graph_k, "autotune_cached": tune["cached"],
            "sequential_single_pipes": {"value": round(B * nf / (ms_seq * 1e-3) / 1e6, 1),
                                        "ms_per_step": round(ms_seq, 4)},
            "speedup_vs_sequential": round(ms_seq / ms_batched, 3),
            "persistent_launch": {"value": round(B * nf / (ms_persistent * 1e-3) / 1e6, 1),
                                  "ms_per_step": round(ms_persistent, 4)},
            "persistent_launch_graph": {"value": round(B * nf / (ms_pgraph * 1e-3) / 1e6, 1),
                                        "ms_per_step": round(ms_pgraph, 4), "steps_per_launch": graph_k},
            "state_finite": ok}


def leg_adjoint():
    """Adjoint workload: 96x96x384 pipe (R = 45), 2000 steps, checkpoints
    every 100; gradient of the streamwise energy over steps 1501..2000 with
    respect to the 12 trigger amplitudes.  Cost ratio = (recompute + adjoint
    sweep) / plain forward over the same steps."""
    import numpy as np
    import torch
    import lbm_inputs as LI
    import paper_2405_12082_amd as P
    from paper_2405_12082_amd.adjoint import EnergyAdjoint
    cfg = LI.preset("adjoint")
    amps = LI.preset_amplitudes(cfg)
    N = cfg["obs_end"] - 1
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        p = P.Pipe(cfg, amps, stream=stream)
        a, b = _events(stream)
        a.record(stream)
        p.step(N)
        b.record(stream)
        b.synchronize()
        ms_fwd = a.elapsed_time(b)
        nf = p.n_fluid
        del p
        run = EnergyAdjoint(cfg, cfg["obs_begin"], cfg["obs_end"], checkpoint_every=cfg["checkpoint_every"],
                            stream=stream, precision="fp32")
        J, g = run.gradient(amps)
        t = dict(run.timing)
        del run
        torch.cuda.empty_cache()
    return {"steps": N, "forward_plain_ms": round(ms_fwd, 2),
            "forward_with_checkpoints_ms": round(t["forward_ms"], 2), "backward_ms": round(t["backward_ms"], 2),
            "adjoint_fwd_cost_ratio": round(t["backward_ms"] / ms_fwd, 3),
            "J": float(J[0]), "grad_norm": float(np.linalg.norm(g[0])), "adjoint_state": "fp32",
            "gradient_accumulation": "fp64",
            "fluid_nodes": nf, "checkpoint_every": cfg["checkpoint_every"]}


def run_precision(steps=5000, sample_every=100, oracle_steps=100):
    """FP32 and FP16 storage against the FP64 reference on the 64x64x256
    precision pipe (R = 30, the turbulent workload's tau and u*): velocity
    error at steps 100 and 1000, and the radial profiles of mean, rms,
    skewness and flatness of u_z over the second half of the run (sampled
    every 100 steps).  The FP64 GPU run is tied to the FP64 oracle at step
    ``oracle_steps``."""
    import numpy as np
    import torch
    import lbm_inputs as LI
    import paper_2405_12082_amd as P
    from paper_2405_12082_amd.pipe import radial_profiles
    from oracle import oracle as O
    cfg = LI.preset("precision_ref")
    amps = LI.preset_amplitudes(cfg)
    first = cfg["force_off_step"]
    res = {}
    for storage in (2, 0, 1):
        c = dict(cfg, storage=storage)
        p = P.Pipe(c, amps)
        snaps = {}
        n = 0
        for target in (oracle_steps, 1000):
            p.step(target - n)
            n = target
            snaps[target] = p.moments()[1][0].cpu().numpy().astype(np.float64)
            if storage == 2 and target == oracle_steps:  # the FP64 channels at the oracle step
                fp64_sums = (p.diagnostics()[0].copy(), float(p.energy()[0]))
        p.profile_reset()
        while n < steps:
            k = min(sample_every - n % sample_every, steps - n)
            p.step(k)
            n += k
            if n >= first and n % sample_every == 0:
                p.profile_accumulate()
        prof = radial_profiles(p.profile_read()[0], c)
        ok = bool(p.diagnostics()[0, 4] == 0)
        res[storage] = (snaps, prof, ok)
        del p
        torch.cuda.empty_cache()
    o = O.Pipe(O.make_config(**cfg), amps[0])
    o.step(oracle_steps)
    uo = o.moments()[1]
    mask = o.fluid_mask()
    so, eo = o.sums(), o.energy()
    del o
    d64, e64 = fp64_sums
    ref_snaps, ref_prof, _ = res[2]

    def verr(u, ur):
        return float(np.abs(u - ur)[:, mask].max() / np.abs(ur[:, mask]).max())

    rmax = cfg["radius"] - 1.0
    sel = (ref_prof["count"] > 0) & (ref_prof["r"] < rmax)

    def perr(pa, key, relative=True):
        d = np.abs(pa[key][sel] - ref_prof[key][sel]).max()
        return float(d / np.abs(ref_prof[key][sel]).max()) if relative else float(d)

    out = {"pipe": "64x64x256 R=30", "steps": steps, "stats_window": [first, steps],
           "fp64_gpu_vs_oracle_velocity": {f"step_{oracle_steps}": verr(ref_snaps[oracle_steps], uo),
                                           "through": "the FP32 moments export"},
           "fp64_gpu_vs_oracle_sums": {"step": oracle_steps,
                                       "mass": float(abs(d64[0] - so[0]) / so[0]),
                                       "momentum": float(np.abs(d64[1:4] - so[1:4]).max() / np.abs(so[1:4]).max()),
                                       "energy": float(abs(e64 - eo) / eo)}}
    for storage, name in ((0, "fp32"), (1, "fp16")):
        snaps, prof, ok = res[storage]
        out[name] = {"velocity_step_100": verr(snaps[100], ref_snaps[100]),
                     "velocity_step_1000": verr(snaps[1000], ref_snaps[1000]),
                     "mean_profile": perr(prof, "mean"), "rms_profile": perr(prof, "rms"),
                     "skewness_profile_abs": perr(prof, "skewness", False),
                     "flatness_profile_abs": perr(prof, "flatness", False), "state_finite": ok}
    out["reference_profiles"] = {k: [round(float(v), 8) for v in ref_prof[k][sel]]
                                 for k in ("r", "mean", "rms", "skewness", "flatness")}
    return out


def leg_precision():
    return run_precision()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="turbulent")
    ap.add_argument("--storage", type=int, default=0, help="0: FP32, 1: FP16 deviations")
    ap.add_argument("--pattern", type=int, default=0, help="0: two buffers, 1: AA in place")
    ap.add_argument("--wall", type=int, default=None, help="0: halfway bounce-back, 1: interpolated (default: the workload's)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--xcd-remap", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="fp16,aa,bouzidi,two_step,paper,batched,adjoint,precision,turbulent_stats",
                    help="extra measurements after the timed region (comma list, or 'none')")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run this many steps only (for profiler runs) and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="copy a buffer of this many MiB 10 times (plain copy kernel of known "
                         "size, to calibrate HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the stepper runs one pipe per GPU); --gpus {args.gpus} "
              "is not supported", file=sys.stderr)
        sys.exit(2)

    import lbm_inputs as LI

    # the oracle's one-thread rate runs in a child process: started before
    # this process touches the GPU
    single = None
    if not args.no_cpu_baseline and not args.profile_steps and not args.copy_calibration:
        c0 = LI.preset(args.workload)
        if args.wall is not None:
            c0["wall"] = args.wall
        single = cpu_single_thread(c0, LI.preset_amplitudes(c0)[0])

    import numpy as np
    import torch

    import paper_2405_12082_amd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    P.lib()
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4,
                          "launches": 10}))
        return
    cfg = LI.preset(args.workload)
    cfg["storage"] = args.storage
    cfg["pattern"] = args.pattern
    if args.wall is not None:
        cfg["wall"] = args.wall
    cfg["block"] = args.block
    cfg["zchunk"] = args.zchunk
    cfg["xcd_remap"] = args.xcd_remap
    amps = LI.preset_amplitudes(cfg)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pipe = P.Pipe(cfg, amps, stream=stream)
        if args.profile_steps:
            pipe.step(args.profile_steps)
            pipe.stream_copy(args.profile_steps)
            torch.cuda.synchronize()
            print(json.dumps({"profile_steps": args.profile_steps, "workload": args.workload}))
            return
        nf = pipe.n_fluid
        pipe.step(args.warmup)
        torch.cuda.synchronize()

        # timed region: K steps, velocity statistics sampled every 100 steps
        ev_pairs = []
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        n_seg = 5 if args.steps >= 5 else 1  # five equal segments: median and spread
        seg_ev = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_start.record(stream)
        for s in range(args.steps):
            if s % (args.steps // n_seg) == 0 and len(seg_ev) < n_seg:
                e = torch.cuda.Event(enable_timing=True)
                e.record(stream)
                seg_ev.append((s, e))
            if s % 10 == 5:  # bracket every tenth step kernel with events
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                pipe.step(1)
                b.record(stream)
                ev_pairs.append((a, b))
            else:
                pipe.step(1)
            if (pipe.step_index % SAMPLE_EVERY) == 0:
                pipe.profile_accumulate()
        t_end.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms_total = t_start.elapsed_time(t_end)
        bounds = seg_ev + [(args.steps, t_end)]
        seg_mlups = [nf * cfg["batch"] * (s1 - s0) / (e0.elapsed_time(e1) * 1e-3) / 1e6
                     for (s0, e0), (s1, e1) in zip(bounds[:-1], bounds[1:])]
        kern_ms = [a.elapsed_time(b) for a, b in ev_pairs]
        diag = pipe.diagnostics()
        # practical ceiling: the same access pattern as a plain 27-stream copy
        pipe.stream_copy(5)
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        n_copy = max(20, min(200, args.steps // 10))
        c0.record(stream)
        pipe.stream_copy(n_copy)
        c1.record(stream)
        torch.cuda.synchronize()
        copy_ms = c0.elapsed_time(c1) / n_copy
    finite = bool(np.all(diag[:, 4] == 0) and np.all(np.isfinite(diag[:, :4])))
    ms_step = max(ms_total, wall * 1e3) / args.steps
    mlups = nf * cfg["batch"] / (ms_step * 1e-3) / 1e6
    lay = pipe.layout
    bpu = int(lay.bytes_per_update)
    kavg_ms = float(np.mean(kern_ms)) if kern_ms else float("nan")
    alg_bytes = nf * cfg["batch"] * bpu
    achieved = alg_bytes / (kavg_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, args.storage) if args.pattern == 0 and cfg["wall"] == 0 else None
    out = {
        "metric": "MLUPS + % HBM roofline (D3Q27 MRT fwd); adjoint/fwd cost ratio",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == 0 else "f32 compute, f16 storage",
        "data": "synthetic",
        "segments": {"mlups": [round(x, 1) for x in seg_mlups], "median_mlups": round(float(np.median(seg_mlups)), 1),
                     "all_node_mlups": round(mlups * cfg["nx"] * cfg["ny"] / (nf / cfg["nz"]), 1)},
        "config": {"workload": f"{args.workload} pipe {cfg['nx']}x{cfg['ny']}x{cfg['nz']} R={cfg['radius']}",
                   "fluid_nodes": nf, "batch": cfg["batch"], "storage": "fp32" if args.storage == 0 else "fp16",
                   "tau": round(cfg["tau"], 6), "n_modes": cfg["n_modes"], "force_off_step": cfg["force_off_step"],
                   "wall": ["halfway bounce-back", "interpolated (Bouzidi)"][cfg["wall"]],
                   "pattern": ["two buffers", "AA in place"][cfg["pattern"]],
                   "sample_every": SAMPLE_EVERY, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_step", "kernel_avg_ms": round(kavg_ms, 5),
                     "bytes_per_update": bpu, "kernel_samples": len(kern_ms),
                     "copy_ceiling_gbs": round(alg_bytes / (copy_ms * 1e-3) / 1e9, 1),
                     "frac_of_copy_ceiling": round(kavg_ms and copy_ms / kavg_ms, 4)},
        "state_finite": finite,
        "mass": float(diag[0, 0]),
    }
    del pipe
    torch.cuda.empty_cache()
    legs = [x for x in args.legs.split(",") if x and x != "none"]
    extra = {}
    for leg in legs:
        extra[leg] = {"fp16": leg_fp16, "aa": leg_aa, "bouzidi": leg_bouzidi, "paper": leg_paper,
                      "two_step": leg_two_step,
                      "batched": leg_batched, "turbulent_stats": leg_turbulent_stats,
                      "adjoint": leg_adjoint,
                      "precision": leg_precision}[leg]()
    if extra:
        out["extra"] = extra
    if not args.no_cpu_baseline:
        c1 = dict(cfg)
        out["cpu_baseline"] = cpu_baseline(c1, amps[0], args.cpu_seconds, single)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
