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
    for f in ("lbm_device.h", "lbm_step.h", "lbm_kernels.hip"):
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


def _counter_kib(folder, kernel_prefix, counter):
    """Mean per-dispatch value (KiB) of one counter over the dispatches of
    the kernels whose name starts with kernel_prefix, from a rocprofv3
    --pmc CSV folder (``<folder>/*counter_collection.csv``)."""
    import csv
    import glob
    vals = []
    for path in glob.glob(os.path.join(folder, "*counter_collection.csv")):
        for row in csv.DictReader(open(path)):
            if row["Counter_Name"] == counter and row["Kernel_Name"].startswith(kernel_prefix):
                vals.append(float(row["Counter_Value"]))
    if not vals:
        raise ValueError(f"{folder}: no {counter} for {kernel_prefix}")
    return sum(vals) / len(vals), len(vals)


def record_traffic(folder, workload, storage):
    """HBM bytes per step-kernel launch from four rocprofv3 --pmc runs under
    folder (fetch<S>/ and write<S>/: ``bench.py --profile-steps 10 --storage
    S``; copyf/ and copyw/: ``bench.py --copy-calibration 2048``), each
    counter scaled by what it reads for the plain 2 GiB copy; written into
    profiles/step_kernel_hbm_traffic.json under the current kernel source
    hash.  Host only."""
    import lbm_inputs as LI
    from paper_2405_12082_amd import _lib
    copy_bytes = 2048 * (1 << 20)
    cf, _ = _counter_kib(os.path.join(folder, "copyf"), "__amd_rocclr_copyBuffer", "FETCH_SIZE")
    cw, _ = _counter_kib(os.path.join(folder, "copyw"), "__amd_rocclr_copyBuffer", "WRITE_SIZE")
    fetch_scale, write_scale = copy_bytes / (cf * 1024), copy_bytes / (cw * 1024)
    f, nd = _counter_kib(os.path.join(folder, f"fetch{storage}"), "void lbm::k_step<", "FETCH_SIZE")
    w, _ = _counter_kib(os.path.join(folder, f"write{storage}"), "void lbm::k_step<", "WRITE_SIZE")
    cfg = LI.preset(workload)
    cfg["storage"] = storage
    lay = _lib.describe(_lib.make_config(**cfg))
    alg = float(lay.n_fluid_nodes) * 27 * (2 if storage == 1 else 8 if storage == 2 else 4)
    read, written = f * 1024 * fetch_scale, w * 1024 * write_scale
    path = os.path.join(ROOT, "profiles", "step_kernel_hbm_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        rec = {}
    rec[f"{workload}:{storage}"] = {
        "algorithmic_read": alg, "algorithmic_write": alg, "bytes_per_launch": int(round(read + written)),
        "dispatches": nd, "fetch_scale": fetch_scale, "read_bytes": int(round(read)), "source_hash": kernel_source_hash(),
        "write_bytes": int(round(written)), "write_scale": write_scale}
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
    return rec[f"{workload}:{storage}"]


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
    """Step rate of a preset in a storage form, buffer pattern and wall (the
    fp16 leg: the turbulent pipe in FP16 storage, 108 B per update)."""
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
    (the interpolation of Eqs. (fbc1)/(fbc2)) and its k_theta = 2 trigger,
    and the same in FP16 storage (the form of the long runs); plus the cost
    of one coherent-structure sample (Section II.C: u_z on r = 0.78 R at
    every plane, transform of the azimuthal correlation, dominant mode)."""
    import torch
    import lbm_inputs as LI
    import paper_2405_12082_amd as P
    r = leg_fp16(steps, storage=0, pattern=0, wall=1, preset="paper")
    r["workload"] = "paper pipe 300x300x600 R=149.5, interpolated wall"
    torch.cuda.empty_cache()
    r["fp16"] = leg_fp16(steps, storage=1, pattern=0, wall=1, preset="paper")
    torch.cuda.empty_cache()
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
    wall units, at a few radii; in FP32 and again in FP16 storage, compared
    statistically (the two trajectories part after some hundred steps, so
    only the statistics can agree: differences as the precision study states
    them, over the bins with at least 1% of the mean bin count)."""
    import numpy as np
    from paper_2405_12082_amd import run
    out = {"steps": steps, "stats_window": [stats_from, steps]}
    profs = {}
    for name, storage in (("fp32", 0), ("fp16", 1)):
        res = run.run("turbulent", steps, stats_from, every=100, progress=steps, log=lambda s: None, storage=storage)
        p = res["profiles"]
        profs[name] = p
        yp = np.asarray(p["y_plus"])
        pick = [int(np.argmin(np.abs(yp - y))) for y in (5.0, 15.0, 30.0, 60.0, 120.0)] + [0]
        nf = res["fluid_nodes"]
        out[name] = {"samples": res["samples"], "wall_time_s": res["wall_time_s"],
                     "mlups_whole_run": round(nf * steps / res["wall_time_s"] / 1e6, 1),
                     "profiles_at": {k: [round(float(np.asarray(p[k])[i]), 4) for i in pick]
                                     for k in ("y_plus", "U_plus", "rms_plus", "skewness", "flatness")}}
    a, b = profs["fp32"], profs["fp16"]
    cnt = np.asarray(a["count"])
    sel = cnt >= 0.01 * cnt[cnt > 0].mean()
    diff = lambda k: np.abs(np.asarray(b[k]) - np.asarray(a[k]))[sel]
    out["fp16_vs_fp32"] = {
        "mean_profile": float(diff("mean").max() / np.abs(np.asarray(a["mean"])[sel]).max()),
        "rms_profile": float(diff("rms").max() / np.abs(np.asarray(a["rms"])[sel]).max()),
        "skewness_profile_abs": float(diff("skewness").max()),
        "flatness_profile_abs": float(diff("flatness").max()),
        "bins": int(sel.sum())}
    # the first entries stay where they were for readers of earlier lines
    out.update({k: out["fp32"][k] for k in ("samples", "wall_time_s", "mlups_whole_run", "profiles_at")})
    return out


def _timed_steps(stream, fn, steps):
    """ms per step of fn(steps) between HIP events on ``stream``."""
    a, b = _events(stream)
    a.record(stream)
    fn(steps)
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / steps


def leg_batched(steps=5000, graph_k=50, persistent_steps=1000):
    """64 independent pipes 64x64x256 (R = 30) with their own seeded forcing,
    5000 steps: one context, autotuned buffer pattern, launch geometry, step
    order and launch form (graph replay of ordinary launches, or of one
    persistent launch); against the same pipes run one after another as
    single-pipe contexts, each in its own autotuned pattern and launch
    geometry as graph replays (so the ratio isolates the batching).  The
    persistent forms are also timed on their own (over 1000 steps)."""
    import torch
    import lbm_inputs as LI
    import paper_2405_12082_amd as P
    from paper_2405_12082_amd import autotune
    cfg = LI.preset("batched")
    amps = LI.preset_amplitudes(cfg)
    B = cfg["batch"]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        tune = autotune.choose_pattern(cfg, amps, steps=10, stream=stream, persistent=True)
        p = P.Pipe(dict(cfg, pattern=tune["pattern"]), amps, stream=stream)
        p.set_launch(**tune["best"])
        run = p.step_graph if tune["mode"] == "graph" else p.step_persistent_graph
        run(2 * graph_k, graph_k)  # capture + warm
        ms_batched = _timed_steps(stream, lambda n: run(n, graph_k), steps)
        nf = p.n_fluid
        ok = bool((p.diagnostics()[:, 4] == 0).all())
        del p
        torch.cuda.empty_cache()
        # the persistent forms in the persistent tuner's pattern and geometry
        pt = tune["persistent"]
        q = P.Pipe(dict(cfg, pattern=pt["pattern"]), amps, stream=stream)
        q.set_launch(**pt["best"])
        q.step_persistent(2)
        ms_persistent = _timed_steps(stream, q.step_persistent, persistent_steps)
        q.step_persistent_graph(2 * graph_k, graph_k)
        ms_pgraph = _timed_steps(stream, lambda n: q.step_persistent_graph(n, graph_k), persistent_steps)
        del q
        torch.cuda.empty_cache()
        # sequential single pipes, each tuned and run as graph replays
        c1 = dict(cfg, batch=1)
        t1 = autotune.choose_pattern(c1, amps[:1], steps=10, stream=stream)
        singles = [P.Pipe(dict(c1, pattern=t1["pattern"]), amps[i:i + 1], stream=stream) for i in range(B)]
        for q in singles:
            q.set_launch(**t1["best"])
            q.step_graph(2 * graph_k, graph_k)

        def seq(n):
            for q in singles:
                q.step_graph(n, graph_k)
        ms_seq = _timed_steps(stream, seq, steps)
        del singles
        torch.cuda.empty_cache()
    agg = lambda ms: round(B * nf / (ms * 1e-3) / 1e6, 1)
    return {"value": agg(ms_batched), "unit": "MLUPS (aggregate)", "steps": steps,
            "ms_per_step": round(ms_batched, 4), "pipes": B, "fluid_nodes_per_pipe": nf,
            "launch": tune["best"], "launch_form": tune["mode"], "pattern": ["two buffers", "AA"][tune["pattern"]],
            "autotune_ms_by_pattern": {["two buffers", "AA"][q]: round(v, 4) for q, v in tune["by_pattern"].items()},
            "autotune_ms_by_form": {k: round(v, 4) for k, v in tune["by_mode"].items()},
            "graph_steps": graph_k, "autotune_cached": tune["cached"],
            "sequential_single_pipes": {"value": agg(ms_seq), "ms_per_step": round(ms_seq, 4),
                                        "pattern": ["two buffers", "AA"][t1["pattern"]], "launch": t1["best"],
                                        "form": "graph replay, autotuned per pipe", "steps": steps},
            "speedup_vs_sequential": round(ms_seq / ms_batched, 3),
            "persistent_launch": {"value": agg(ms_persistent), "ms_per_step": round(ms_persistent, 4),
                                  "pattern": ["two buffers", "AA"][pt["pattern"]], "launch": pt["best"],
                                  "steps": persistent_steps},
            "persistent_launch_graph": {"value": agg(ms_pgraph), "ms_per_step": round(ms_pgraph, 4),
                                        "steps_per_launch": graph_k, "steps": persistent_steps},
            "state_finite": ok}


def elementwise_add_rate(gib=4, reps=20):
    """Read + write GB/s of torch.add(a, 1, out=b) over two FP32 tensors of
    `gib` GiB each: the rate a plain streaming kernel reaches on this part
    (one read and one write stream, no reuse)."""
    import torch
    n = gib << 28
    a = torch.ones(n, device="cuda")
    b = torch.empty(n, device="cuda")
    torch.add(a, 1.0, out=b)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.add(a, 1.0, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * 4 * n / (ms * 1e-3) / 1e9


def leg_adjoint(fd_frac=1e-2):
    """Adjoint workload: 96x96x384 pipe (R = 45), 2000 steps, checkpoints
    every 100; gradient of the streamwise energy over steps 1501..2000 with
    respect to the 12 trigger amplitudes (gradient_cost_ratio: the whole
    gradient, forward with checkpoints and energy sampling plus the reverse
    sweep, over one plain forward; recorded_forward: the FP32-state gradient
    with the moments of every forward state kept in device memory instead
    of checkpoints, no recompute), by the FP32 forward with the
    adjoint state stored in FP32 (the bench's path) and in FP64, FP64
    vector-Jacobian arithmetic in both, the recompute keeping the moments
    (rho - 1, j) of each forward state.  Cost ratio = (recompute + adjoint
    sweep) / plain forward over the same steps.  Accuracy: relative L2
    distance to central differences (step 1% of the largest amplitude) of
    the FP64-storage forward."""
    import numpy as np
    import torch
    import lbm_inputs as LI
    import paper_2405_12082_amd as P
    from paper_2405_12082_amd.adjoint import EnergyAdjoint
    cfg = LI.preset("adjoint")
    amps = LI.preset_amplitudes(cfg)
    N = cfg["obs_end"] - 1
    b, e, C = cfg["obs_begin"], cfg["obs_end"], cfg["checkpoint_every"]
    stream = torch.cuda.Stream()
    out = {"steps": N, "checkpoint_every": C, "gradient_accumulation": "fp64"}
    with torch.cuda.stream(stream):
        p = P.Pipe(cfg, amps, stream=stream)
        p.step(2)
        ms_fwd = _timed_steps(stream, p.step, N) * N
        nf = p.n_fluid
        del p
        grads = {}
        for prec in ("fp64", "fp32"):
            run = EnergyAdjoint(cfg, b, e, checkpoint_every=C, stream=stream, precision=prec)
            run.gradient(amps)  # warm (allocations, first launches)
            J, g = run.gradient(amps)
            t = dict(run.timing)
            grads[prec] = g[0]
            out[f"adjoint_state_{prec}"] = {"backward_ms": round(t["backward_ms"], 2),
                                            "forward_with_checkpoints_ms": round(t["forward_ms"], 2),
                                            "cost_ratio": round(t["backward_ms"] / ms_fwd, 3),
                                            "gradient_cost_ratio": round((t["forward_ms"] + t["backward_ms"]) / ms_fwd, 3),
                                            "J": float(J[0])}
            del run
            torch.cuda.empty_cache()
        # the same gradient with the moments of every forward state kept in
        # device memory (no recompute): the whole gradient's cost
        run = EnergyAdjoint(cfg, b, e, stream=stream, precision="fp32", recompute=False)
        run.gradient(amps)
        J, g = run.gradient(amps)
        t = dict(run.timing)
        out["recorded_forward"] = {"backward_ms": round(t["backward_ms"], 2),
                                   "forward_with_records_ms": round(t["forward_ms"], 2),
                                   "cost_ratio": round(t["backward_ms"] / ms_fwd, 3),
                                   "gradient_cost_ratio": round((t["forward_ms"] + t["backward_ms"]) / ms_fwd, 3),
                                   "record_bytes": int(run.all_records.numel()),
                                   "equals_checkpoint_and_recompute": bool(np.array_equal(g[0], grads["fp32"]))}
        del run
        torch.cuda.empty_cache()
        ref = EnergyAdjoint(dict(cfg, storage=2), b, e, checkpoint_every=C, stream=stream, precision="fp64")
        eps = fd_frac * np.abs(amps).max()
        fd = np.zeros_like(grads["fp32"])
        for q in range(fd.size):
            ap, am = amps.copy(), amps.copy()
            ap[0, q] += eps
            am[0, q] -= eps
            fd[q] = (ref.objective(ap)[0] - ref.objective(am)[0]) / (2 * eps)
        del ref
        torch.cuda.empty_cache()
    for prec, g in grads.items():
        out[f"adjoint_state_{prec}"]["rel_err_vs_central_differences"] = float(np.linalg.norm(g - fd) /
                                                                               np.linalg.norm(fd))
    out.update({"forward_plain_ms": round(ms_fwd, 2), "fluid_nodes": nf, "adjoint_state": "fp32",
                "adjoint_arithmetic": "fp64", "recompute_records": "moments (rho - 1, j)",
                "adjoint_fwd_cost_ratio": out["adjoint_state_fp32"]["cost_ratio"],
                "grad_norm": float(np.linalg.norm(grads["fp32"])),
                "central_differences": {"forward": "fp64 storage", "step": f"{fd_frac:g} * max|amps|"}})
    return out


def leg_variants(steps=300):
    """Comparison schemes (the BGK operator of Eq. (srt) and the second-order
    equilibrium of the LBM-O(2) scheme, Section III) against the paper's
    scheme: step rate on the turbulent pipe (FP32, 216 B per update for
    every kind), and the A/B accuracy on a decaying shear wave u_x = 1e-4
    sin(2 pi z / 64) at tau = 0.8 (FP64 storage): the fitted viscosity's
    relative error, and its shift under a background velocity U_z = 0.1
    (Galilean invariance: about -3 U^2 with the second-order equilibrium)."""
    import numpy as np
    import torch
    import lbm_inputs as LI
    import paper_2405_12082_amd as P
    names = {(0, 0): "mrt_o6 (paper)", (0, 1): "mrt_o2", (1, 0): "bgk_o6", (1, 1): "bgk_o2"}
    out = {}
    for (coll, eq), name in names.items():
        r = leg_fp16(steps, storage=0) if (coll, eq) == (0, 0) else _leg_kind(steps, coll, eq)
        N, tau, amp = 64, 0.8, 1e-4
        nu = (tau - 0.5) / 3.0
        kk = 2 * np.pi / N
        T = int(1.0 / (nu * kk * kk))
        z = np.arange(N)
        fits = {}
        for U0 in (0.0, 0.1):
            c = dict(nx=1, ny=1, nz=N, batch=1, radius=0.0, tau=tau, accel_z=0.0, storage=2, init=0,
                     collision=coll, equilibrium=eq)
            p = P.Pipe(c)
            g = _shear_wave_state(N, amp, U0, eq)
            p.set_populations(torch.from_numpy(g[None]).cuda(), 0)
            a = []
            for n in (T // 4, T):
                p.step(n)
                ux = p.moments()[1].cpu().numpy()[0, 0, :, 0, 0].astype(np.float64)
                a.append(abs(np.sum(ux * np.exp(-2j * np.pi * z / N))) * 2 / N)
            fits[U0] = float(np.log(a[0] / a[1]) / (kk * kk * T) / nu - 1.0)
            del p
        out[name] = {"mlups": r["value"], "ms_per_step": r["ms_per_step"], "frac": r["frac"],
                     "shear_wave_nu_rel_err": fits[0.0], "galilean_shift_U0.1": fits[0.1] - fits[0.0]}
    return out


def _leg_kind(steps, collision, equilibrium):
    import torch
    import lbm_inputs as LI
    import paper_2405_12082_amd as P
    cfg = dict(LI.preset("turbulent"), collision=collision, equilibrium=equilibrium)
    amps = LI.preset_amplitudes(cfg)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        p = P.Pipe(cfg, amps, stream=stream)
        p.step(20)
        ms = _timed_steps(stream, p.step, steps)
        nf, bpu = p.n_fluid, int(p.layout.bytes_per_update)
        del p
        torch.cuda.empty_cache()
    gbs = nf * bpu / (ms * 1e-3) / 1e9
    return {"value": round(nf / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def _shear_wave_state(N, amp, U0, equilibrium):
    """Deviations f^eq(1, (amp sin(2 pi z / N), 0, U0)) - w of a 1x1xN column
    (sixth- or second-order equilibrium, the same expansion as the kernels'
    initial states)."""
    import numpy as np
    c = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                  [1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0], [1, 0, 1], [-1, 0, 1], [1, 0, -1], [-1, 0, -1],
                  [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1], [1, 1, 1], [-1, 1, 1], [1, -1, 1], [-1, -1, 1],
                  [1, 1, -1], [-1, 1, -1], [1, -1, -1], [-1, -1, -1]], float)
    w = np.array([8 / 27 / 4 ** int(np.dot(ci, ci)) for ci in c])
    g = np.zeros((27, N, 1, 1))
    for k in range(N):
        u = np.array([amp * np.sin(2 * np.pi * k / N), 0.0, U0])
        if equilibrium:  # second order: w (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u)
            cu = c @ u
            feq = w * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u @ u)
        else:  # sixth order, product form: w prod_a (1 - 3/2 u_a^2 | 1 +- 3 u_a + 3 u_a^2)
            feq = w * np.prod(np.where(c == 0, 1 - 1.5 * u ** 2, 1 + 3 * c * u + 3 * u ** 2), axis=1)
        g[:, k, 0, 0] = feq - w
    return g.astype(np.float32)


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
    ap.add_argument("--legs", default="fp16,aa,bouzidi,two_step,paper,batched,adjoint,variants,precision,"
                                      "turbulent_stats",
                    help="extra measurements after the timed region (comma list, or 'none')")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run this many steps only (for profiler runs) and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="copy a buffer of this many MiB 10 times (plain copy kernel of known "
                         "size, to calibrate HBM byte counters) and exit")
    ap.add_argument("--record-traffic", default=None, metavar="DIR",
                    help="host only: write the HBM traffic record of --workload/--storage from the "
                         "rocprofv3 counter folders under DIR, and exit")
    args = ap.parse_args()
    if args.record_traffic:
        print(json.dumps(record_traffic(args.record_traffic, args.workload, args.storage)))
        return
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
            if args.steps < 100 or s % 10 == 5:  # bracket every step kernel of a short run, else every tenth
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
        # reference point: the same access pattern as a plain 27-stream copy
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
                     "copy_reference_gbs": round(alg_bytes / (copy_ms * 1e-3) / 1e9, 1),
                     "step_vs_copy_rate": round(kavg_ms and copy_ms / kavg_ms, 4)},
        "state_finite": finite,
        "mass": float(diag[0, 0]),
    }
    del pipe
    torch.cuda.empty_cache()
    # second reference point: the streaming rate of a plain elementwise kernel
    add_gbs = elementwise_add_rate()
    out["roofline"]["elementwise_add_gbs"] = round(add_gbs, 1)
    if traffic:
        out["roofline"]["traffic_gbs"] = round(traffic / (kavg_ms * 1e-3) / 1e9, 1)
        out["roofline"]["traffic_vs_add_rate"] = round(traffic / (kavg_ms * 1e-3) / 1e9 / add_gbs, 4)
    legs = [x for x in args.legs.split(",") if x and x != "none"]
    extra = {}
    for leg in legs:
        extra[leg] = {"fp16": leg_fp16, "aa": leg_aa, "bouzidi": leg_bouzidi, "paper": leg_paper,
                      "two_step": leg_two_step,
                      "batched": leg_batched, "turbulent_stats": leg_turbulent_stats,
                      "adjoint": leg_adjoint, "variants": leg_variants,
                      "precision": leg_precision}[leg]()
    if extra:
        out["extra"] = extra
    if not args.no_cpu_baseline:
        c1 = dict(cfg)
        out["cpu_baseline"] = cpu_baseline(c1, amps[0], args.cpu_seconds, single)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
