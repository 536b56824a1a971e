"""Launch-geometry autotuner for the fused step.

Exhaustive search over (threads per block, z planes per thread, tile order,
pipes per launch, step order) on a live context: each candidate is set with
``lbm_set_launch`` and timed over a replay of a graph of a few steps with HIP
events on the pipe's stream.  The state is saved before and restored after the search, so tuning
does not advance the simulation.  Results are cached in a JSON file keyed by
the pipe shape, batch, storage, buffer pattern and GPU architecture.
:func:`choose_pattern` tunes the two-buffer and the AA pattern of a
configuration and returns the faster (the pattern is fixed when a context is
created, so it creates one context per pattern); with ``persistent=True`` it
also times replays of a graph holding one persistent launch of the same
steps (``lbm_step_persistent_graph``) at each block size and z-chunk, and
picks the faster launch form.
"""
from __future__ import annotations

import itertools
import json
import os

import torch

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "lbm_mi355x", "autotune.json")


def _key(pipe) -> str:
    c = pipe.cfg
    arch = torch.cuda.get_device_properties(pipe.device).gcnArchName.split(":")[0]
    return f"{arch}|{c.nx}x{c.ny}x{c.nz}|R{c.radius:g}|B{c.batch}|s{c.storage}|p{c.pattern}"


def candidates(batch: int):
    # pipes per launch: fractions of the batch, and a few small groups whose
    # working set can stay in the 256 MB last-level cache across the steps of
    # a pipe-major replay
    small = {p for p in (1, 2, 3, 4, 6) if p <= batch}
    ppl = sorted({batch, max(1, batch // 2), max(1, batch // 4), max(1, batch // 8)} | small, reverse=True)
    orders = (0, 1) if batch > 1 else (0,)
    for block, zchunk, xcd, p, pm in itertools.product((64, 128, 256, 512), (1, 2, 4, 8), (0, 1, 8), ppl, orders):
        if pm == 1 and p == batch:
            continue  # one group: both orders are the same launch sequence
        yield dict(block=block, zchunk=zchunk, xcd_remap=xcd, pipes_per_launch=p, pipe_major=pm)


def _time(pipe, steps: int) -> float:
    """ms per step of graph replays of ``steps`` steps (the way ensembles are
    run), after one replay that captures the graph."""
    steps += steps % 2
    stream = pipe.stream
    pipe.step_graph(steps, steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    pipe.step_graph(steps, steps)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps


def autotune(pipe, steps: int = 10, cache_path: str | None = DEFAULT_CACHE, force: bool = False,
             verbose: bool = False) -> dict:
    """Pick the fastest launch geometry for ``pipe`` and apply it.

    Returns {"best": {...}, "ms_per_step": t, "tried": n, "cached": bool}."""
    key = _key(pipe)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if not force and key in cache:
        best = cache[key]["best"]
        pipe.set_launch(**best)
        return dict(cache[key], cached=True)
    blob, step0 = pipe.save()
    blob = blob.clone()
    results = []
    for cand in candidates(pipe.cfg.batch):
        pipe.set_launch(**cand)
        ms = _time(pipe, steps)
        results.append((ms, cand))
        if verbose:
            print(f"autotune {cand} {ms:.4f} ms/step", flush=True)
    pipe.load(blob, step0)
    torch.cuda.synchronize()
    ms, best = min(results, key=lambda r: r[0])
    pipe.set_launch(**best)
    rec = {"best": best, "ms_per_step": ms, "tried": len(results)}
    if cache_path:
        cache[key] = rec
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return dict(rec, cached=False)


def _time_persistent(pipe, steps: int) -> float:
    """ms per step of replays of a graph holding one persistent launch of
    ``steps`` steps, after one replay that captures it."""
    steps += steps % 2
    stream = pipe.stream
    pipe.step_persistent_graph(steps, steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    pipe.step_persistent_graph(steps, steps)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps


def tune_persistent(pipe, steps: int = 10) -> dict:
    """Fastest (block, zchunk) of the persistent-launch graph form (the
    co-resident workgroups own whole pipes, so pipes per launch, step order
    and tile order do not apply); the state is restored afterwards."""
    blob, step0 = pipe.save()
    blob = blob.clone()
    res = []
    for block, zchunk in itertools.product((64, 128, 256, 512), (1, 2, 4)):
        pipe.set_launch(block=block, zchunk=zchunk)
        res.append((_time_persistent(pipe, steps), dict(block=block, zchunk=zchunk)))
    pipe.load(blob, step0)
    torch.cuda.synchronize()
    ms, best = min(res, key=lambda r: r[0])
    return {"best": best, "ms_per_step": ms, "tried": len(res)}


def choose_pattern(cfg: dict, amps, steps: int = 10, cache_path: str | None = DEFAULT_CACHE, force: bool = False,
                   device="cuda", stream=None, persistent: bool = False) -> dict:
    """Autotune the two-buffer (0) and the AA (1) pattern of ``cfg`` and
    return the faster: {"pattern", "best" (launch geometry), "ms_per_step",
    "by_pattern": {pattern: ms_per_step}, "mode" ("graph": replays of a graph
    of ordinary launches; "persistent_graph": replays of a graph holding one
    persistent launch), "by_mode", "cached"}.  Configurations with adjoint
    buffers allow only the two-buffer pattern; the persistent form is timed
    only when ``persistent`` is set (its result is not cached)."""
    from .pipe import Pipe
    patterns = (0,) if cfg.get("adjoint", 0) else (0, 1)
    res, pers = {}, {}
    for pat in patterns:
        p = Pipe(dict(cfg, pattern=pat), amps, device=device, stream=stream)
        res[pat] = autotune(p, steps, cache_path, force)
        if persistent:
            pers[pat] = tune_persistent(p, steps)
        del p
        torch.cuda.empty_cache()
    pat = min(res, key=lambda q: res[q]["ms_per_step"])
    out = {"pattern": pat, "best": res[pat]["best"], "ms_per_step": res[pat]["ms_per_step"],
           "by_pattern": {q: res[q]["ms_per_step"] for q in res}, "mode": "graph",
           "cached": all(r["cached"] for r in res.values())}
    if persistent:
        pp = min(pers, key=lambda q: pers[q]["ms_per_step"])
        out["by_mode"] = {"graph": res[pat]["ms_per_step"], "persistent_graph": pers[pp]["ms_per_step"]}
        out["persistent"] = {"pattern": pp, "best": pers[pp]["best"], "ms_per_step": pers[pp]["ms_per_step"],
                             "by_pattern": {q: pers[q]["ms_per_step"] for q in pers}}
        if pers[pp]["ms_per_step"] < out["ms_per_step"]:
            out.update(pattern=pp, best=pers[pp]["best"], ms_per_step=pers[pp]["ms_per_step"],
                       mode="persistent_graph")
    return out
