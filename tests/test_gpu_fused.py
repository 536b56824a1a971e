"""Two time steps per launch (temporal blocking, ``lbm_set_fused``) on the GPU
(needs an MI355X).

The two-step kernel runs step n on a tile and its halo ring from HBM, keeps
the post-collision values in LDS and runs step n+1 on the tile from them.
Each step is the same per-node arithmetic as the single-step kernel, so from
the same state its states equal single steps bitwise (FP32 and FP16, whose
intermediate state is rounded through the storage codec); two steps from a
random state are also checked against the FP64 oracle directly.  Covered:
ragged tiles and z-ranges, a periodic box smaller than one tile (the halo
wraps onto the tile itself), odd step counts, graphs with an odd number of
two-step launches (replays alternate between the buffers), several pipes
per launch in both step orders, persistent launches, save / load and the
adjoint's recompute after two-step launches.
"""
import sys

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


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cfg(**kw):
    cfg = dict(nx=21, ny=23, nz=13, batch=1, radius=9.6, tau=0.56, accel_z=3e-6, n_modes=6,
               kz=3.0, kappa=0.5, l0_frac=0.2, l_frac=0.4, period=40.0, force_off_step=1000,
               storage=0, wall=0, pattern=0, init=1, u_tau=0.01)
    cfg.update(kw)
    return cfg


def _box(**kw):
    """Periodic box without a wall (every column fluid), smaller than a tile."""
    return _cfg(nx=12, ny=10, nz=5, radius=0.0, n_modes=0, init=0, accel_z=2e-5, **kw)


def _amps(cfg, seed=5, boost=1.0):
    if cfg["n_modes"] == 0:
        return None
    return LI.batch_amplitudes(seed, cfg["batch"], cfg["n_modes"], cfg["u_tau"], cfg["period"]) * boost


def _pops(p):
    return p.populations().cpu().numpy()


def _pair(P, cfg, amps, fused=dict(steps_per_launch=2)):
    """A single-step pipe and a two-step pipe holding the same start."""
    one = P.Pipe(cfg, amps)
    two = P.Pipe(cfg, amps)
    two.set_fused(**fused)
    assert np.array_equal(_pops(one), _pops(two))
    return one, two


@pytest.mark.parametrize("shape,zchunk,s0", [("pipe", 32, 10), ("pipe", 3, 11), ("pipe", 1, 0),
                                             ("box", 2, 4), ("box", 64, 7)])
def test_two_steps_random_state_vs_oracle(P, oracle_mod, shape, zchunk, s0):
    """Two steps (one two-step launch) from seeded random deviations: every
    population of every fluid node matches two steps of the oracle, within
    128 * 2^-24 * (max|g_in| + max|g_out|)."""
    O = oracle_mod
    cfg = _cfg() if shape == "pipe" else _box()
    amps = _amps(cfg, boost=40.0)
    _log(f"two-step launch vs oracle: {shape} zchunk={zchunk} s0={s0}")
    mask = O.Pipe(O.make_config(**cfg)).fluid_mask()
    g0 = LI.random_deviations(321, (cfg["nz"], cfg["ny"], cfg["nx"]))
    g0[:, ~mask] = 0.0
    p = P.Pipe(cfg, amps)
    p.set_fused(2, zchunk)
    p.set_populations(torch.from_numpy(g0[None]).cuda(), step=s0)
    p.step(2)
    g2 = _pops(p)[0].astype(np.float64)
    o = O.Pipe(O.make_config(**cfg), None if amps is None else amps[0])
    _, w, _ = O.lattice()
    f0 = g0.astype(np.float64) + w[:, None, None, None]
    f0[:, ~mask] = 0.0
    o.set_f(f0, s0)
    o.step(2)
    go = o.get_f() - w[:, None, None, None]
    tol = 128 * 2.0 ** -24 * (np.abs(g0).max() + np.abs(go[:, mask]).max())
    err = np.abs(g2[:, mask] - go[:, mask]).max()
    _log(f"max abs error {err:.3e} (tolerance {tol:.3e})")
    assert err <= tol
    assert np.all(g2[:, ~mask] == 0)


@pytest.mark.parametrize("storage", [0, 1])
@pytest.mark.parametrize("zchunk", [32, 5])
def test_two_step_launches_equal_single_steps(P, storage, zchunk):
    """Log-law start, six trigger modes, a pipe whose cross-section takes
    3 x 3 tiles: populations, moments and FP64 diagnostics after 2, 3, 7,
    14 and 24 steps (odd counts end with a single step) equal the
    single-step run bitwise."""
    cfg = _cfg(nx=34, ny=36, nz=24, radius=16.3, storage=storage)
    amps = _amps(cfg, seed=9)
    one, two = _pair(P, cfg, amps, dict(steps_per_launch=2, zchunk=zchunk))
    for n in (2, 1, 4, 7, 10):
        one.step(n)
        two.step(n)
        assert two.step_index == one.step_index
        a, b = _pops(one), _pops(two)
        if not np.array_equal(a, b):
            d = np.abs(a.astype(np.float64) - b)
            _log(f"step {one.step_index}: {np.count_nonzero(d)} values differ, max {d.max():.3e}")
        assert np.array_equal(a, b), f"step {one.step_index}"
        ra, ua = one.moments()
        rb, ub = two.moments()
        assert torch.equal(ra, rb) and torch.equal(ua, ub)
        assert np.array_equal(one.diagnostics(raise_on_nan=True), two.diagnostics(raise_on_nan=True))
    _log(f"storage {storage} zchunk {zchunk}: two-step launches == single steps over {one.step_index} steps")


@pytest.mark.parametrize("nz,zchunk", [(1, 1), (1, 32), (2, 1), (2, 32), (3, 2)])
def test_short_pipes(P, nz, zchunk):
    """Pipes of 1, 2 and 3 planes (the periodic z neighbours of a plane
    coincide or wrap within one z-range): 6 steps equal single steps
    bitwise."""
    cfg = _cfg(nz=nz)
    one, two = _pair(P, cfg, _amps(cfg), dict(steps_per_launch=2, zchunk=zchunk))
    one.step(6)
    two.step(6)
    assert np.array_equal(_pops(one), _pops(two))


def test_periodic_box_smaller_than_a_tile(P):
    """12 x 10 periodic box (no wall): the 16 x 16 box of the only tile wraps
    onto its own columns; 9 steps equal single steps bitwise."""
    cfg = _box()
    one, two = _pair(P, cfg, None)
    one.step(9)
    two.step(9)
    assert np.array_equal(_pops(one), _pops(two))


@pytest.mark.parametrize("launch", [
    dict(pipes_per_launch=2, pipe_major=0),
    dict(pipes_per_launch=1, pipe_major=1),
])
def test_batched_graph_persistent_save_load(P, launch):
    """Three pipes: two-step launches per pipe group in both step orders,
    graphs of 6 steps (three two-step launches: consecutive replays start
    from alternating buffers) and of 4, persistent launches in between,
    save / load: the single-step states throughout."""
    cfg = _cfg(batch=3)
    amps = _amps(cfg, seed=21)
    one, two = _pair(P, cfg, amps, dict(steps_per_launch=2, zchunk=4, xcd_remap=0))
    two.set_launch(**launch)
    one.step(3)
    two.step(3)
    for n, how in ((12, "graph6"), (7, "graph6"), (5, "persistent"), (16, "graph4"), (6, "persistent"),
                   (18, "graph6"), (2, "eager")):
        one.step(n)
        if how.startswith("graph"):
            two.step_graph(n, int(how[-1]))
        elif how == "persistent":
            two.step_persistent(n)
        else:
            two.step(n)
        assert two.step_index == one.step_index
        assert np.array_equal(_pops(one), _pops(two)), f"{how} to step {one.step_index}"
    blob, s = two.save()
    blob = blob.clone()
    two.step(6)
    a = _pops(two)
    two.load(blob, s)
    two.step(6)
    assert np.array_equal(a, _pops(two))
    one.step(6)
    assert np.array_equal(a, _pops(one))


def test_recompute_after_two_step_launches(P):
    """A checkpoint saved after two-step launches recomputes (single steps,
    every state kept) to the states the two-step run passes through."""
    cfg = _cfg()
    amps = _amps(cfg)
    p = P.Pipe(cfg, amps)
    p.set_fused(2)
    p.step(6)
    blob, s = p.save()
    blob = blob.clone()
    sb = p.state_bytes
    stride = (sb + 255) // 256 * 256
    ring = torch.empty((5, stride), dtype=torch.uint8, device="cuda")
    p.recompute(blob, s, ring)
    p.step(4)
    q = P.Pipe(cfg, amps)
    q.load(ring[4, :sb], s + 4)
    assert np.array_equal(_pops(p), _pops(q))


def test_unsupported_configurations_rejected(P):
    for kw in (dict(pattern=1), dict(wall=1), dict(storage=2)):
        cfg = _cfg(**kw)
        p = P.Pipe(cfg, _amps(cfg))
        with pytest.raises(P.LbmError):
            p.set_fused(2)
        p.set_fused(1)
    p = P.Pipe(_cfg(), _amps(_cfg()))
    for bad in (dict(steps_per_launch=3), dict(zchunk=1025), dict(xcd_remap=4097)):
        with pytest.raises(P.LbmError):
            p.set_fused(**bad)


def test_full_size_turbulent_pipe_in_the_bench_launch(P):
    """The turbulent pipe 192 x 192 x 1152 (R = 90, log-law start, trigger
    force) in the launch the bench times (two steps per launch, 32 planes per
    workgroup, XCD eighths): after 2, 4 and 5 steps the state equals single
    steps bitwise (compared on the device)."""
    cfg = LI.preset("turbulent")
    amps = LI.preset_amplitudes(cfg)
    one = P.Pipe(cfg, amps)
    two = P.Pipe(cfg, amps)
    two.set_fused(2, 32, 1)
    for n in (2, 2, 1):
        one.step(n)
        two.step(n)
        a, _ = one.save()
        b, _ = two.save()
        assert torch.equal(a, b), f"step {one.step_index}"
        del a, b
    _log(f"full-size turbulent pipe: two-step launches == single steps over {one.step_index} steps")
