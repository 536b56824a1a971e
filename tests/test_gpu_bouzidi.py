"""The interpolated (Bouzidi) pipe wall of Eqs. (fbc1)/(fbc2) on the GPU
against the FP64 oracle (needs an MI355X).

Each cut link carries the exact fraction Delta at which it crosses r = R;
the pull combines the bounce-back value with the node's own outgoing value
(Delta >= 1/2) or with the value coming back from the next fluid node
(Delta < 1/2).  Tolerances as for the bounce-back wall: one step from a
random state within 64 * 2^-24 * (max|g_in| + max|g_out|) per population,
velocity of multi-step runs within 1e-5 of max|u|.  Writing a state
(set_populations) inverts the interpolation, so a round trip is exact only
up to a few roundings.
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
               storage=0, wall=1, pattern=0, init=1, u_tau=0.01)
    cfg.update(kw)
    return cfg


def _amps(cfg, seed=5, boost=1.0):
    return LI.batch_amplitudes(seed, cfg["batch"], cfg["n_modes"], cfg["u_tau"], cfg["period"]) * boost


def _pops(p):
    return p.populations().cpu().numpy()


def _vel_err(u_gpu, u_orc, mask):
    return np.abs(u_gpu - u_orc)[:, mask].max() / np.abs(u_orc[:, mask]).max()


@pytest.mark.parametrize("nx,ny,radius,zchunk,block,nz", [
    (21, 23, 9.6, 4, 256, 13), (21, 23, 9.3, 1, 64, 13), (21, 23, 8.45, 5, 128, 13),
    # thin pipes: links whose far node is solid (bounce-back fallback of
    # Eq. (fbc2)) and nodes with two cut links on one line (coupled inverse)
    (7, 7, 1.1, 4, 64, 13), (6, 7, 1.3, 2, 64, 13),
    # one and two planes: the far node x + c_i of a c_z link wraps onto the same or the other plane
    (21, 23, 9.6, 1, 256, 1), (21, 23, 8.45, 2, 128, 2)])
def test_bouzidi_single_step_random_state(P, oracle_mod, nx, ny, radius, zchunk, block, nz):
    """One step from seeded random deviations with the trigger force active:
    every population of every fluid node matches the oracle's collide +
    stream with the interpolated wall.  The radii give different cut-link
    fractions: both branches of the interpolation (around 60 links each on
    the 21x23 sections), and on the thin pipes the far-node fallback and the
    coupled inverse in set_populations."""
    O = oracle_mod
    cfg = _cfg(nx=nx, ny=ny, radius=radius, zchunk=zchunk, block=block, nz=nz)
    amps = _amps(cfg, boost=40.0)
    _log(f"Bouzidi single step R={radius} zchunk={zchunk} block={block} nz={nz}")
    mask = O.Pipe(O.make_config(**cfg)).fluid_mask()
    g0 = LI.random_deviations(77, (cfg["nz"], cfg["ny"], cfg["nx"]))
    g0[:, ~mask] = 0.0
    p = P.Pipe(cfg, amps)
    p.set_populations(torch.from_numpy(g0[None]).cuda(), step=10)
    back = _pops(p)[0]
    rt = np.abs(back - g0).max()
    _log(f"set/get round trip {rt:.3e}")
    assert rt <= 16 * 2.0 ** -24 * np.abs(g0).max()
    p.step(1)
    g1 = _pops(p)[0].astype(np.float64)
    o = O.Pipe(O.make_config(**cfg), amps[0])
    _, w, _ = O.lattice()
    f0 = g0.astype(np.float64) + w[:, None, None, None]
    f0[:, ~mask] = 0.0
    o.set_f(f0, 10)
    o.step(1)
    go = o.get_f() - w[:, None, None, None]
    tol = 64 * 2.0 ** -24 * (np.abs(g0).max() + np.abs(go[:, mask]).max())
    err = np.abs(g1[:, mask] - go[:, mask]).max()
    _log(f"max abs error {err:.3e} (tolerance {tol:.3e})")
    assert err <= tol
    assert np.all(g1[:, ~mask] == 0)


def test_bouzidi_laminar_pipe_100_steps(P, oracle_mod):
    """Laminar pipe 24x24x48, R = 10, tau = 0.8, a = 1e-6 from rest with the
    interpolated wall: velocity within 1e-5 of the oracle after 100 steps."""
    O = oracle_mod
    cfg = dict(LI.preset("laminar"), wall=1)
    p = P.Pipe(cfg)
    p.step(100)
    _, u_g = p.moments()
    o = O.Pipe(O.make_config(**cfg))
    o.step(100)
    _, u_o = o.moments()
    err = _vel_err(u_g.cpu().numpy()[0].astype(np.float64), u_o, o.fluid_mask())
    _log(f"Bouzidi laminar velocity error {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("storage,tol", [(0, 1e-5), (2, 1e-9), (1, 1e-3)])
def test_bouzidi_forced_loglaw_run(P, oracle_mod, storage, tol):
    """Log-law start (written through the inverse of the interpolation), six
    trigger modes, 80 steps with the force switched off at 60: velocity
    against the oracle, for FP32, FP64 and FP16 storage."""
    O = oracle_mod
    cfg = _cfg(nx=30, ny=28, nz=24, radius=13.4, force_off_step=60, storage=storage)
    amps = _amps(cfg, seed=9)
    p = P.Pipe(cfg, amps)
    o = O.Pipe(O.make_config(**cfg), amps[0])
    mask = o.fluid_mask()
    for n in (0, 30, 50):
        p.step(n)
        o.step(n)
        _, u_g = p.moments()
        _, u_o = o.moments()
        err = _vel_err(u_g.cpu().numpy()[0].astype(np.float64), u_o, mask)
        _log(f"storage {storage}, step {o.step_index}: velocity error {err:.3e}")
        assert err <= (tol if storage != 2 else 2e-7)  # FP32 export of the FP64 state
    d = p.diagnostics(raise_on_nan=True)[0]
    s = o.sums()
    assert abs(d[0] - s[0]) <= (1e-9 if storage != 1 else 1e-5) * s[0]
    if storage == 2:  # FP64 throughout: the FP64 sums at rounding level
        mom = np.abs(d[1:4] - s[1:4]).max() / np.abs(s[1:4]).max()
        e, eo = p.energy()[0], o.energy()
        _log(f"FP64 storage: mass {abs(d[0] - s[0]) / s[0]:.2e}, momentum {mom:.2e}, energy {abs(e - eo) / eo:.2e}")
        assert abs(d[0] - s[0]) < 1e-12 * s[0] and mom < 1e-11 and abs(e - eo) < 1e-11 * eo


def test_bouzidi_graph_persistent_and_batch(P):
    """Batch of three, graph replays and persistent launches give the eager
    states bitwise; each pipe of the batch equals a single-pipe run."""
    cfg = _cfg(batch=3)
    amps = _amps(cfg, seed=21)
    pe = P.Pipe(cfg, amps)
    pg = P.Pipe(cfg, amps)
    pg.set_launch(block=64, zchunk=3, pipes_per_launch=2, pipe_major=1)
    pe.step(3)
    pg.step(3)
    for n, how in ((10, "graph"), (7, "persistent"), (16, "graph")):
        pe.step(n)
        if how == "graph":
            pg.step_graph(n, 4)
        else:
            pg.step_persistent(n)
        assert np.array_equal(_pops(pe), _pops(pg)), f"{how} to step {pe.step_index}"
    gb = _pops(pe)
    for b in range(3):
        p1 = P.Pipe(dict(cfg, batch=1), amps[b:b + 1])
        p1.step(pe.step_index)
        assert np.array_equal(_pops(p1)[0], gb[b]), f"pipe {b}"
