"""GPU parity of the HIP stepper against the FP64 oracle (needs an MI355X).

Inputs are seeded and identical on both sides: the oracle receives
f = w + g with g the same FP32 deviations the GPU stores.  Tolerances:
 * velocity after the 100-step laminar run: max|u - u_oracle| / max|u_oracle|
   <= 1e-5 (the target tolerance on velocity);
 * one step from a random state: every population within
   64 * 2^-24 * (max|g_in| + max|g_out|), i.e. a few dozen FP32 roundings
   of the magnitudes the collision combines;
 * batching, graph replay and save/load: bitwise equality.
"""
import os
import sys

import numpy as np
import pytest

import lbm_inputs as LI

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_12082_amd as P
    P.lib()  # fails loudly when the library is not built
    return P


@pytest.fixture(scope="module")
def O(oracle_mod):
    return oracle_mod


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_pipe(O, cfg, amps=None):
    return O.Pipe(O.make_config(**cfg), None if amps is None else np.asarray(amps).reshape(-1))


def _fluid(O, cfg):
    return O.Pipe(O.make_config(**cfg)).fluid_mask()


def _gpu_u(pipe):
    rho, u = pipe.moments()
    torch.cuda.synchronize()
    return rho.cpu().numpy().astype(np.float64), u.cpu().numpy().astype(np.float64)


def _vel_err(u_gpu, u_orc, mask):
    d = np.abs(u_gpu - u_orc)[:, mask]
    return d.max() / np.abs(u_orc[:, mask]).max()


# ------------------------------------------------------------------ laminar
def test_laminar_velocity_parity_100_steps(gpu, O):
    """Laminar pipe 24x24x48, R = 10, tau = 0.8, a = 1e-6 from rest, halfway
    bounce-back: after 100 steps the FP32 kernel's velocity is within 1e-5
    (relative max norm) of the FP64 oracle."""
    cfg = LI.preset("laminar")
    _log(f"laminar parity: {cfg['nx']}x{cfg['ny']}x{cfg['nz']}")
    p = gpu.Pipe(cfg)
    p.step(100)
    rho_g, u_g = _gpu_u(p)
    o = _oracle_pipe(O, cfg)
    o.step(100)
    rho_o, u_o = o.moments()
    mask = o.fluid_mask()
    err = _vel_err(u_g[0], u_o, mask)
    _log(f"laminar velocity error {err:.3e}")
    assert err <= 1e-5
    assert np.abs(rho_g[0][mask] - rho_o[mask]).max() < 1e-6
    # solid nodes read as zero
    assert np.all(u_g[0][:, ~mask] == 0) and np.all(rho_g[0][~mask] == 0)


def test_laminar_populations_parity_500_steps(gpu, O):
    cfg = LI.preset("laminar")
    p = gpu.Pipe(cfg)
    p.step(500)
    g = p.populations().cpu().numpy()[0].astype(np.float64)
    o = _oracle_pipe(O, cfg)
    o.step(500)
    _, w, _ = O.lattice()
    go = o.get_f() - w[:, None, None, None]
    mask = o.fluid_mask()
    err = np.abs(g[:, mask] - go[:, mask]).max() / np.abs(go[:, mask]).max()
    _log(f"laminar 500-step population error {err:.3e}")
    assert err < 1e-4
    _, u_g = _gpu_u(p)
    _, u_o = o.moments()
    assert _vel_err(u_g[0], u_o, mask) < 2e-5


# ------------------------------------------------------------------ one step, random state
def _forced_cfg(**kw):
    cfg = dict(nx=21, ny=23, nz=13, batch=1, radius=9.6, tau=0.56, accel_z=3e-6, n_modes=6,
               kz=3.0, kappa=0.5, l0_frac=0.2, l_frac=0.4, period=40.0, force_off_step=1000,
               storage=0, wall=0, pattern=0, init=1, u_tau=0.01)
    cfg.update(kw)
    return cfg


def _amps(cfg, seed=5, boost=1.0):
    """Seeded amplitudes; ``boost`` scales them up for single-step checks of
    the forcing terms (the flow would not stay stable over many steps)."""
    return LI.batch_amplitudes(seed, cfg["batch"], cfg["n_modes"], cfg["u_tau"], cfg["period"]) * boost


@pytest.mark.parametrize("zchunk,block,nz", [(4, 256, 13), (1, 64, 13), (5, 128, 13), (1, 256, 1), (4, 512, 1),
                                             (2, 128, 2), (1, 64, 2)])
def test_single_step_random_state_all_populations(gpu, O, zchunk, block, nz):
    """One fused step from seeded random deviations with the trigger force
    active (step index 10, sin(2 pi 10/40) = 1): every population of every
    fluid node matches the oracle's collide + stream; also on pipes of one
    and two planes, where the periodic z neighbours of a plane coincide."""
    cfg = _forced_cfg(zchunk=zchunk, block=block, nz=nz)
    amps = _amps(cfg, boost=40.0)
    _log(f"single step parity zchunk={zchunk} block={block} nz={nz}")
    mask = _fluid(O, cfg)
    g0 = LI.random_deviations(123, (cfg["nz"], cfg["ny"], cfg["nx"]))
    g0[:, ~mask] = 0.0
    p = gpu.Pipe(cfg, amps)
    p.set_populations(torch.from_numpy(g0[None]).cuda(), step=10)
    back = p.populations().cpu().numpy()[0]
    assert np.array_equal(back, g0), "set/get populations must round-trip exactly"
    p.step(1)
    g1 = p.populations().cpu().numpy()[0].astype(np.float64)
    o = _oracle_pipe(O, cfg, amps[0])
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


def test_forced_loglaw_run_parity(gpu, O):
    """Log-law start, six trigger modes, 80 steps (force switched off at 60):
    velocity within 1e-5 of the oracle."""
    cfg = _forced_cfg(nx=30, ny=28, nz=24, radius=13.4, force_off_step=60)
    amps = _amps(cfg, seed=9)
    p = gpu.Pipe(cfg, amps)
    o = _oracle_pipe(O, cfg, amps[0])
    mask = o.fluid_mask()
    _, u_g = _gpu_u(p)
    _, u_o = o.moments()
    assert _vel_err(u_g[0], u_o, mask) < 1e-6, "initial log-law state"
    for n in (30, 50):
        p.step(n)
        o.step(n)
        _, u_g = _gpu_u(p)
        _, u_o = o.moments()
        err = _vel_err(u_g[0], u_o, mask)
        _log(f"forced run, step {o.step_index}: velocity error {err:.3e}")
        assert err <= 1e-5


def test_periodic_box_shear_wave(gpu, O):
    """No wall (radius <= 0): fully periodic 2x3x32 box with a shear wave."""
    cfg = dict(nx=2, ny=3, nz=32, batch=1, radius=0.0, tau=0.7, accel_z=0.0)
    mask = np.ones((32, 3, 2), bool)
    o = _oracle_pipe(O, cfg)
    f = np.zeros((27, 32, 3, 2))
    for k in range(32):
        f[:, k] = O.feq(1.0, [0.01 * np.sin(2 * np.pi * k / 32), 0.0, 0.02])[:, None, None]
    _, w, _ = O.lattice()
    g = (f - w[:, None, None, None]).astype(np.float32)
    o.set_f(g.astype(np.float64) + w[:, None, None, None], 0)
    p = gpu.Pipe(cfg)
    p.set_populations(torch.from_numpy(g[None]).cuda(), 0)
    p.step(200)
    o.step(200)
    _, u_g = _gpu_u(p)
    _, u_o = o.moments()
    assert _vel_err(u_g[0], u_o, mask) < 1e-5


# ------------------------------------------------------------------ FP64 reference storage
def test_fp64_storage_forced_run(gpu, O):
    """FP64 deviations, collision and force tables: the forced log-law run
    matches the oracle after 50 steps to FP32 export precision in the
    populations and to rounding level in the FP64 channels (mass, momentum
    and energy sums)."""
    cfg = _forced_cfg(nx=30, ny=28, nz=24, radius=13.4, storage=2)
    amps = _amps(cfg, seed=9)
    p = gpu.Pipe(cfg, amps)
    o = _oracle_pipe(O, cfg, amps[0])
    p.step(50)
    o.step(50)
    g = p.populations().cpu().numpy()[0].astype(np.float64)  # exported as FP32
    _, w, _ = O.lattice()
    go = o.get_f() - w[:, None, None, None]
    mask = o.fluid_mask()
    err = np.abs(g[:, mask] - go[:, mask]).max() / np.abs(go[:, mask]).max()
    _log(f"fp64 storage: population error {err:.3e} (FP32 export)")
    assert err < 2e-7  # the export rounds to FP32
    d = p.diagnostics(raise_on_nan=True)[0]
    s = o.sums()
    e, eo = p.energy()[0], o.energy()
    mom = np.abs(d[1:4] - s[1:4]).max() / np.abs(s[1:4]).max()
    _log(f"fp64 storage: mass {abs(d[0] - s[0]) / s[0]:.2e}, momentum {mom:.2e}, energy {abs(e - eo) / eo:.2e}")
    assert abs(d[0] - s[0]) < 1e-12 * s[0]
    assert mom < 1e-11
    assert abs(e - eo) < 1e-11 * eo


# ------------------------------------------------------------------ FP16 storage
def test_fp16_storage_forced_run(gpu, O):
    """FP16 scaled-deviation storage, FP32 collision: velocity error against
    the FP64 oracle after 50 forced steps stays below 1e-3 of max|u|."""
    cfg = _forced_cfg(nx=30, ny=28, nz=24, radius=13.4, storage=1)
    amps = _amps(cfg, seed=9)
    p = gpu.Pipe(cfg, amps)
    o = _oracle_pipe(O, cfg, amps[0])
    p.step(50)
    o.step(50)
    _, u_g = _gpu_u(p)
    _, u_o = o.moments()
    err = _vel_err(u_g[0], u_o, o.fluid_mask())
    _log(f"fp16 forced run velocity error {err:.3e}")
    assert err < 1e-3


def test_fp16_storage_laminar(gpu, O):
    """Laminar pipe in FP16 storage, 100 steps: velocity within 1e-3 of the
    oracle (the stated FP16 accuracy: its deviations carry 11 significant
    bits, and the laminar case, with deviations of ~1e-6 relative to the
    weights, is its worst case)."""
    cfg = LI.preset("laminar")
    cfg["storage"] = 1
    p = gpu.Pipe(cfg)
    p.step(100)
    o = _oracle_pipe(O, cfg)
    o.step(100)
    _, u_g = _gpu_u(p)
    _, u_o = o.moments()
    err = _vel_err(u_g[0], u_o, o.fluid_mask())
    _log(f"fp16 laminar velocity error {err:.3e}")
    assert err < 1e-3


# ------------------------------------------------------------------ batching, graphs, checkpoints
def test_batch_equals_single_pipes(gpu):
    cfg = _forced_cfg(batch=3)
    amps = _amps(cfg, seed=21)
    pb = gpu.Pipe(cfg, amps)
    pb.step(17)
    gb = pb.populations().cpu().numpy()
    for b in range(3):
        c1 = dict(cfg, batch=1)
        p1 = gpu.Pipe(c1, amps[b:b + 1])
        p1.step(17)
        g1 = p1.populations().cpu().numpy()[0]
        assert np.array_equal(gb[b], g1), f"pipe {b}"


@pytest.mark.parametrize("storage", [0, 1])
def test_graph_replay_equals_eager(gpu, storage):
    cfg = _forced_cfg(storage=storage)
    amps = _amps(cfg)
    pe = gpu.Pipe(cfg, amps)
    pg = gpu.Pipe(cfg, amps)
    pe.step(3)
    pg.step(3)
    for n in (10, 7, 16):  # replays at both buffer parities plus eager remainders
        pe.step(n)
        pg.step_graph(n, 4)
        assert pg.step_index == pe.step_index
        assert np.array_equal(pe.populations().cpu().numpy(), pg.populations().cpu().numpy())


def test_save_load_roundtrip(gpu):
    cfg = _forced_cfg()
    amps = _amps(cfg)
    p = gpu.Pipe(cfg, amps)
    p.step(5)
    blob, s = p.save()
    blob = blob.clone()
    p.step(9)
    a = p.populations().cpu().numpy()
    p.load(blob, s)
    assert p.step_index == 5
    p.step(9)
    assert np.array_equal(a, p.populations().cpu().numpy())


# ------------------------------------------------------------------ diagnostics
def test_diagnostics_match_oracle_sums_and_mass_is_conserved(gpu, O):
    cfg = _forced_cfg(nx=30, ny=28, nz=24, radius=13.4)
    amps = _amps(cfg, seed=3)
    p = gpu.Pipe(cfg, amps)
    o = _oracle_pipe(O, cfg, amps[0])
    d0 = p.diagnostics(raise_on_nan=True)[0]
    s0 = o.sums()
    assert abs(d0[0] - s0[0]) < 1e-9 * s0[0]
    np.testing.assert_allclose(d0[1:4], s0[1:4], rtol=0, atol=1e-6 * np.abs(s0[1:4]).max() + 1e-9 * s0[0])
    p.step(40)
    o.step(40)
    d1 = p.diagnostics(raise_on_nan=True)[0]
    s1 = o.sums()
    assert abs(d1[0] / d0[0] - 1) < 1e-7
    np.testing.assert_allclose(d1[1:4], s1[1:4], rtol=0, atol=1e-5 * np.abs(s1[1:4]).max() + 1e-9 * s1[0])
    assert d1[4] == 0


def test_diagnostics_flag_non_finite(gpu, O):
    cfg = LI.preset("laminar")
    p = gpu.Pipe(cfg)
    g = p.populations()
    mask = torch.from_numpy(_fluid(O, cfg)).cuda()
    idx = torch.nonzero(mask)[7]
    g[0, 13, idx[0], idx[1], idx[2]] = float("nan")
    p.set_populations(g, 0)
    d = p.diagnostics()
    assert d[0, 4] >= 1
    with pytest.raises(gpu.LbmError):
        p.diagnostics(raise_on_nan=True)


def test_profile_sums_match_oracle(gpu, O):
    cfg = _forced_cfg(nx=30, ny=28, nz=24, radius=13.4)
    amps = _amps(cfg, seed=4)
    p = gpu.Pipe(cfg, amps)
    o = _oracle_pipe(O, cfg, amps[0])
    acc = np.zeros((cfg["ny"], cfg["nx"], 5))
    for _ in range(3):
        p.step(7)
        o.step(7)
        p.profile_accumulate()
        _, u = o.moments()
        uz = u[2]
        for q in range(4):
            acc[..., q] += (uz ** (q + 1)).sum(0)
        acc[..., 4] += cfg["nz"]
    got = p.profile_read()[0]
    mask = o.fluid_mask()[0]
    for q in range(4):
        ref = acc[..., q][mask]
        assert np.abs(got[..., q][mask] - ref).max() <= 1e-5 * np.abs(ref).max() * (q + 1)
    assert np.array_equal(got[..., 4][mask], acc[..., 4][mask])
    assert np.all(got[~mask] == 0)


def test_energy_matches_oracle(gpu, O):
    cfg = _forced_cfg(nx=30, ny=28, nz=24, radius=13.4)
    amps = _amps(cfg, seed=4)
    p = gpu.Pipe(cfg, amps)
    o = _oracle_pipe(O, cfg, amps[0])
    p.step(11)
    o.step(11)
    e = p.energy()[0]
    assert abs(e - o.energy()) < 1e-5 * o.energy()


def test_recompute_records_the_stepped_states(gpu):
    cfg = _forced_cfg()
    amps = _amps(cfg)
    p = gpu.Pipe(cfg, amps)
    p.step(6)
    start, s0 = p.save()
    start = start.clone()
    ref = []
    for j in range(5):
        ref.append(p.save()[0].clone())
        p.step(1)
    ring = torch.empty((5, p.state_bytes), dtype=torch.uint8, device="cuda")
    p.recompute(start, s0, ring)
    torch.cuda.synchronize()
    ncol, P = int(p.layout.n_fluid_columns), int(p.layout.plane_pitch)
    ps, nz = int(p.layout.population_stride), cfg["nz"]

    def valid(blob):  # the stored columns of every (population, plane); padding excluded
        pops = blob[:4 * 27 * ps].view(torch.float32).reshape(27, ps)[:, :nz * P]
        return pops.reshape(27 * nz, P)[:, :ncol]

    for j in range(5):
        assert torch.equal(valid(ring[j]), valid(ref[j])), j
    assert p.step_index == 11  # own state untouched


def test_energy_accumulate_matches_energy(gpu):
    cfg = _forced_cfg(batch=2)
    amps = _amps(cfg)
    p = gpu.Pipe(cfg, amps)
    acc = torch.zeros(2, dtype=torch.float64, device="cuda")
    tot = np.zeros(2)
    for _ in range(3):
        p.step(4)
        p.energy_accumulate(acc)
        tot += p.energy()
    np.testing.assert_allclose(acc.cpu().numpy(), tot, rtol=1e-14, atol=0)
