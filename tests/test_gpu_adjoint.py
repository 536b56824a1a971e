"""GPU discrete adjoint against the FP64 oracle adjoint and against central
finite differences of the GPU forward model (needs an MI355X).

Tolerances: the GPU gradient (FP32 forward states, FP32 or FP64 adjoint
states, FP64 vector-Jacobian arithmetic and gradient accumulation) agrees
with the oracle's FP64 adjoint to 1e-6 relative (max norm over the
amplitudes) on a tiny pipe over 40 steps (the FP32 forward states' rounding,
6e-8 relative per state), with the oracle's tangent over 2000 steps to 1e-5,
and with central finite differences of its own forward model to 1e-4
relative (2-norm).
"""
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
    from paper_2405_12082_amd import adjoint
    P.lib()
    return adjoint


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


TINY = dict(nx=12, ny=12, nz=8, batch=1, radius=5.0, tau=0.6, accel_z=1e-5, n_modes=2, kz=1.0, kappa=0.5,
            l0_frac=0.2, l_frac=0.4, period=20.0, force_off_step=1000, init=1, u_tau=0.01)
TINY_AMPS = np.array([1e-4, 2e-4, 3e-4, 1.5e-4])


@pytest.mark.parametrize("precision,wall,nz,storage,tol", [
    ("fp32", 0, 8, 0, 1e-6), ("fp64", 0, 8, 0, 1e-6), ("fp32", 1, 8, 0, 1e-6), ("fp64", 1, 8, 0, 1e-6),
    # FP16 forward states (11 significant bits of each deviation from its
    # column's reference): the gradient target, 1e-4 (measured 1.2e-5..1.5e-5)
    ("fp32", 0, 8, 1, 1e-4), ("fp64", 0, 8, 1, 1e-4), ("fp32", 1, 8, 1, 1e-4),
    # FP64 storage: FP64 forward, adjoint and force tables, so the hand-derived
    # vector-Jacobian products meet the oracle's complex-step adjoint at
    # rounding level (measured 1e-12)
    ("fp64", 0, 8, 2, 1e-10), ("fp64", 1, 8, 2, 1e-10),
    # one and two planes (the transposed gather along z lands in the same or
    # the other plane): there the gradient is 10-1000x smaller relative to
    # the state (the k_z = 1 forcing alternates between the planes), below
    # what FP32 forward states resolve to 1e-4, so with the FP64 forward
    ("fp64", 0, 1, 2, 1e-10), ("fp64", 0, 2, 2, 1e-10), ("fp64", 1, 2, 2, 1e-10)])
def test_adjoint_matches_oracle_adjoint(gpu, oracle_mod, precision, wall, nz, storage, tol):
    """wall = 1: the interpolated wall; the 12x12 section (R = 5) has cut
    links in both modes of the interpolation and nodes with two cut links on
    one line.  Gradient error (max norm, relative) within tol of the oracle's
    FP64 adjoint."""
    O = oracle_mod
    cfg = dict(TINY, wall=wall, nz=nz, storage=storage)
    run = gpu.EnergyAdjoint(cfg, 20, 40, checkpoint_every=7, precision=precision)
    J, g = run.gradient(TINY_AMPS[None])
    Jo, go = O.adjoint_gradient(O.make_config(**cfg), TINY_AMPS, 20, 40)
    err = np.abs(g[0] - go).max() / np.abs(go).max()
    _log(f"J gpu {J[0]:.10e} oracle {Jo:.10e}; gradient error vs oracle adjoint {err:.3e}")
    # FP32 state: u_z to ~1e-6 relative; FP16: ~1e-5 (measured 8.5e-6); FP64 storage: rounding level
    assert abs(J[0] - Jo) < {0: 1e-5, 1: 1e-4, 2: 1e-12}[storage] * abs(Jo)
    assert err < tol


@pytest.mark.parametrize("precision,tol,wall,storage", [("fp64", 1e-5, 0, 0), ("fp32", 1e-5, 0, 0), ("fp64", 1e-5, 1, 0),
                                                      ("fp32", 1e-4, 0, 1),
                                                      ("fp64", 1e-10, 0, 2), ("fp64", 1e-10, 1, 2)])
def test_long_horizon_adjoint_matches_oracle_tangent(gpu, oracle_mod, precision, tol, wall, storage):
    """2000 steps of a 16x16x32 pipe (R = 7) with the adjoint workload's
    physics: the GPU adjoint against the oracle's complex-step tangent of
    the whole FP64 run (the exact derivative); wall = 1 with the
    interpolated wall; storage 0: FP32 forward, 1: FP16 forward (the
    gradient target 1e-4, measured 3.1e-5), 2: FP64 forward (rounding
    level)."""
    O = oracle_mod
    cfg = LI.preset("adjoint")
    cfg.update(nx=16, ny=16, nz=32, radius=7.0, accel_z=2 * cfg["u_tau"] ** 2 / 7.0,
               period=float(round(0.052 * 7.0 / cfg["u_tau"])), force_off_step=2000, wall=wall, storage=storage)
    amps = LI.preset_amplitudes(cfg)
    J, g = gpu.EnergyAdjoint(cfg, 1501, 2001, checkpoint_every=100, precision=precision).gradient(amps)
    Jt, gt = O.tangent_gradient(O.make_config(**cfg), amps[0], 1501, 2001)
    err = np.linalg.norm(g[0] - gt) / np.linalg.norm(gt)
    _log(f"{precision} adjoint (storage {storage}) vs oracle tangent over 2000 steps: {err:.3e}")
    assert err < tol


def test_checkpoint_interval_does_not_change_the_gradient(gpu):
    g1 = gpu.EnergyAdjoint(TINY, 20, 40, checkpoint_every=7).gradient(TINY_AMPS[None])[1]
    g2 = gpu.EnergyAdjoint(TINY, 20, 40, checkpoint_every=40).gradient(TINY_AMPS[None])[1]
    assert np.array_equal(g1, g2)


def test_batched_adjoint_equals_single_pipes(gpu):
    cfg = dict(TINY, batch=3)
    amps = np.stack([TINY_AMPS, 0.5 * TINY_AMPS, TINY_AMPS[::-1].copy()])
    Jb, gb = gpu.EnergyAdjoint(cfg, 20, 40, checkpoint_every=10).gradient(amps)
    for b in range(3):
        J1, g1 = gpu.EnergyAdjoint(TINY, 20, 40, checkpoint_every=10).gradient(amps[b:b + 1])
        assert J1[0] == Jb[b]
        assert np.array_equal(g1[0], gb[b])


def test_autograd_function(gpu):
    run = gpu.EnergyAdjoint(TINY, 20, 40, checkpoint_every=9)
    amps = torch.tensor(TINY_AMPS[None], dtype=torch.float64, requires_grad=True)
    J = gpu.PipeEnergy.apply(amps, run)
    (3.0 * J.sum()).backward()
    _, g = gpu.EnergyAdjoint(TINY, 20, 40, checkpoint_every=9).gradient(TINY_AMPS[None])
    np.testing.assert_allclose(amps.grad.numpy(), 3.0 * g, rtol=0, atol=0)


def _fd_config():
    # a small pipe in the shape of the adjoint workload (nu = 0.0032, trigger
    # force active throughout, log-law start)
    cfg = LI.preset("adjoint")
    cfg.update(nx=32, ny=32, nz=96, radius=15.0)
    cfg["period"] = float(round(0.052 * 15.0 / cfg["u_tau"]))
    return cfg


def test_adjoint_matches_central_differences(gpu):
    cfg = _fd_config()
    b, e = 150, 300
    amps = LI.preset_amplitudes(cfg) * 20.0
    run = gpu.EnergyAdjoint(cfg, b, e, checkpoint_every=50)
    J, g = run.gradient(amps)
    g = g[0]
    rel = {}
    for frac in (1e-1, 3e-2):
        fd = np.zeros_like(g)
        for q in range(g.size):
            eps = frac * np.abs(amps).max()
            ap, am = amps.copy(), amps.copy()
            ap[0, q] += eps
            am[0, q] -= eps
            fd[q] = (run.objective(ap)[0] - run.objective(am)[0]) / (2 * eps)
        rel[frac] = np.linalg.norm(g - fd) / np.linalg.norm(fd)
        _log(f"eps = {frac:g} * max|amps|: |g - g_fd| / |g_fd| = {rel[frac]:.3e}")
    assert min(rel.values()) < 1e-4


@pytest.mark.parametrize("storage,wall", [(0, 0), (1, 0), (2, 0), (0, 1)])
def test_recompute_moments_steps_and_records(gpu, storage, wall):
    """lbm_recompute_moments: the states it steps through equal
    lbm_recompute's bitwise (compared as exported populations: the padding of
    a saved state is never written by a step), and the moments it records of
    each state sum to that state's FP64 mass and momentum (lbm_diagnostics, a
    separate reduction of the populations)."""
    import paper_2405_12082_amd as P
    cfg = dict(TINY, storage=storage, wall=wall)
    p = P.Pipe(cfg, TINY_AMPS[None])
    p.step(5)
    start, s0 = p.save()
    n = 4
    ring = torch.empty((n + 1, p.state_bytes), dtype=torch.uint8, device="cuda")
    p.recompute(start, s0, ring)
    scratch = torch.empty((2, p.state_bytes), dtype=torch.uint8, device="cuda")
    rec = torch.empty((n, p.record_bytes), dtype=torch.uint8, device="cuda")
    p.recompute_moments(start, s0, scratch, rec)

    def pops(blob, step):
        p.load(blob, step)
        return p.populations().clone()
    for j in (n - 1, n):
        assert torch.equal(pops(scratch[j & 1], s0 + j), pops(ring[j], s0 + j)), j
    lay = p.layout
    ncol, pitch, ps, nz = int(lay.n_fluid_columns), int(lay.plane_pitch), int(lay.population_stride), cfg["nz"]
    dt = np.float64 if storage == 2 else np.float32
    nf = ncol * nz
    for j in range(n):
        p.load(ring[j], s0 + j)
        d = p.diagnostics()[0]
        r = rec[j].cpu().numpy().view(dt)[:4 * ps].reshape(4, ps)[:, :nz * pitch].reshape(4, nz, pitch)[:, :, :ncol]
        sums = r.astype(np.float64).sum(axis=(1, 2))
        ref = np.array([d[0] - nf, d[1], d[2], d[3]])
        # per-node moments rounded once in FP32 (FP64 storage: FP64)
        tol = (1e-13 if storage == 2 else 1e-6) * (np.abs(r).max() * nf)
        _log(f"storage {storage} wall {wall} state {j}: record sums - FP64 sums {np.abs(sums - ref).max():.3e} "
             f"(bound {tol:.3e})")
        assert np.all(np.abs(sums - ref) <= tol)
    p.close()


@pytest.mark.parametrize("storage,wall,precision,tol", [(0, 0, "fp32", 1e-6), (0, 1, "fp32", 1e-6),
                                                        (1, 0, "fp32", 1e-6), (2, 0, "fp64", 1e-12),
                                                        (2, 1, "fp64", 1e-12)])
def test_moment_and_state_records_give_the_same_gradient(gpu, storage, wall, precision, tol):
    """The reverse sweep from moment records against the sweep from whole
    saved states: the only difference is the forward moments, rounded once
    in the collision's arithmetic type against FP64 sums of the gathered
    state (FP64 storage: FP64 either way, summed in another order)."""
    cfg = dict(TINY, wall=wall, storage=storage)
    g = {}
    for rec in ("moments", "states"):
        run = gpu.EnergyAdjoint(cfg, 20, 40, checkpoint_every=7, precision=precision, records=rec)
        g[rec] = run.gradient(TINY_AMPS[None])[1][0]
    err = np.abs(g["moments"] - g["states"]).max() / np.abs(g["states"]).max()
    _log(f"storage {storage} wall {wall}: moment records vs state records {err:.3e}")
    assert err < tol


def test_recompute_moments_rejects_bad_arguments(gpu):
    import paper_2405_12082_amd as P
    p = P.Pipe(TINY, TINY_AMPS[None])
    start, s0 = p.save()
    sb, rb = p.state_bytes, p.record_bytes
    scratch = torch.empty((2, sb), dtype=torch.uint8, device="cuda")
    rec = torch.empty((2, rb), dtype=torch.uint8, device="cuda")
    bad_scratch = torch.empty((2, sb + 64), dtype=torch.uint8, device="cuda")  # stride not a multiple of 256
    with pytest.raises(RuntimeError, match="lbm_recompute_moments"):
        p.recompute_moments(start, s0, bad_scratch, rec)
    short = torch.empty((2, rb - 256), dtype=torch.uint8, device="cuda")  # record stride below the record size
    with pytest.raises(RuntimeError, match="lbm_recompute_moments"):
        p.recompute_moments(start, s0, scratch, short)
    with pytest.raises(RuntimeError, match="lbm_recompute_moments"):
        p.recompute_moments(scratch[1], s0, scratch, rec)  # start inside the second scratch state
    with pytest.raises(RuntimeError, match="lbm_adjoint_step_moments"):
        p.adjoint_step_moments(rec, torch.zeros((1, 4), dtype=torch.float64, device="cuda"))  # no adjoint buffers
    p.close()
    aa = P.Pipe(dict(TINY, pattern=1), TINY_AMPS[None])
    with pytest.raises(RuntimeError, match="two-buffer"):
        aa.recompute_moments(aa.save()[0], 0, scratch, rec)
    aa.close()


@pytest.mark.parametrize("storage,wall,precision", [(0, 0, "fp32"), (0, 1, "fp32"), (1, 0, "fp32"), (2, 0, "fp64")])
def test_recorded_forward_equals_checkpoint_and_recompute(gpu, storage, wall, precision):
    """recompute=False (the forward run records the moments of every state;
    the reverse sweep reads them in one call): J and the gradient equal
    checkpoint-and-recompute's bitwise, since the recording step's states and
    records are the forward's, and the sensitivities are summed per step
    whatever the split of the sweep into calls."""
    cfg = dict(TINY, wall=wall, storage=storage)
    J1, g1 = gpu.EnergyAdjoint(cfg, 20, 40, checkpoint_every=7, precision=precision).gradient(TINY_AMPS[None])
    J2, g2 = gpu.EnergyAdjoint(cfg, 20, 40, precision=precision, recompute=False).gradient(TINY_AMPS[None])
    assert np.array_equal(J1, J2) and np.array_equal(g1, g2)


def test_step_recording_rejects_bad_arguments(gpu):
    import paper_2405_12082_amd as P
    p = P.Pipe(TINY, TINY_AMPS[None])
    rec = torch.empty((2, p.record_bytes), dtype=torch.uint8, device="cuda")
    short = torch.empty((2, p.record_bytes - 256), dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError, match="lbm_step_recording"):
        p.step_recording(short)
    p.set_fused(2)
    with pytest.raises(RuntimeError, match="one step per launch"):
        p.step_recording(rec)
    p.close()
    aa = P.Pipe(dict(TINY, pattern=1), TINY_AMPS[None])
    with pytest.raises(RuntimeError, match="two-buffer"):
        aa.step_recording(rec)
    aa.close()
    with pytest.raises(ValueError):
        gpu.EnergyAdjoint(TINY, 20, 40, records="states", recompute=False)


@pytest.mark.parametrize("storage,wall", [(0, 0), (0, 1), (1, 0), (2, 0)])
def test_recorded_moments_match_the_oracle_per_node(gpu, oracle_mod, storage, wall):
    """Each recorded moment, node by node, against the FP64 oracle's moments
    of the same state (the exported populations f^n): rho - 1, and j from
    the oracle's u = j/rho + a(x, n)/2 and its force at that step.  Bound per
    node: 27 roundings of the largest population, 27 * 2^-24 * sum_i |g_i|
    (the FP32 sum, or the FP32 export the oracle starts from)."""
    import paper_2405_12082_amd as P
    O = oracle_mod
    cfg = dict(TINY, storage=storage, wall=wall)
    p = P.Pipe(cfg, TINY_AMPS[None])
    p.step(6)
    start, s0 = p.save()
    g = p.populations()[0].cpu().numpy().astype(np.float64)  # [27][nz][ny][nx]
    scratch = torch.empty((2, p.state_bytes), dtype=torch.uint8, device="cuda")
    rec = torch.empty((1, p.record_bytes), dtype=torch.uint8, device="cuda")
    p.recompute_moments(start, s0, scratch, rec)
    lay = p.layout
    ncol, pitch, ps, nz = int(lay.n_fluid_columns), int(lay.plane_pitch), int(lay.population_stride), cfg["nz"]
    dt = np.float64 if storage == 2 else np.float32
    r = rec[0].cpu().numpy().view(dt)[:4 * ps].reshape(4, ps)[:, :nz * pitch].reshape(4, nz, pitch)[:, :, :ncol]
    p.close()
    o = O.Pipe(O.make_config(**cfg), TINY_AMPS)
    mask = o.fluid_mask()
    ys, xs = np.nonzero(mask[0])  # the fluid columns in row-major order
    assert ys.size == ncol
    _, w, _ = O.lattice()
    o.set_f(g + w[:, None, None, None], s0)
    rho, u = o.moments()
    a = o.force(s0)
    ref = np.stack([rho - 1.0] + [rho * (u[q] - 0.5 * a[q]) for q in range(3)])[:, :, ys, xs]
    bound = 27 * 2.0 ** -24 * np.abs(g).sum(axis=0)[:, ys, xs]
    err = np.abs(r.astype(np.float64) - ref)
    _log(f"storage {storage} wall {wall}: records vs oracle moments, worst ratio to the bound "
         f"{(err / bound[None]).max():.3f}")
    assert np.all(err <= bound[None])
