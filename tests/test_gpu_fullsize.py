"""Parity at the full workload sizes, in the launch configuration bench.py
times (needs an MI355X).

* The turbulent pipe 192x192x1152 (R = 90; FP32, FP16 storage, AA
  pattern) and the paper's pipe 300x300x600 (R = 149.5, interpolated
  wall): one fused step from seeded random
  deviations with the trigger force active; every population of ~400
  sampled nodes (wall-adjacent columns, both periodic z ends, the last
  columns of the layout, random interior nodes) against the FP64 oracle's
  collide + stream computed node by node.
* The adjoint pipe 96x96x384 (R = 45), 2000 steps: the gradient of the
  streamwise energy over steps 1501..2000 against central finite
  differences of the GPU forward model, within 1e-4 (2-norm).
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


SEED, AMP = 2024, 0.02


# FP16 storage codec (include/lbm.h): g stored as fp16_rne(g 2^k), 2^k by shell
FP16_SCALE = np.array([4.0 if s == 0 else 16.0 if s == 1 else 64.0 if s == 2 else 256.0
                       for s in (0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3)])


def _fp16_stored(g):
    """What FP16 storage holds and returns for FP32 deviations g [..., 27]."""
    g = np.asarray(g, np.float32)
    return (np.float16(g * FP16_SCALE.astype(np.float32)).astype(np.float64) / FP16_SCALE)


def _sampled_step_parity(P, O, name, s, **over):
    """One fused step of preset ``name`` from seeded random deviations at step
    s, in the default launch geometry (as bench.py); ~400 sampled nodes (wall
    columns, both periodic z ends, the last columns of the layout, random
    interior nodes), every population against the FP64 oracle's collide +
    stream computed node by node (halfway bounce-back or, wall = 1, the
    interpolation of Eqs. (fbc1)/(fbc2) with the oracle's wall fraction).
    ``over`` overrides config fields (storage, pattern).  FP16 storage: the
    oracle starts from the FP16-stored inputs, and the tolerance adds one
    FP16 rounding of each output."""
    cfg = dict(LI.preset(name), **over)
    amps = LI.preset_amplitudes(cfg)
    nx, ny, nz = LI.dims_of(cfg)
    ocfg = O.make_config(**cfg)
    mask2d = O.Pipe(O.make_config(**dict(cfg, nz=1))).fluid_mask()[0]
    _log(f"full-size parity ({name}, wall {cfg['wall']}): {nx}x{ny}x{nz}, {int(mask2d.sum())} fluid columns")

    pipe = P.Pipe(cfg, amps)  # default launch geometry, as bench.py
    g = LI.random_deviations_torch(SEED, (nz, ny, nx), AMP)
    g *= torch.from_numpy(mask2d).cuda()[None, None]
    pipe.set_populations(g[None], step=s)
    torch.cuda.synchronize()
    del g
    pipe._keep = None
    torch.cuda.empty_cache()
    pipe.step(1)
    out = pipe.populations()[0]  # [27][nz][ny][nx]

    rng = np.random.default_rng(7)
    fy, fx = np.nonzero(mask2d)
    wall = np.zeros_like(mask2d)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            wall |= mask2d & ~np.roll(np.roll(mask2d, -dy, 0), -dx, 1)
    wy, wx = np.nonzero(wall)
    pick = []
    for _ in range(120):
        j = rng.integers(len(wy))
        pick.append((wx[j], wy[j], rng.integers(nz)))
    for _ in range(120):
        j = rng.integers(len(fy))
        pick.append((fx[j], fy[j], rng.integers(nz)))
    for zz in (0, nz - 1):
        for _ in range(40):
            j = rng.integers(len(fy))
            pick.append((fx[j], fy[j], zz))
    for j in range(len(fy) - 30, len(fy)):  # the last columns of the row-major layout
        pick.append((fx[j], fy[j], rng.integers(nz)))
    pick = np.array(pick)

    c, w, opp = O.lattice()
    omega = 1.0 / cfg["tau"]
    shape = (nz, ny, nx)

    fp16 = cfg.get("storage", 0) == 1

    def f_at(x, y, z):
        flat = np.full(27, (z * ny + y) * nx + x)
        g0 = LI.random_deviations_at(SEED, shape, np.arange(27), flat, AMP)
        return w + (_fp16_stored(g0) if fp16 else g0.astype(np.float64))

    def collided(x, y, z):
        a = O.force_at(ocfg, amps[0], x, y, z, s)
        return O.collide(f_at(x, y, z), a, omega)

    expect = np.zeros((len(pick), 27))
    for n, (x, y, z) in enumerate(pick):
        own = collided(x, y, z)
        for i in range(27):
            sx, sy, sz = (x - c[i, 0]) % nx, (y - c[i, 1]) % ny, (z - c[i, 2]) % nz
            if mask2d[sy, sx]:
                v = collided(sx, sy, sz)[i]
            elif cfg["wall"] == 0:
                v = own[opp[i]]
            else:
                delta = O.wall_fraction(ocfg, x, y, opp[i])
                fx_, fy_, fz_ = (x + c[i, 0]) % nx, (y + c[i, 1]) % ny, (z + c[i, 2]) % nz
                has_ff = bool(mask2d[fy_, fx_])
                far = collided(fx_, fy_, fz_)[opp[i]] if has_ff else 0.0
                v = O.bouzidi(delta, own[opp[i]], own[i], far, has_ff)
            expect[n, i] = v - w[i]
    px = torch.as_tensor(pick[:, 0], device="cuda")
    py = torch.as_tensor(pick[:, 1], device="cuda")
    pz = torch.as_tensor(pick[:, 2], device="cuda")
    got = out[:, pz, py, px].T.cpu().numpy().astype(np.float64)
    g_in_max = AMP * max(LI.DEV_SHELL_SCALE)
    tol = 64 * 2.0 ** -24 * (g_in_max + np.abs(expect).max())
    if fp16:  # one FP16 rounding of each stored output: half an ulp of g 2^k, relative 2^-11
        tol = tol + 2.0 ** -11 * np.abs(expect)
    err = np.abs(got - expect)
    _log(f"{len(pick)} sampled nodes x 27 populations (storage {cfg.get('storage', 0)}, pattern {cfg.get('pattern', 0)}): max abs error {err.max():.3e} "
         f"(max tolerance {np.max(tol):.3e}, worst ratio {np.max(err / tol):.3f})")
    assert np.all(err <= tol)


def test_turbulent_pipe_one_step_sampled_parity(P, oracle_mod):
    # s = 301: sin(2 pi s / T) ~ 1 with T = 1206, trigger force at full strength
    _sampled_step_parity(P, oracle_mod, "turbulent", 301)


def test_turbulent_pipe_fp16_one_step_sampled_parity(P, oracle_mod):
    """FP16 storage, as the bench's fp16 leg (its default launch geometry)."""
    _sampled_step_parity(P, oracle_mod, "turbulent", 301, storage=1)


@pytest.mark.parametrize("s", [301, 302])
def test_turbulent_pipe_aa_one_step_sampled_parity(P, oracle_mod, s):
    """AA pattern in place, as the bench's aa leg, from an odd (exchanged
    slots) and an even (own slots) step index."""
    _sampled_step_parity(P, oracle_mod, "turbulent", s, pattern=1)


def test_paper_pipe_one_step_sampled_parity(P, oracle_mod):
    """The paper's pipe, 300x300x600 (R = 149.5) with the interpolated wall
    and its k_theta = 2 trigger mode; s = 501: sin(2 pi s / T) = 1 at T = 2004."""
    _sampled_step_parity(P, oracle_mod, "paper", 501)


def test_adjoint_pipe_gradient_vs_central_differences(P):
    """Adjoint workload at full size.  The check against central differences
    runs on the FP64 reference forward (storage = 2): a step of size eps on
    the amplitudes moves the state by only a few FP32 units in the last
    place, so differences of the FP32 forward cannot resolve 1e-4 (the FP32
    product adjoint's agreement with the exact derivative is checked against
    the oracle's complex-step tangent in test_gpu_adjoint.py)."""
    from paper_2405_12082_amd.adjoint import EnergyAdjoint
    cfg = LI.preset("adjoint")
    amps = LI.preset_amplitudes(cfg)
    b, e, C = cfg["obs_begin"], cfg["obs_end"], cfg["checkpoint_every"]
    run32 = EnergyAdjoint(cfg, b, e, checkpoint_every=C, precision="fp32")
    J32, g32 = run32.gradient(amps)
    del run32
    run64 = EnergyAdjoint(dict(cfg, storage=2), b, e, checkpoint_every=C, precision="fp64")
    J64, g64 = run64.gradient(amps)
    g32, g64 = g32[0], g64[0]
    _log(f"adjoint pipe: J32 = {J32[0]:.9e}, J64 = {J64[0]:.9e}, |g| = {np.linalg.norm(g64):.4e}")
    best = np.inf
    for frac in (3e-2, 1e-2):
        eps = frac * np.abs(amps).max()
        fd = np.zeros_like(g64)
        for q in range(g64.size):
            ap, am = amps.copy(), amps.copy()
            ap[0, q] += eps
            am[0, q] -= eps
            fd[q] = (run64.objective(ap)[0] - run64.objective(am)[0]) / (2 * eps)
        rel = np.linalg.norm(g64 - fd) / np.linalg.norm(fd)
        rel32 = np.linalg.norm(g32 - fd) / np.linalg.norm(fd)
        best = min(best, rel)
        _log(f"eps = {frac:g} * max|amps|: FP64 adjoint vs FD {rel:.3e}; FP32 product adjoint vs FD {rel32:.3e}")
    assert best < 1e-4
    assert np.linalg.norm(g32 - g64) / np.linalg.norm(g64) < 1e-2
