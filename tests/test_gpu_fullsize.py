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


# FP16 storage codec (include/lbm.h): a value g of population i produced by
# column y is held as h = fp16_rne(2^k g - E_c(y)) (one rounding of the exact
# difference) and read as fp32(h / 2^k + E_c(y) / 2^k), 2^k by shell, c = c_z
# of i
FP16_SCALE = np.array([4.0 if s == 0 else 16.0 if s == 1 else 64.0 if s == 2 else 256.0
                       for s in (0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3)])


def _fp16_refs(O, cfg):
    """The codec's per-column references E_c, c_z = 0, +1, -1 ([3][ny][nx]),
    from the oracle's initial state: the initial deviation of population i
    is w_i d_c(u0) and 2^k w_i = 32/27, so E_c = fp32(2^k g_i) with
    populations 0, 5, 6 (rest, +z, -z)."""
    _, w, _ = O.lattice()
    g = O.Pipe(O.make_config(**dict(cfg, nz=1))).get_f()[:, 0] - w[:, None, None]
    return np.stack([np.float32(4.0 * g[0]), np.float32(16.0 * g[5]), np.float32(16.0 * g[6])])


def _czi(c):
    return 0 if c == 0 else (1 if c > 0 else 2)


def _fp16_round(g, s, E):
    """What FP16 storage returns for the FP32 value g of scale s and reference E."""
    # 2^k g - E is exact in FP64 (FP32 operands, power-of-two scale); numpy
    # rounds FP64 to FP16 directly, once
    h = np.float64(np.float16(np.float64(np.float32(g)) * s - np.float64(E)))
    return np.float64(np.float32(h / s + np.float64(E) / s))


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
    E = _fp16_refs(O, cfg) if fp16 else None

    def producer_ref(x, y, i):
        """FP16 reference of the value population i receives at (x, y): that
        of its producer, x - c_i, or x itself (as opp(i)) for a bounce-back."""
        sx, sy = (x - c[i, 0]) % nx, (y - c[i, 1]) % ny
        if mask2d[sy, sx]:
            return E[_czi(c[i, 2]), sy, sx]
        return E[_czi(-c[i, 2]), y, x]

    def f_at(x, y, z):
        flat = np.full(27, (z * ny + y) * nx + x)
        g0 = LI.random_deviations_at(SEED, shape, np.arange(27), flat, AMP)
        if fp16:  # the state writer encodes each input with its producer's reference
            g0 = np.array([_fp16_round(g0[i], FP16_SCALE[i], producer_ref(x, y, i)) for i in range(27)])
        return w + g0.astype(np.float64)

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
    if fp16:  # one FP16 rounding of each stored output: half an ulp of 2^k g - E, relative 2^-11
        ref = np.array([[producer_ref(x, y, i) / FP16_SCALE[i] for i in range(27)] for (x, y, z) in pick])
        tol = tol + 2.0 ** -11 * np.abs(expect - ref) + 2.0 ** -25 / FP16_SCALE
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
    """Adjoint workload at full size (96x96x384, 2000 steps, checkpoints every
    100), against central differences of the FP64-storage forward (a step of
    1% or 3% of the largest amplitude; differences of the FP32 forward move
    the state by only a few FP32 ulps and cannot resolve 1e-4).  Stated
    accuracies: the FP32 forward with the adjoint state stored in FP32 (the
    path the benchmark times) or FP64, FP64 arithmetic in both, within 1e-4
    (measured 3.6e-5 for both: what remains is the FP32 forward's own
    trajectory); the FP64 forward within 1e-6 (6.7e-8)."""
    from paper_2405_12082_amd.adjoint import EnergyAdjoint
    cfg = LI.preset("adjoint")
    amps = LI.preset_amplitudes(cfg)
    b, e, C = cfg["obs_begin"], cfg["obs_end"], cfg["checkpoint_every"]
    grads = {}
    for name, c, prec in (("fwd32_adj32", cfg, "fp32"), ("fwd32_adj64", cfg, "fp64")):
        run = EnergyAdjoint(c, b, e, checkpoint_every=C, precision=prec)
        grads[name] = run.gradient(amps)[1][0]
        del run
    run64 = EnergyAdjoint(dict(cfg, storage=2), b, e, checkpoint_every=C, precision="fp64")
    J64, g64 = run64.gradient(amps)
    grads["fwd64_adj64"] = g64[0]
    best = {k: np.inf for k in grads}
    for frac in (3e-2, 1e-2):
        eps = frac * np.abs(amps).max()
        fd = np.zeros_like(g64[0])
        for q in range(fd.size):
            ap, am = amps.copy(), amps.copy()
            ap[0, q] += eps
            am[0, q] -= eps
            fd[q] = (run64.objective(ap)[0] - run64.objective(am)[0]) / (2 * eps)
        for k, g in grads.items():
            rel = np.linalg.norm(g - fd) / np.linalg.norm(fd)
            best[k] = min(best[k], rel)
            _log(f"eps = {frac:g} * max|amps|: {k} vs FD {rel:.3e}")
    assert best["fwd32_adj32"] < 1e-4
    assert best["fwd32_adj64"] < 1e-4
    assert best["fwd64_adj64"] < 1e-6


def test_pipe_beyond_2_31_state_elements_one_step_sampled_parity(P, oracle_mod):
    """A pipe whose state holds more than 2^31 elements: 384^2 x 1024 with
    R = 180, 104 M fluid nodes, 2.8 G elements per buffer (the kernels take
    64-bit pipe and population bases and 32-bit byte offsets within one
    population, 417 MB here); the one-step sampled parity above, FP32."""
    cfg = dict(nx=384, ny=384, nz=1024, radius=180.0)
    lay = P.describe(P.make_config(**dict(LI.preset("turbulent"), **cfg)))
    assert 27 * lay.population_stride > 2 ** 31
    _sampled_step_parity(P, oracle_mod, "turbulent", 301, **cfg)
