"""Coherent-structure identification on the GPU (Section II.C) against the
oracle (needs an MI355X).

* Ring samples of u_z at r0 = 0.78 R: against bilinear interpolation of the
  FP64 oracle's velocity of the same state (random deviations, trigger force
  active, so u_z carries the a/2 shift with its z dependence), for FP32,
  FP64 and FP16 storage, the AA pattern at an odd step and the interpolated
  wall.  Tolerance: FP32 rounding of the velocity, 1e-6 of max|u_z| (the
  FP16 state differs from the oracle's FP64 input by its own rounding).
* Spectra: the GPU transform of the plane-averaged correlation against the
  oracle's literal correlation sum and DFT on the same ring samples (FP64
  on both sides, 1e-9 relative); the dominant mode, an argmax taken in FP64
  on both sides, equal.
* A field with a prescribed azimuthal structure: the dominant mode found.
"""
import sys

import numpy as np
import pytest

import lbm_inputs as LI
from oracle import structures as S

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
    cfg = dict(nx=40, ny=38, nz=12, batch=1, radius=17.6, tau=0.56, accel_z=3e-6, n_modes=6,
               kz=3.0, kappa=0.5, l0_frac=0.2, l_frac=0.4, period=40.0, force_off_step=1000,
               storage=0, wall=0, pattern=0, init=1, u_tau=0.01)
    cfg.update(kw)
    return cfg


def _amps(cfg, boost=20.0):
    return LI.batch_amplitudes(5, cfg["batch"], cfg["n_modes"], cfg["u_tau"], cfg["period"]) * boost


def _state(P, O, cfg, amps, s, g0):
    """GPU and oracle pipes holding f = w + g0 at step s."""
    p = P.Pipe(cfg, amps)
    p.set_populations(torch.from_numpy(g0[None]).cuda(), step=s)
    o = O.Pipe(O.make_config(**cfg), amps[0])
    _, w, _ = O.lattice()
    mask = o.fluid_mask()
    f0 = g0.astype(np.float64) + w[:, None, None, None]
    f0[:, ~mask] = 0.0
    o.set_f(f0, s)
    return p, o


@pytest.mark.parametrize("kw,s", [
    (dict(), 10), (dict(storage=2), 10), (dict(storage=1), 10), (dict(pattern=1), 11), (dict(wall=1), 10),
])
def test_ring_samples_match_oracle(P, oracle_mod, kw, s):
    O = oracle_mod
    cfg = _cfg(**kw)
    amps = _amps(cfg)
    mask = O.Pipe(O.make_config(**cfg)).fluid_mask()
    g0 = LI.random_deviations(31, (cfg["nz"], cfg["ny"], cfg["nx"]), 0.01)
    g0[:, ~mask] = 0.0
    p, o = _state(P, O, cfg, amps, s, g0)
    r0, n = 0.78 * cfg["radius"], 256
    ring = p.ring_sample(r0, n)[0].cpu().numpy().astype(np.float64)
    _, u = o.moments()
    ref = S.ring_sample(u[2], r0, n)
    err = np.abs(ring - ref).max() / np.abs(ref).max()
    _log(f"ring samples {kw} step {s}: relative error {err:.3e}")
    tol = 1e-3 if cfg["storage"] == 1 else 1e-6
    assert err <= tol


def test_spectrum_and_dominant_mode_match_oracle(P, oracle_mod):
    O = oracle_mod
    cfg = _cfg(batch=2)
    amps = _amps(cfg)
    mask = O.Pipe(O.make_config(**cfg)).fluid_mask()
    g = np.stack([LI.random_deviations(40 + b, (cfg["nz"], cfg["ny"], cfg["nx"]), 0.01) for b in range(2)])
    g[:, :, ~mask] = 0.0
    p = P.Pipe(cfg, amps)
    p.set_populations(torch.from_numpy(g).cuda(), step=10)
    n, mmax = 200, 40
    ring = p.ring_sample(0.78 * cfg["radius"], n)
    spec, mean, dom = p.ring_spectrum(ring, mmax)
    ring = ring.cpu().numpy().astype(np.float64)
    spec, mean, dom = spec.cpu().numpy(), mean.cpu().numpy(), dom.cpu().numpy()
    for b in range(2):
        ref = S.correlation_spectrum(ring[b], mmax)
        np.testing.assert_allclose(mean[b], ref, rtol=1e-9, atol=1e-12 * n)
        for z in (0, cfg["nz"] - 1):
            np.testing.assert_allclose(spec[b, z], S.correlation_spectrum(ring[b, z:z + 1], mmax),
                                       rtol=1e-9, atol=1e-12 * n)
        assert dom[b] == S.dominant_mode(ref)
        _log(f"pipe {b}: dominant mode {dom[b]}")


def test_dominant_mode_of_a_structured_field(P, oracle_mod):
    """u_z = U(r) + eps cos(5 theta + phi(z)) g(r) (plus 1% noise) written as
    the equilibrium of that velocity: dominant mode 5 on the GPU and in the
    oracle's pipeline on the oracle's own velocity."""
    O = oracle_mod
    cfg = _cfg(n_modes=0, accel_z=0.0, init=0)
    nx, ny, nz, R = cfg["nx"], cfg["ny"], cfg["nz"], cfg["radius"]
    c, w, _ = O.lattice()
    mask = O.Pipe(O.make_config(**cfg)).fluid_mask()
    rng = np.random.default_rng(9)
    g0 = np.zeros((27, nz, ny, nx), np.float32)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if not mask[z, y, x]:
                    continue
                dx, dy = x - 0.5 * (nx - 1), y - 0.5 * (ny - 1)
                r, th = np.hypot(dx, dy), np.arctan2(dy, dx)
                uz = 0.05 * (1 - (r / R) ** 2) + 0.004 * np.cos(5 * th + 0.3 * z) * np.sin(np.pi * r / R) \
                    + 0.0004 * rng.normal()
                g0[:, z, y, x] = O.feq(1.0, [0.0, 0.0, uz]) - w
    p, o = _state(P, O, cfg, np.zeros((1, 0)), 0, g0)
    r0, n = 0.78 * R, 256
    _, _, dom = p.ring_spectrum(p.ring_sample(r0, n), 32)
    _, u = o.moments()
    ref = S.correlation_spectrum(S.ring_sample(u[2], r0, n), 32)
    assert S.dominant_mode(ref) == 5
    assert int(dom.cpu()[0]) == 5


def test_ring_arguments_are_checked(P):
    cfg = _cfg()
    p = P.Pipe(cfg, _amps(cfg))
    with pytest.raises(P.LbmError):
        p.ring_sample(cfg["radius"] - 0.3, 64)  # touches the wall
    with pytest.raises(P.LbmError):
        p.ring_sample(5.0, 4097)
    ring = p.ring_sample(5.0, 64)
    with pytest.raises(P.LbmError):
        p.ring_spectrum(ring, 33)
