"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the lattice Boltzmann method itself: only
the pipe configurations (plain numbers) and a counter-based random generator
for the trigger-force amplitudes.  Both the HIP library and the FP64 oracle
receive the same amplitude arrays from here.

Parameter sources (arXiv:2405.12082, Section II.B): nu = 0.0032,
u* = 0.00388, Re_tau = u* R / nu ~ 181.3, Re ~ 5329.3 (bulk velocity and
diameter), u* = sqrt(h R / 2), forcing period T ~ 0.052 T^LET with
T^LET = R / u*, k_z = 3, kappa = 0.5, l_0 = 0.2 R, l = 0.4 R.
"""
from __future__ import annotations

import math

import numpy as np

# --- the paper's printed flow parameters (Section II.B) ---
PAPER_NU = 0.0032
PAPER_U_TAU = 0.00388
PAPER_RE_TAU = 181.3
PAPER_RE_BULK = 5329.3
PAPER_RADIUS = 149.5
PAPER_GRID = (300, 300, 600)
PAPER_K_THETA = 2   # azimuthal wavenumber of the trigger force
PAPER_A0 = 50.0     # trigger-force amplitude in units of h
#: bulk-to-friction velocity ratio implied by the printed Reynolds numbers:
#: Re = U_b (2R) / nu and Re_tau = u* R / nu give U_b / u* = Re / (2 Re_tau).
BULK_OVER_UTAU = PAPER_RE_BULK / (2.0 * PAPER_RE_TAU)

_MASK64 = (1 << 64) - 1


def splitmix64(state: int):
    """One step of SplitMix64 (Steele, Lea & Flood 2014). Returns (state, out)."""
    state = (state + 0x9E3779B97F4A7C15) & _MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return state, z ^ (z >> 31)


def uniform01(seed: int, n: int) -> np.ndarray:
    """n doubles in [0, 1) from SplitMix64 seeded with ``seed`` (53-bit mantissa)."""
    s = seed & _MASK64
    out = np.empty(n)
    for k in range(n):
        s, z = splitmix64(s)
        out[k] = (z >> 11) * (1.0 / (1 << 53))
    return out


_GOLDEN = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB


def hash_uniform(seed: int, idx) -> np.ndarray:
    """Counter-based U[0,1): element ``idx`` of the SplitMix64 sequence seeded
    with ``seed`` (equal to ``uniform01(seed, n)[idx]``), vectorised."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK64) + (idx + np.uint64(1)) * np.uint64(_GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_MIX2)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def _signed(v: int) -> int:
    return v - (1 << 64) if v >= (1 << 63) else v


def hash_uniform_torch(seed: int, idx):
    """Same sequence as :func:`hash_uniform` for an int64 torch tensor of
    indices, on the tensor's device (wrapping int64 arithmetic, logical shifts)."""
    import torch

    def lsr(z, s):
        return (z >> s) & ((1 << (64 - s)) - 1)

    z = (idx + 1) * _signed(_GOLDEN) + _signed(seed & _MASK64)
    z = (z ^ lsr(z, 30)) * _signed(_MIX1)
    z = (z ^ lsr(z, 27)) * _signed(_MIX2)
    z = z ^ lsr(z, 31)
    return lsr(z, 11).to(torch.float64) * (1.0 / (1 << 53))


#: per-direction magnitude of the synthetic population deviations, by shell
#: |c|^2 = 0, 1, 2, 3 (input shaping only)
DEV_SHELL_SCALE = (0.3, 0.075, 0.01875, 0.0046875)
_SHELL = np.array([0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 3])


def deviation_scale(i):
    """Magnitude of synthetic deviations for direction(s) i (appendix order)."""
    return np.asarray(DEV_SHELL_SCALE)[_SHELL[np.asarray(i)]]


def random_deviations(seed: int, shape, amp: float = 0.02) -> np.ndarray:
    """Seeded population deviations [27][...] (float32): amp * scale_i * U(-1, 1),
    element (i, rest) taken from the counter-based stream at its flat index."""
    n = int(np.prod(shape))
    idx = np.arange(27 * n, dtype=np.uint64)
    u = hash_uniform(seed, idx).reshape((27,) + tuple(shape))
    sc = deviation_scale(np.arange(27)).reshape((27,) + (1,) * len(shape))
    return (amp * sc * (2.0 * u - 1.0)).astype(np.float32)


def random_deviations_torch(seed: int, shape, amp: float = 0.02, device="cuda"):
    """Same values as :func:`random_deviations`, generated on the device one
    direction at a time (for full-size fields): float32 tensor [27][...]."""
    import torch
    n = int(np.prod(shape))
    out = torch.empty((27,) + tuple(shape), dtype=torch.float32, device=device)
    for i in range(27):
        idx = torch.arange(i * n, (i + 1) * n, dtype=torch.int64, device=device)
        u = hash_uniform_torch(seed, idx)
        del idx
        sc = float(amp * deviation_scale(i))
        out[i] = (sc * (2.0 * u - 1.0)).to(torch.float32).reshape(shape)
        del u
    return out


def random_deviations_at(seed: int, shape, i, idx_rest, amp: float = 0.02) -> np.ndarray:
    """Entries of :func:`random_deviations` at direction(s) i and flat index
    idx_rest within ``shape`` (vectorised, float32)."""
    n = int(np.prod(shape))
    i = np.asarray(i)
    flat = i.astype(np.uint64) * np.uint64(n) + np.asarray(idx_rest, dtype=np.uint64)
    u = hash_uniform(seed, flat)
    return (amp * deviation_scale(i) * (2.0 * u - 1.0)).astype(np.float32)


def amplitude_unit(u_tau: float, period: float) -> float:
    """Acceleration per unit dimensionless amplitude: u_b * pi / T.

    A mode of peak acceleration A acting for half a period T/2 with a
    sin(2 pi t/T) time factor imparts a velocity impulse A T / pi, so an
    amplitude s in units of u_b pi / T imparts s * u_b.  The bulk velocity is
    taken from the paper's Reynolds numbers, u_b = (Re / 2 Re_tau) u*."""
    return BULK_OVER_UTAU * u_tau * math.pi / period


def amplitudes(seed: int, n_modes: int, u_tau: float, period: float, s_max: float = 0.05):
    """Trigger-force amplitudes for one pipe: 2*n_modes values, ordered
    (m=1 cos, m=1 sin, m=2 cos, ...), each s * amplitude_unit with s ~ U(0, s_max)."""
    s = uniform01(seed, 2 * n_modes) * s_max
    return s * amplitude_unit(u_tau, period)


def batch_amplitudes(seed0: int, batch: int, n_modes: int, u_tau: float, period: float):
    """[batch][2*n_modes] amplitudes, pipe b seeded with seed0 + b."""
    return np.stack([amplitudes(seed0 + b, n_modes, u_tau, period) for b in range(batch)]) \
        if n_modes > 0 else np.zeros((batch, 0))


def _pipe(nx, ny, nz, radius, nu, u_tau, *, batch=1, n_modes=6, force_off_step=None, steps=1000,
          init=1, seed=0, **extra):
    tau = 3.0 * nu + 0.5
    h = 2.0 * u_tau * u_tau / radius
    period = round(0.052 * radius / u_tau)
    cfg = dict(nx=nx, ny=ny, nz=nz, batch=batch, radius=float(radius), tau=tau, accel_z=h,
               n_modes=n_modes, kz=3.0, kappa=0.5, l0_frac=0.2, l_frac=0.4,
               period=float(period), force_off_step=int(force_off_step if force_off_step is not None
                                                         else steps),
               storage=0, wall=0, pattern=0, init=init, u_tau=u_tau, steps=steps, seed=seed)
    cfg.update(extra)
    return cfg


def preset(name: str) -> dict:
    """Named pipe configurations (plain dicts; keys are config fields plus
    ``steps`` and ``seed``)."""
    if name == "laminar":  # 24x24x48, R=10, tau=0.8, a=1e-6, rest start, halfway bounce-back
        return dict(nx=24, ny=24, nz=48, batch=1, radius=10.0, tau=0.8, accel_z=1e-6, n_modes=0,
                    kz=3.0, kappa=0.5, l0_frac=0.2, l_frac=0.4, period=1.0, force_off_step=0,
                    storage=0, wall=0, pattern=0, init=0, u_tau=0.0, steps=500, seed=0)
    if name == "turbulent":  # 192x192x1152, R=90, Re_tau ~ 181 at the paper's u*
        nu = PAPER_U_TAU * 90.0 / PAPER_RE_TAU
        return _pipe(192, 192, 1152, 90.0, nu, PAPER_U_TAU, force_off_step=5000, steps=20000)
    if name == "precision_ref":  # 64x64x256, R=30, the turbulent pipe's tau and u*
        nu = PAPER_U_TAU * 90.0 / PAPER_RE_TAU
        return _pipe(64, 64, 256, 30.0, nu, PAPER_U_TAU, force_off_step=2500, steps=5000)
    if name == "batched":  # 64 pipes of 64x64x256, R=30, nu = 0.0032
        return _pipe(64, 64, 256, 30.0, PAPER_NU, PAPER_U_TAU, batch=64, force_off_step=5000,
                     steps=5000)
    if name == "paper":  # the paper's pipe (Section II.B): 300x300x600, R = 149.5, Bouzidi wall,
        # one trigger mode k_theta = 2 (cos) of amplitude h A_0 for the first 3 T^LET, 30 T^LET in all
        t_let = round(PAPER_RADIUS / PAPER_U_TAU)
        return _pipe(*PAPER_GRID, PAPER_RADIUS, PAPER_NU, PAPER_U_TAU, n_modes=PAPER_K_THETA,
                     force_off_step=3 * t_let, steps=30 * t_let, wall=1, paper_A0=PAPER_A0)
    if name == "adjoint":  # 96x96x384, R=45, nu = 0.0032, J over steps 1501..2000
        return _pipe(96, 96, 384, 45.0, PAPER_NU, PAPER_U_TAU, force_off_step=2000, steps=2000,
                     obs_begin=1501, obs_end=2001, checkpoint_every=100)
    raise KeyError(name)


def preset_amplitudes(cfg: dict) -> np.ndarray:
    """[batch][2*n_modes] amplitudes for a preset (seed, seed+1, ...).  The
    paper's pipe has one cosine mode k_theta = n_modes of amplitude h A_0."""
    if "paper_A0" in cfg:
        a = np.zeros((int(cfg.get("batch", 1)), 2 * int(cfg["n_modes"])))
        a[:, 2 * (int(cfg["n_modes"]) - 1)] = float(cfg["paper_A0"]) * float(cfg["accel_z"])
        return a
    return batch_amplitudes(int(cfg.get("seed", 0)), int(cfg.get("batch", 1)),
                            int(cfg["n_modes"]), float(cfg["u_tau"]), float(cfg["period"]))


def random_populations(seed: int, shape, scale: float = 1e-3) -> np.ndarray:
    """Seeded random deviation field for parity tests: N(0, scale) values."""
    return np.random.default_rng(seed).normal(0.0, scale, size=shape)


def dims_of(cfg: dict):
    return int(cfg["nx"]), int(cfg["ny"]), int(cfg["nz"])
