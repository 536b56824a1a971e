"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It loads ``oracle/liblbm_oracle.so`` (built by ``oracle/build.py``)
and exposes the per-node formulas of the paper's appendix and a pipe stepper.

Array layouts returned here: populations [27][nz][ny][nx], scalars
[nz][ny][nx], vectors [3][nz][ny][nx].
"""
import ctypes as C
import os
from dataclasses import dataclass, fields

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liblbm_oracle.so")


class OrcConfig(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("radius", C.c_double), ("tau", C.c_double), ("accel_z", C.c_double),
        ("n_modes", C.c_int32),
        ("kz", C.c_double), ("kappa", C.c_double), ("l0_frac", C.c_double),
        ("l_frac", C.c_double), ("period", C.c_double),
        ("force_off_step", C.c_int64),
        ("wall", C.c_int32), ("init", C.c_int32), ("u_tau", C.c_double),
        ("collision", C.c_int32), ("equilibrium", C.c_int32),
    ]


def make_config(**kw) -> OrcConfig:
    """Oracle configuration from keyword values (unknown keys are ignored)."""
    defaults = dict(nx=24, ny=24, nz=48, radius=10.0, tau=0.8, accel_z=0.0, n_modes=0,
                    kz=3.0, kappa=0.5, l0_frac=0.2, l_frac=0.4, period=1.0,
                    force_off_step=0, wall=0, init=0, u_tau=0.0, collision=0, equilibrium=0)
    names = [f[0] for f in OrcConfig._fields_]
    vals = {k: kw.get(k, defaults[k]) for k in names}
    return OrcConfig(**vals)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"oracle library not built: {_LIB_PATH} (run oracle/build.py)")
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        u8p = C.POINTER(C.c_uint8)
        cfgp = C.POINTER(OrcConfig)
        L.orc_lattice.argtypes = [ip, dp, ip]
        L.orc_moment_matrix.argtypes = [dp]
        L.orc_moment_matrix_inverse.argtypes = [dp]
        L.orc_feq.argtypes = [C.c_double, dp, dp]
        L.orc_meq.argtypes = [C.c_double, dp, dp]
        L.orc_rmrt.argtypes = [C.c_double, dp, dp, dp]
        L.orc_collide.argtypes = [dp, dp, C.c_double, dp]
        L.orc_feq2.argtypes = [C.c_double, dp, dp]
        L.orc_force2.argtypes = [C.c_double, dp, dp, dp]
        L.orc_collide_kind.argtypes = [dp, dp, C.c_double, C.c_int32, C.c_int32, dp]
        L.orc_feq_cplx.argtypes = [dp, dp, dp]
        L.orc_meq_cplx.argtypes = [dp, dp, dp]
        L.orc_collide_cplx.argtypes = [dp, dp, C.c_double, dp]
        L.orc_bouzidi.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32]
        L.orc_bouzidi.restype = C.c_double
        L.orc_wall_fraction.argtypes = [cfgp, C.c_int32, C.c_int32, C.c_int32]
        L.orc_wall_fraction.restype = C.c_double
        L.orc_trigger_shape.argtypes = [cfgp, dp, C.c_double, C.c_double, C.c_double, dp]
        L.orc_force_at.argtypes = [cfgp, dp, C.c_int32, C.c_int32, C.c_int32, C.c_int64, dp]
        L.orc_pipe_new.argtypes = [cfgp, dp]
        L.orc_pipe_new.restype = C.c_void_p
        L.orc_pipe_free.argtypes = [C.c_void_p]
        L.orc_pipe_step_index.argtypes = [C.c_void_p]
        L.orc_pipe_step_index.restype = C.c_int64
        L.orc_pipe_fluid_count.argtypes = [C.c_void_p]
        L.orc_pipe_fluid_count.restype = C.c_int64
        L.orc_pipe_fluid_mask.argtypes = [C.c_void_p, u8p]
        L.orc_pipe_step.argtypes = [C.c_void_p, C.c_int32]
        L.orc_pipe_get_f.argtypes = [C.c_void_p, dp]
        L.orc_pipe_stream.argtypes = [C.c_void_p]
        L.orc_pipe_set_f.argtypes = [C.c_void_p, dp, C.c_int64]
        L.orc_pipe_force.argtypes = [C.c_void_p, C.c_int64, dp]
        L.orc_pipe_moments.argtypes = [C.c_void_p, dp, dp]
        L.orc_pipe_sums.argtypes = [C.c_void_p, dp]
        L.orc_pipe_energy.argtypes = [C.c_void_p]
        L.orc_pipe_energy.restype = C.c_double
        L.orc_num_threads.restype = C.c_int32
        for fn in (L.orc_adjoint_gradient, L.orc_tangent_gradient):
            fn.argtypes = [cfgp, dp, C.c_int64, C.c_int64, dp]
            fn.restype = C.c_double
        L.orc_objective.argtypes = [cfgp, dp, C.c_int64, C.c_int64]
        L.orc_objective.restype = C.c_double
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- per node
def lattice():
    c = np.zeros((27, 3), np.int32)
    w = np.zeros(27)
    opp = np.zeros(27, np.int32)
    lib().orc_lattice(c.ctypes.data_as(C.POINTER(C.c_int32)), _p(w),
                      opp.ctypes.data_as(C.POINTER(C.c_int32)))
    return c, w, opp


def moment_matrix():
    A = np.zeros((27, 27))
    lib().orc_moment_matrix(_p(A))
    return A


def moment_matrix_inverse():
    A = np.zeros((27, 27))
    lib().orc_moment_matrix_inverse(_p(A))
    return A


def feq(rho, u):
    u = _f64(u)
    out = np.zeros(27)
    lib().orc_feq(float(rho), _p(u), _p(out))
    return out


def meq(rho, u):
    u = _f64(u)
    out = np.zeros(27)
    lib().orc_meq(float(rho), _p(u), _p(out))
    return out


def rmrt(rho, u, F):
    u, F = _f64(u), _f64(F)
    out = np.zeros(27)
    lib().orc_rmrt(float(rho), _p(u), _p(F), _p(out))
    return out


def collide(f, a, omega):
    f, a = _f64(f), _f64(a)
    out = np.zeros(27)
    lib().orc_collide(_p(f), _p(a), float(omega), _p(out))
    return out


def feq2(rho, u):
    """Second-order equilibrium (the LBM-O(2) comparison scheme)."""
    u = _f64(u)
    out = np.zeros(27)
    lib().orc_feq2(float(rho), _p(u), _p(out))
    return out


def force2(rho, u, a):
    """Population forcing a . grad_u of the second-order equilibrium."""
    u, a = _f64(u), _f64(a)
    out = np.zeros(27)
    lib().orc_force2(float(rho), _p(u), _p(a), _p(out))
    return out


def collide_kind(f, a, omega, collision=0, equilibrium=0):
    """Collision of a given kind: collision 0 MRT / 1 SRT (BGK), equilibrium
    0 sixth-order Hermite / 1 second order.  (0, 0) equals :func:`collide`."""
    f, a = _f64(f), _f64(a)
    out = np.zeros(27)
    lib().orc_collide_kind(_p(f), _p(a), float(omega), int(collision), int(equilibrium), _p(out))
    return out


def _ri(z):
    z = np.asarray(z, dtype=np.complex128)
    return np.ascontiguousarray(np.stack([z.real, z.imag], axis=-1).reshape(-1))


def _from_ri(a):
    return a[0::2] + 1j * a[1::2]


def feq_complex(rho, u):
    out = np.zeros(54)
    r, uu = _ri([rho]), _ri(u)
    lib().orc_feq_cplx(_p(r), _p(uu), _p(out))
    return _from_ri(out)


def meq_complex(rho, u):
    out = np.zeros(54)
    r, uu = _ri([rho]), _ri(u)
    lib().orc_meq_cplx(_p(r), _p(uu), _p(out))
    return _from_ri(out)


def collide_complex(f, a, omega):
    out = np.zeros(54)
    ff, aa = _ri(f), _ri(a)
    lib().orc_collide_cplx(_p(ff), _p(aa), float(omega), _p(out))
    return _from_ri(out)


def bouzidi(delta, fs_out_x, fs_in_x, fs_out_xff, has_ff=True):
    return lib().orc_bouzidi(float(delta), float(fs_out_x), float(fs_in_x), float(fs_out_xff),
                             int(bool(has_ff)))


def wall_fraction(cfg: OrcConfig, x, y, d):
    """Delta of the link from fluid node (x, y) along direction d to r = R."""
    return lib().orc_wall_fraction(C.byref(cfg), int(x), int(y), int(d))


def trigger_shape(cfg: OrcConfig, amps, x, y, z):
    amps = _f64(np.resize(np.asarray(amps, float), 12) if len(amps) else np.zeros(12))
    out = np.zeros(3)
    lib().orc_trigger_shape(C.byref(cfg), _p(amps), float(x), float(y), float(z), _p(out))
    return out


def force_at(cfg: OrcConfig, amps, x, y, z, n):
    """Body acceleration a(x, n) at node (x, y, z) and step n."""
    a = np.zeros(12)
    k = 2 * max(cfg.n_modes, 0)
    if k:
        a[:k] = np.asarray(amps, float)[:k]
    out = np.zeros(3)
    lib().orc_force_at(C.byref(cfg), _p(a), int(x), int(y), int(z), int(n), _p(out))
    return out


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ---------------------------------------------------------------- pipe
class Pipe:
    """FP64 pipe stepper: collide then stream, state f^n at step n."""

    def __init__(self, cfg: OrcConfig, amps=None):
        self.cfg = cfg
        n = 2 * max(cfg.n_modes, 0)
        a = np.zeros(12)
        if amps is not None and n:
            a[:n] = np.asarray(amps, float)[:n]
        self._amps = a
        self._h = lib().orc_pipe_new(C.byref(cfg), _p(self._amps))
        if not self._h:
            raise MemoryError("oracle pipe allocation failed")
        self.shape = (cfg.nz, cfg.ny, cfg.nx)

    def close(self):
        if self._h:
            lib().orc_pipe_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def step_index(self) -> int:
        return int(lib().orc_pipe_step_index(self._h))

    @property
    def n_fluid(self) -> int:
        return int(lib().orc_pipe_fluid_count(self._h))

    def fluid_mask(self):
        m = np.zeros(self.shape, np.uint8)
        lib().orc_pipe_fluid_mask(self._h, m.ctypes.data_as(C.POINTER(C.c_uint8)))
        return m.astype(bool)

    def step(self, n: int = 1):
        lib().orc_pipe_step(self._h, int(n))

    def stream_only(self):
        """Apply the streaming step alone to the stored state (f <- S f)."""
        lib().orc_pipe_stream(self._h)

    def get_f(self):
        out = np.zeros((27,) + self.shape)
        lib().orc_pipe_get_f(self._h, _p(out))
        return out

    def set_f(self, f, step=None):
        f = _f64(f)
        lib().orc_pipe_set_f(self._h, _p(f), int(self.step_index if step is None else step))

    def force(self, n=None):
        out = np.zeros((3,) + self.shape)
        lib().orc_pipe_force(self._h, int(self.step_index if n is None else n), _p(out))
        return out

    def moments(self):
        rho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        lib().orc_pipe_moments(self._h, _p(rho), _p(u))
        return rho, u

    def sums(self):
        out = np.zeros(4)
        lib().orc_pipe_sums(self._h, _p(out))
        return out

    def energy(self) -> float:
        return float(lib().orc_pipe_energy(self._h))


def _amps12(cfg, amps):
    a = np.zeros(12)
    n = 2 * max(cfg.n_modes, 0)
    if amps is not None and n:
        a[:n] = np.asarray(amps, float)[:n]
    return a


def adjoint_gradient(cfg, amps, obs_begin, obs_end):
    a = _amps12(cfg, amps)
    g = np.zeros(12)
    J = lib().orc_adjoint_gradient(C.byref(cfg), _p(a), int(obs_begin), int(obs_end), _p(g))
    return J, g[:2 * cfg.n_modes]


def tangent_gradient(cfg, amps, obs_begin, obs_end):
    a = _amps12(cfg, amps)
    g = np.zeros(12)
    J = lib().orc_tangent_gradient(C.byref(cfg), _p(a), int(obs_begin), int(obs_end), _p(g))
    return J, g[:2 * cfg.n_modes]


def objective(cfg, amps, obs_begin, obs_end):
    a = _amps12(cfg, amps)
    return float(lib().orc_objective(C.byref(cfg), _p(a), int(obs_begin), int(obs_end)))
