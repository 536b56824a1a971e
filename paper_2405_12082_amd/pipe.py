"""Python front end of the HIP pipe stepper (thin wrapper over include/lbm.h).

PyTorch provides device memory (the workspace and output tensors) and the
stream; every computation runs in the library's kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import LbmError, make_config


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


class Pipe:
    """One context of the library: ``batch`` pipes of one geometry on one GPU.

    cfg:  dict (or keywords) with the ``lbm_config`` fields.
    amps: [batch][2*n_modes] trigger-force amplitudes (acceleration units).
    library: the loaded library to run (``_lib.lib()``, the default, or
    ``_lib.checked_lib()``).
    """

    def __init__(self, cfg: dict | None = None, amps=None, device="cuda", stream=None, library=None, **kw):
        d = dict(cfg or {})
        d.update(kw)
        self.cfg_dict = d
        self.cfg = make_config(**d)
        self.lib = library if library is not None else _lib.lib()
        self.layout = _lib.describe(self.cfg)
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the HIP pipe stepper needs a GPU device")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        B, nq = self.cfg.batch, 2 * self.cfg.n_modes
        a = np.zeros((B, max(nq, 0)), np.float64)
        if nq:
            if amps is None:
                raise ValueError("n_modes > 0 needs amplitudes")
            a[:] = np.asarray(amps, np.float64).reshape(B, nq)
        self.amps = np.ascontiguousarray(a)
        self.workspace = torch.empty(int(self.layout.workspace_bytes), dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace is not 256-byte aligned")
        self._ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.lbm_init(C.byref(self.cfg), self.amps.ctypes.data_as(C.POINTER(C.c_double)),
                                   C.c_void_p(_ptr(self.workspace)), C.c_size_t(self.workspace.numel()),
                                   C.c_void_p(self.stream.cuda_stream), C.byref(self._ctx))
        if rc != 0:
            raise LbmError(rc, "lbm_init failed")

    # ------------------------------------------------------------ plumbing
    def _check(self, rc, what):
        if rc != 0:
            msg = self.lib.lbm_last_error(self._ctx)
            raise LbmError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            self.lib.lbm_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.cfg.batch, self.cfg.nz, self.cfg.ny, self.cfg.nx)

    @property
    def n_fluid(self) -> int:
        return int(self.layout.n_fluid_nodes)

    # ------------------------------------------------------------ stepping
    def step(self, n: int = 1):
        self._check(self.lib.lbm_step(self._ctx, int(n)), "lbm_step")

    def step_recording(self, records: torch.Tensor, n: int | None = None):
        """n steps (default: one per record) recording the moments (rho - 1, j)
        of each consumed state into ``records`` ([n][record_bytes] uint8)."""
        n = records.shape[0] if n is None else n
        stride = records.stride(0) * records.element_size()
        self._check(self.lib.lbm_step_recording(self._ctx, int(n), C.c_void_p(_ptr(records)), C.c_size_t(stride)),
                    "lbm_step_recording")

    def step_graph(self, n: int, k: int = 64):
        self._check(self.lib.lbm_step_graph(self._ctx, int(n), int(k)), "lbm_step_graph")

    def set_launch(self, block: int = 0, zchunk: int = 0, xcd_remap: int = -1, pipes_per_launch: int = 0,
                   pipe_major: int = -1):
        """Change the step's launch geometry and order (0 / -1 keep the current value)."""
        self._check(self.lib.lbm_set_launch(self._ctx, int(block), int(zchunk), int(xcd_remap),
                                            int(pipes_per_launch), int(pipe_major)), "lbm_set_launch")

    def set_fused(self, steps_per_launch: int = 0, zchunk: int = 0, xcd_remap: int = -1):
        """Two steps per launch (2) or one (1) for step / step_graph; zchunk:
        output planes per workgroup of the two-step kernel; 0 / -1 keep."""
        self._check(self.lib.lbm_set_fused(self._ctx, int(steps_per_launch), int(zchunk), int(xcd_remap)),
                    "lbm_set_fused")

    def step_persistent(self, n: int):
        """n steps in one persistent cooperative launch (synchronises)."""
        self._check(self.lib.lbm_step_persistent(self._ctx, int(n)), "lbm_step_persistent")

    def step_persistent_graph(self, n: int, k: int = 50):
        """n steps as replays of a graph holding one persistent launch of k steps."""
        self._check(self.lib.lbm_step_persistent_graph(self._ctx, int(n), int(k)), "lbm_step_persistent_graph")

    def stream_copy(self, n: int = 1):
        """n copies of the state with the step's launch geometry (the access pattern without arithmetic)."""
        self._check(self.lib.lbm_stream_copy(self._ctx, int(n)), "lbm_stream_copy")

    @property
    def step_index(self) -> int:
        v = C.c_int64()
        self._check(self.lib.lbm_get_step(self._ctx, C.byref(v)), "lbm_get_step")
        return int(v.value)

    # ------------------------------------------------------------ observation
    def moments(self):
        B, nz, ny, nx = self.shape
        rho = torch.empty((B, nz, ny, nx), dtype=torch.float32, device=self.device)
        u = torch.empty((B, 3, nz, ny, nx), dtype=torch.float32, device=self.device)
        self._check(self.lib.lbm_moments(self._ctx, C.c_void_p(_ptr(rho)), C.c_void_p(_ptr(u))), "lbm_moments")
        return rho, u

    def populations(self):
        B, nz, ny, nx = self.shape
        g = torch.empty((B, 27, nz, ny, nx), dtype=torch.float32, device=self.device)
        self._check(self.lib.lbm_populations(self._ctx, C.c_void_p(_ptr(g))), "lbm_populations")
        return g

    def set_populations(self, g: torch.Tensor, step: int = 0):
        g = g.to(device=self.device, dtype=torch.float32).contiguous()
        if tuple(g.shape) != (self.cfg.batch, 27) + self.shape[1:]:
            raise ValueError(f"populations must have shape {(self.cfg.batch, 27) + self.shape[1:]}")
        self._keep = g  # alive until the stream has consumed it
        self._check(self.lib.lbm_set_populations(self._ctx, C.c_void_p(_ptr(g)), int(step)), "lbm_set_populations")

    def diagnostics(self, raise_on_nan: bool = False) -> np.ndarray:
        out = np.zeros((self.cfg.batch, 5))
        rc = self.lib.lbm_diagnostics(self._ctx, out.ctypes.data_as(C.POINTER(C.c_double)))
        if rc == _lib.LBM_ENAN and not raise_on_nan:
            return out
        self._check(rc, "lbm_diagnostics")
        return out

    def set_watchdog(self, mass_rel_tol: float):
        """Make diagnostics() fail (LBM_ENAN) when a pipe's mass drifts from its
        reference (the next diagnostics call) by more than mass_rel_tol; 0: off."""
        self._check(self.lib.lbm_set_watchdog(self._ctx, float(mass_rel_tol)), "lbm_set_watchdog")

    def check_flags(self) -> tuple[int, bool]:
        """Bounds-check violations recorded by a checked build since init
        (see ``lbm_check_flags``), and whether this library is one."""
        flags, checked = C.c_uint32(), C.c_int32()
        self._check(self.lib.lbm_check_flags(self._ctx, C.byref(flags), C.byref(checked)), "lbm_check_flags")
        return int(flags.value), bool(checked.value)

    def energy(self) -> np.ndarray:
        out = np.zeros(self.cfg.batch)
        self._check(self.lib.lbm_energy(self._ctx, out.ctypes.data_as(C.POINTER(C.c_double))), "lbm_energy")
        return out

    def energy_accumulate(self, acc: torch.Tensor):
        """acc[b] += E_b of the current state (device FP64 tensor [batch]), no sync."""
        self._check(self.lib.lbm_energy_accumulate(self._ctx, C.c_void_p(_ptr(acc))), "lbm_energy_accumulate")

    def recompute(self, start: torch.Tensor, s0: int, ring: torch.Tensor, n: int | None = None):
        """ring[0] := start (state of step s0), ring[j+1] := step(ring[j]); the
        context's own state is untouched."""
        n = ring.shape[0] if n is None else n
        stride = ring.stride(0) * ring.element_size()
        self._check(self.lib.lbm_recompute(self._ctx, C.c_void_p(_ptr(start)), int(s0), int(n),
                                           C.c_void_p(_ptr(ring)), C.c_size_t(stride)), "lbm_recompute")

    def recompute_moments(self, start: torch.Tensor, s0: int, scratch: torch.Tensor, records: torch.Tensor,
                          n: int | None = None):
        """scratch[0] := start (state of step s0), then n steps alternating
        between the two scratch states, recording the moments (rho - 1, j) of
        each consumed state into records[j]; the context's own state is
        untouched."""
        n = records.shape[0] if n is None else n
        stride = scratch.stride(0) * scratch.element_size()
        rstride = records.stride(0) * records.element_size()
        self._check(self.lib.lbm_recompute_moments(self._ctx, C.c_void_p(_ptr(start)), int(s0), int(n),
                                                   C.c_void_p(_ptr(scratch)), C.c_size_t(stride),
                                                   C.c_void_p(_ptr(records)), C.c_size_t(rstride)),
                    "lbm_recompute_moments")

    def profile_accumulate(self):
        self._check(self.lib.lbm_profile_accumulate(self._ctx), "lbm_profile_accumulate")

    def profile_reset(self):
        self._check(self.lib.lbm_profile_reset(self._ctx), "lbm_profile_reset")

    def profile_read(self) -> np.ndarray:
        out = np.zeros((self.cfg.batch, self.cfg.ny, self.cfg.nx, 5))
        self._check(self.lib.lbm_profile_read(self._ctx, out.ctypes.data_as(C.POINTER(C.c_double))),
                    "lbm_profile_read")
        return out

    # ------------------------------------------------------------ coherent structures
    def ring_sample(self, r0: float, ntheta: int = 1024, out: torch.Tensor | None = None) -> torch.Tensor:
        """u_z on the circle r = r0 at ntheta angles, every plane of every pipe:
        float32 [batch][nz][ntheta] on the device."""
        if out is None:
            out = torch.empty((self.cfg.batch, self.cfg.nz, int(ntheta)), dtype=torch.float32, device=self.device)
        self._check(self.lib.lbm_ring_sample(self._ctx, float(r0), int(ntheta), C.c_void_p(_ptr(out))),
                    "lbm_ring_sample")
        return out

    def ring_spectrum(self, ring: torch.Tensor, mmax: int = 64):
        """Transform of the azimuthal correlation per plane ([batch][nz][mmax+1]),
        its plane average ([batch][mmax+1]) and the dominant mode ([batch])."""
        B, nz, n = ring.shape
        spec = torch.empty((B, nz, mmax + 1), dtype=torch.float64, device=self.device)
        mean = torch.empty((B, mmax + 1), dtype=torch.float64, device=self.device)
        dom = torch.empty((B,), dtype=torch.int32, device=self.device)
        self._check(self.lib.lbm_ring_spectrum(self._ctx, C.c_void_p(_ptr(ring)), int(n), int(mmax),
                                               C.c_void_p(_ptr(spec)), C.c_void_p(_ptr(mean)),
                                               C.c_void_p(_ptr(dom))), "lbm_ring_spectrum")
        return spec, mean, dom

    # ------------------------------------------------------------ checkpoints
    @property
    def state_bytes(self) -> int:
        v = C.c_size_t()
        self._check(self.lib.lbm_state_bytes(self._ctx, C.byref(v)), "lbm_state_bytes")
        return int(v.value)

    @property
    def record_bytes(self) -> int:
        """Bytes of one moment record of :meth:`recompute_moments`."""
        return int(self.layout.record_bytes)

    def save(self, out: torch.Tensor | None = None) -> tuple[torch.Tensor, int]:
        if out is None:
            out = torch.empty(self.state_bytes, dtype=torch.uint8, device=self.device)
        step = C.c_int64()
        self._check(self.lib.lbm_save(self._ctx, C.c_void_p(_ptr(out)), C.byref(step)), "lbm_save")
        return out, int(step.value)

    def load(self, blob: torch.Tensor, step: int):
        self._check(self.lib.lbm_load(self._ctx, C.c_void_p(_ptr(blob)), int(step)), "lbm_load")

    # ------------------------------------------------------------ adjoint
    def adjoint_reset(self, obs_begin: int, obs_end: int):
        self._check(self.lib.lbm_adjoint_reset(self._ctx, int(obs_begin), int(obs_end)), "lbm_adjoint_reset")

    def adjoint_step(self, states: torch.Tensor, grad: torch.Tensor, n: int | None = None):
        """Consume ``states`` ([n][state_bytes] uint8, forward order) last to first."""
        n = states.shape[0] if n is None else n
        stride = states.stride(0) * states.element_size()
        self._check(self.lib.lbm_adjoint_step(self._ctx, int(n), C.c_void_p(_ptr(states)), C.c_size_t(stride),
                                              C.c_void_p(_ptr(grad))), "lbm_adjoint_step")

    def adjoint_step_moments(self, records: torch.Tensor, grad: torch.Tensor, n: int | None = None):
        """Consume moment ``records`` ([n][record_bytes] uint8, forward order,
        from :meth:`recompute_moments`) last to first."""
        n = records.shape[0] if n is None else n
        stride = records.stride(0) * records.element_size()
        self._check(self.lib.lbm_adjoint_step_moments(self._ctx, int(n), C.c_void_p(_ptr(records)),
                                                      C.c_size_t(stride), C.c_void_p(_ptr(grad))),
                    "lbm_adjoint_step_moments")


def radial_profiles(acc: np.ndarray, cfg: dict, bin_width: float = 1.0):
    """Mean, rms, skewness and flatness of u_z per radial bin (Eq. (urmsformula),
    pooled over time, azimuth and z) from the FP64 per-column power sums
    returned by :meth:`Pipe.profile_read` for one pipe ([ny][nx][5])."""
    ny, nx = acc.shape[:2]
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = np.hypot(xx - 0.5 * (nx - 1), yy - 0.5 * (ny - 1))
    nb = int(np.ceil(cfg["radius"] / bin_width))
    idx = np.minimum((r / bin_width).astype(int), nb - 1)
    S = np.zeros((nb, 5))
    for q in range(5):
        S[:, q] = np.bincount(idx.ravel(), weights=acc[..., q].ravel(), minlength=nb)[:nb]
    n = np.maximum(S[:, 4], 1.0)
    m1, m2, m3, m4 = (S[:, q] / n for q in range(4))
    var = np.maximum(m2 - m1 ** 2, 0.0)
    c3 = m3 - 3 * m1 * m2 + 2 * m1 ** 3
    c4 = m4 - 4 * m1 * m3 + 6 * m1 ** 2 * m2 - 3 * m1 ** 4
    rms = np.sqrt(var)
    with np.errstate(invalid="ignore", divide="ignore"):
        skew = np.where(var > 0, c3 / var ** 1.5, 0.0)
        flat = np.where(var > 0, c4 / var ** 2, 0.0)
    rc = (np.arange(nb) + 0.5) * bin_width
    return dict(r=rc, count=S[:, 4], mean=m1, rms=rms, skewness=skew, flatness=flat)
