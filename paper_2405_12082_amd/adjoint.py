"""Gradient of the time-averaged streamwise kinetic energy with respect to
the trigger-force amplitudes, by the library's discrete adjoint.

Objective (time-averaged streamwise kinetic energy over a window of steps):
    J(amps) = 1/W sum_{n=obs_begin}^{obs_end-1} (1/N_f) sum_x 1/2 rho u_z^2 (x, n)
with the pipe started from its configured initial state and stepped
obs_end - 1 times; the amplitudes enter through the trigger force of
Eq. (TurbForce).

Memory: forward saves a checkpoint every ``checkpoint_every`` steps; the
reverse sweep restores one checkpoint at a time, recomputes its segment into
a ring of records (the moments rho - 1 and j of each state, 16 B per node in
FP32, or whole saved states) and runs the adjoint steps over it (checkpoint
and recompute), so device memory is N/C states plus C records instead of N
states.  With ``recompute=False`` the forward run records the moments of
every state itself (N + 1 records, 78 GB for 2000 steps of a 96x96x384
pipe) and the reverse sweep reads them without recomputing.
"""
from __future__ import annotations

import numpy as np
import torch

from .pipe import Pipe


class EnergyAdjoint:
    """Forward runs and adjoint sweeps of J for one pipe configuration.

    cfg:   configuration dict (``lbm_config`` fields).
    obs_begin, obs_end: the window [obs_begin, obs_end) of J.
    precision: the adjoint state's storage, "fp32" (default) or "fp64"; the
    vector-Jacobian arithmetic and the gradient accumulation are FP64 in
    both; the forward model is the configured stepper (FP64 forward storage
    requires "fp64").
    library: the loaded library to run (default: the release build).
    records: what the recompute keeps of each forward state for the reverse
    steps: "moments" (default: rho - 1 and j, 16 B per node, the collision's
    Jacobian needs no more) or "states" (the whole saved state, 108 B).
    recompute: False keeps the moment records of the whole forward run in
    device memory instead of checkpoints (moment records only).
    """

    def __init__(self, cfg: dict, obs_begin: int, obs_end: int, checkpoint_every: int = 100,
                 device="cuda", stream=None, precision: str = "fp32", library=None, records: str = "moments",
                 recompute: bool = True):
        if not (0 <= obs_begin < obs_end):
            raise ValueError("need 0 <= obs_begin < obs_end")
        if precision not in ("fp32", "fp64"):
            raise ValueError("precision must be 'fp32' or 'fp64'")
        if records not in ("moments", "states"):
            raise ValueError("records must be 'moments' or 'states'")
        if not recompute and records != "moments":
            raise ValueError("recompute=False keeps moment records")
        self.records = records
        self.recompute = bool(recompute)
        self.all_records = None  # recompute=False: the forward run's records
        self.scratch = None
        self.cfg = dict(cfg, adjoint=2 if precision == "fp64" else 1)
        self.obs_begin, self.obs_end = int(obs_begin), int(obs_end)
        self.C = int(checkpoint_every)
        self.device = torch.device(device)
        self.stream = stream
        self.pipe = None
        self.ckpt = None
        self.ring = None
        self.timing = {}
        self.runs = 0  # forward runs so far: the checkpoints belong to the last one
        self.library = library

    @property
    def last_step(self) -> int:
        return self.obs_end - 1

    def _new_pipe(self, amps):
        if self.pipe is not None:
            self.pipe.close()
        self.pipe = Pipe(self.cfg, amps, device=self.device, stream=self.stream, library=self.library)
        return self.pipe

    def objective(self, amps, keep_checkpoints: bool = False) -> np.ndarray:
        """Run the forward model and return J per pipe ([batch] FP64)."""
        p = self._new_pipe(amps)
        N = self.last_step
        if keep_checkpoints and not self.recompute:
            return self._objective_recording(p, N)
        if keep_checkpoints:
            nck = N // self.C + 1
            if self.ckpt is None or self.ckpt.shape != (nck, p.state_bytes):
                self.ckpt = torch.empty((nck, p.state_bytes), dtype=torch.uint8, device=self.device)
        acc = torch.zeros(p.cfg.batch, dtype=torch.float64, device=self.device)
        for n in range(N + 1):
            if keep_checkpoints and n % self.C == 0:
                p.save(self.ckpt[n // self.C])
            if self.obs_begin <= n:
                p.energy_accumulate(acc)
            if n < N:
                p.step(1)
        return acc.cpu().numpy() / (self.obs_end - self.obs_begin)

    def _objective_recording(self, p, N) -> np.ndarray:
        """The forward run recording the moments of states 0..N (the last by
        one more step, whose state is not used)."""
        if self.all_records is None or self.all_records.shape != (N + 1, p.record_bytes):
            self.all_records = None
            self.all_records = torch.empty((N + 1, p.record_bytes), dtype=torch.uint8, device=self.device)
        acc = torch.zeros(p.cfg.batch, dtype=torch.float64, device=self.device)
        n = 0
        while n <= N:
            if self.obs_begin <= n:
                p.energy_accumulate(acc)
                k = 1
            else:
                k = self.obs_begin - n  # up to the window in one call
            p.step_recording(self.all_records[n:n + k])
            n += k
        self.ckpt = self.all_records  # marks a recorded run for backward
        return acc.cpu().numpy() / (self.obs_end - self.obs_begin)

    def forward(self, amps) -> np.ndarray:
        """Forward run keeping checkpoints for :meth:`backward`; returns J."""
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        J = self.objective(amps, keep_checkpoints=True)
        self.runs += 1
        e1.record()
        torch.cuda.synchronize()
        self.timing = {"forward_ms": e0.elapsed_time(e1), "steps": self.last_step}
        return J

    def backward(self) -> np.ndarray:
        """Reverse sweep over the last forward run: dJ/d amps [batch][2*n_modes]."""
        p = self.pipe
        if p is None or self.ckpt is None:
            raise RuntimeError("backward() needs a forward() run first")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        B, nq = p.cfg.batch, 2 * p.cfg.n_modes
        grad = torch.zeros((B, max(nq, 1)), dtype=torch.float64, device=self.device)
        N = self.last_step
        if not self.recompute:
            p.adjoint_reset(self.obs_begin, self.obs_end)
            p.adjoint_step_moments(self.all_records[:N + 1], grad, N + 1)
            e1.record()
            torch.cuda.synchronize()
            self.timing["backward_ms"] = e0.elapsed_time(e1)
            return grad[:, :nq].cpu().numpy()
        moments = self.records == "moments"
        rec = p.record_bytes if moments else p.state_bytes
        if self.ring is None or self.ring.shape != (self.C, rec):
            self.ring = torch.empty((self.C, rec), dtype=torch.uint8, device=self.device)
        if moments and (self.scratch is None or self.scratch.shape != (2, p.state_bytes)):
            self.scratch = torch.empty((2, p.state_bytes), dtype=torch.uint8, device=self.device)
        p.adjoint_reset(self.obs_begin, self.obs_end)
        cursor = N
        while cursor >= 0:
            k = cursor // self.C
            start = k * self.C
            count = cursor - start + 1
            if moments:  # the segment's moment records
                p.recompute_moments(self.ckpt[k], start, self.scratch, self.ring, count)
                p.adjoint_step_moments(self.ring[:count], grad, count)
            else:  # the segment's states
                p.recompute(self.ckpt[k], start, self.ring, count)
                p.adjoint_step(self.ring[:count], grad, count)
            cursor = start - 1
        e1.record()
        torch.cuda.synchronize()
        self.timing["backward_ms"] = e0.elapsed_time(e1)
        return grad[:, :nq].cpu().numpy()

    def gradient(self, amps):
        """J and dJ/d amps ([batch], [batch][2*n_modes])."""
        J = self.forward(amps)
        return J, self.backward()


class PipeEnergy(torch.autograd.Function):
    """J(amps) as an autograd node: forward runs the pipe (keeping
    checkpoints), backward runs the checkpointed discrete adjoint.
    ``amps``: [batch][2*n_modes] float64 tensor; returns J [batch]."""

    @staticmethod
    def forward(ctx, amps: torch.Tensor, runner: EnergyAdjoint):
        J = runner.forward(amps.detach().cpu().numpy().astype(np.float64))
        ctx.runner = runner
        ctx.run = runner.runs
        ctx.meta = (amps.dtype, amps.device)
        return torch.as_tensor(J, dtype=amps.dtype, device=amps.device)

    @staticmethod
    def backward(ctx, gJ):
        dtype, device = ctx.meta
        if ctx.runner.runs != ctx.run:
            raise RuntimeError("PipeEnergy: the runner ran another forward pass after this node; its checkpoints "
                               "belong to that run (use one EnergyAdjoint per node)")
        g = torch.as_tensor(ctx.runner.backward(), dtype=dtype, device=device)
        return gJ.reshape(-1, 1) * g, None
