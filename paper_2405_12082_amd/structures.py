"""Statistics of the series of dominant azimuthal modes (arXiv:2405.12082,
Section III), on the host: the series is a few thousand small integers per
run, produced on the GPU by ``Pipe.ring_spectrum`` (one dominant mode per
sampling step).

* ``transition_matrix``: T[i][j] = P(mode i + 1 after ``lag`` samples | mode
  j + 1 now), columns summing to 1 (the convention of the printed matrix);
* ``ck_test``: eigenvalue magnitudes of the transition matrices of the
  decimated series (every d-th sample) against the Markov prediction
  |lambda(T_1)|^d (the Chapman-Kolmogorov test);
* ``self_correlation``: F_m(tau) = (<V_m(t) V_m(t+tau)> - <V_m>^2) / (value at
  tau = 0) with V_m(t) = [mode at t == m], per mode and averaged over the
  modes that occur;
* ``streamwise_lengths``: Taylor's frozen hypothesis, length = persistence
  time of a mode x convection velocity, mean and largest per mode.
"""
from __future__ import annotations

import numpy as np


def _as_modes(modes) -> np.ndarray:
    return np.asarray(modes, dtype=np.int64).ravel()


def transition_matrix(modes, n_modes: int, lag: int = 1) -> np.ndarray:
    m = _as_modes(modes)
    if m.size and (m.min() < 1 or m.max() > n_modes):
        raise ValueError("modes must lie in 1..n_modes")
    counts = np.zeros((n_modes, n_modes))
    np.add.at(counts, (m[lag:] - 1, m[:-lag] - 1), 1.0)
    col = counts.sum(axis=0)
    return np.divide(counts, col, out=np.zeros_like(counts), where=col > 0)


def ck_test(modes, n_modes: int, orders=(1, 2, 3, 4, 5)):
    """[(order, |lambda(T_order)| sorted, |lambda(T_1)|^order sorted)]."""
    m = _as_modes(modes)
    lam1 = np.sort(np.abs(np.linalg.eigvals(transition_matrix(m, n_modes))))[::-1]
    out = []
    for d in orders:
        lam = np.sort(np.abs(np.linalg.eigvals(transition_matrix(m[::d], n_modes))))[::-1]
        out.append((d, lam, lam1 ** d))
    return out


def self_correlation(modes, n_modes: int, max_lag: int):
    """(F [n_modes][max_lag+1], mode average [max_lag+1])."""
    m = _as_modes(modes)
    n = m.size
    v = (m[None, :] == np.arange(1, n_modes + 1)[:, None]).astype(np.float64)
    mean = v.mean(axis=1)
    f = np.empty((n_modes, max_lag + 1))
    for tau in range(max_lag + 1):
        f[:, tau] = (v[:, :n - tau] * v[:, tau:]).mean(axis=1) - mean * mean
    occ = f[:, 0] > 0
    fn = np.zeros_like(f)
    fn[occ] = f[occ] / f[occ, :1]
    if not occ.any():  # no mode comes and goes (a constant series): undefined
        return fn, np.full(max_lag + 1, np.nan)
    return fn, fn[occ].mean(axis=0)


def streamwise_lengths(modes, n_modes: int, dt_steps: float, u_conv: float):
    """Per mode: (mean, largest) streamwise length, in lattice units, of its
    runs of consecutive samples: run length x dt_steps x u_conv."""
    m = _as_modes(modes)
    edges = np.flatnonzero(np.diff(m)) + 1
    starts = np.concatenate(([0], edges))
    lengths = np.diff(np.concatenate((starts, [m.size])))
    out = {}
    for k in range(1, n_modes + 1):
        runs = lengths[m[starts] == k] * dt_steps * u_conv
        out[k] = (float(runs.mean()), float(runs.max())) if runs.size else (0.0, 0.0)
    return out
