"""Plain reference of the coherent-structure identification (test
infrastructure only, like the rest of ``oracle/``).

Section II.C: the streamwise velocity-velocity correlation on the circle
r = r0 (r0 = 0.78 R),
    R_uu(r0, dtheta) = < u_z(r0, theta0) u_z(r0, theta0 + dtheta) >_theta0 / u_rms^2,
with u_z the fluctuation, and the azimuthally dominant mode is the highest
peak of the power of its Fourier transform.  Readings (the paper leaves
them open): theta_j = 2 pi j / N measured as atan2(y - y_c, x - x_c); u_z at
a ring point by bilinear interpolation of the four surrounding nodes; the
fluctuation is taken about the ring mean (which only touches the m = 0
term); one correlation per z plane, averaged over the planes (the flow is
homogeneous along the pipe).  Everything is written out literally:
correlation by the sum over theta0, its transform by the DFT sum.

Section III: the series of dominant modes, its transition matrix, the
Chapman-Kolmogorov test on decimated series and the self mode correlation
function, written as loops over the series.
"""
import numpy as np


def ring_nodes(nx, ny, r0, ntheta):
    """For each of the ntheta ring points: the four surrounding nodes (x, y)
    and their bilinear weights."""
    xc, yc = 0.5 * (nx - 1), 0.5 * (ny - 1)
    out = []
    for j in range(ntheta):
        th = 2.0 * np.pi * j / ntheta
        px, py = xc + r0 * np.cos(th), yc + r0 * np.sin(th)
        x0, y0 = int(np.floor(px)), int(np.floor(py))
        fx, fy = px - x0, py - y0
        out.append([((x0, y0), (1 - fx) * (1 - fy)), ((x0 + 1, y0), fx * (1 - fy)),
                    ((x0, y0 + 1), (1 - fx) * fy), ((x0 + 1, y0 + 1), fx * fy)])
    return out


def ring_sample(uz, r0, ntheta):
    """u_z [nz][ny][nx] -> samples on the ring [nz][ntheta]."""
    nz, ny, nx = uz.shape
    nodes = ring_nodes(nx, ny, r0, ntheta)
    out = np.zeros((nz, ntheta))
    for j, quad in enumerate(nodes):
        for (x, y), w in quad:
            out[:, j] += w * uz[:, y, x]
    return out


def correlation(ring_z):
    """R_uu(dtheta_k) of one plane: (1/N) sum_j du_j du_(j+k) / u_rms^2."""
    n = len(ring_z)
    du = ring_z - ring_z.mean()
    rms2 = np.mean(du * du)
    r = np.zeros(n)
    for k in range(n):
        r[k] = np.mean(du * np.roll(du, -k)) / rms2
    return r


def correlation_spectrum(ring, mmax):
    """Fourier transform of the plane-averaged correlation, modes 0..mmax:
    S(m) = (1/nz) sum_z sum_k R_z(k) exp(-2 pi i m k / N) (real: R_z is even)."""
    nz, n = ring.shape
    k = np.arange(n)
    s = np.zeros(mmax + 1)
    for z in range(nz):
        r = correlation(ring[z])
        for m in range(mmax + 1):
            s[m] += np.real(np.sum(r * np.exp(-2j * np.pi * m * k / n)))
    return s / nz


def dominant_mode(spectrum):
    """Highest peak of the power |S(m)|^2 among m >= 1 (first one on ties)."""
    p = np.abs(spectrum[1:]) ** 2
    return int(np.argmax(p)) + 1


def transition_matrix(modes, lag, n_states):
    """T[i][j] = P(mode i at t + lag | mode j at t), columns summing to 1 as
    in the printed matrix of Section III (its columns sum to 1 within
    rounding, its rows do not), from a sequence of dominant modes
    (1..n_states); columns of modes never left stay zero."""
    t = np.zeros((n_states, n_states))
    for a, b in zip(modes[:-lag], modes[lag:]):
        t[b - 1, a - 1] += 1
    cols = t.sum(axis=0, keepdims=True)
    return np.divide(t, cols, out=np.zeros_like(t), where=cols > 0)


def decimate(modes, order):
    """The series sampled every order-th element (decimation of that order)."""
    return list(modes[::order])


def ck_eigenvalues(modes, n_states, orders):
    """Chapman-Kolmogorov test: for each decimation order d, the eigenvalue
    magnitudes of the transition matrix of the decimated series, and the
    Markov prediction |lambda(T_1)|^d, both sorted in decreasing order."""
    lam1 = np.sort(np.abs(np.linalg.eigvals(transition_matrix(modes, 1, n_states))))[::-1]
    out = []
    for d in orders:
        lam = np.sort(np.abs(np.linalg.eigvals(transition_matrix(decimate(modes, d), 1, n_states))))[::-1]
        out.append((lam, lam1 ** d))
    return out


def self_correlation(modes, n_states, max_lag):
    """F_m(tau) = (<V_m(t) V_m(t + tau)> - <V_m>^2) / (same at tau = 0), V_m(t)
    = 1 if the mode at t is m else 0, for m = 1..n_states and tau =
    0..max_lag (averages over the available pairs); and their average over
    the modes that occur."""
    v = np.array([[1.0 if k == m else 0.0 for k in modes] for m in range(1, n_states + 1)])
    f = np.zeros((n_states, max_lag + 1))
    for m in range(n_states):
        mean = v[m].mean()
        for tau in range(max_lag + 1):
            pairs = [v[m, t] * v[m, t + tau] for t in range(len(modes) - tau)]
            f[m, tau] = np.mean(pairs) - mean * mean
    occ = f[:, 0] > 0
    fn = np.zeros_like(f)
    fn[occ] = f[occ] / f[occ, :1]
    return fn, fn[occ].mean(axis=0)


def run_lengths(modes, n_states):
    """Lengths (in samples) of the runs of consecutive equal modes, per mode."""
    runs = {m: [] for m in range(1, n_states + 1)}
    start = 0
    for t in range(1, len(modes) + 1):
        if t == len(modes) or modes[t] != modes[start]:
            runs[modes[start]].append(t - start)
            start = t
    return runs
