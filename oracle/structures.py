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
    """T[i][j] = P(mode j at t + lag | mode i at t) from a sequence of
    dominant modes (1..n_states); rows without visits stay zero."""
    t = np.zeros((n_states, n_states))
    for a, b in zip(modes[:-lag], modes[lag:]):
        t[a - 1, b - 1] += 1
    rows = t.sum(axis=1, keepdims=True)
    return np.divide(t, rows, out=np.zeros_like(t), where=rows > 0)
