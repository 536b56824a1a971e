"""Pins of the oracle's coherent-structure identification (Section II.C):
bilinear ring sampling, the azimuthal correlation R_uu, its Fourier
transform and the dominant mode, against closed forms and an FFT library
routine (CPU only)."""
import numpy as np
import pytest

from oracle import structures as S


def test_ring_sampling_is_exact_for_linear_fields():
    """Bilinear interpolation reproduces a + b x + c y at every ring point."""
    nz, ny, nx = 3, 40, 36
    zz, yy, xx = np.mgrid[0:nz, 0:ny, 0:nx]
    uz = 0.1 + 0.02 * xx - 0.03 * yy + 0.5 * zz
    r0, n = 13.7, 64
    ring = S.ring_sample(uz.astype(float), r0, n)
    th = 2 * np.pi * np.arange(n) / n
    px, py = 17.5 + r0 * np.cos(th), 19.5 + r0 * np.sin(th)
    for z in range(nz):
        np.testing.assert_allclose(ring[z], 0.1 + 0.02 * px - 0.03 * py + 0.5 * z, rtol=0, atol=1e-12)


def test_correlation_of_a_single_mode_is_its_cosine():
    n, m = 96, 4
    th = 2 * np.pi * np.arange(n) / n
    r = S.correlation(0.7 + 0.2 * np.cos(m * th + 0.3))
    np.testing.assert_allclose(r, np.cos(m * th), atol=1e-12)


def test_spectrum_of_two_modes_in_closed_form():
    """du = A cos(3 theta) + B cos(5 theta + phi): S(3) = N A^2 / (2 (A^2+B^2)),
    S(5) = N B^2 / (2 (A^2+B^2)), zero elsewhere; the dominant mode is 3."""
    n, A, B = 128, 0.3, 0.2
    th = 2 * np.pi * np.arange(n) / n
    ring = np.stack([1.0 + A * np.cos(3 * th) + B * np.cos(5 * th + 1.1),
                     2.0 + A * np.cos(3 * th + 0.4) + B * np.cos(5 * th - 0.2)])
    s = S.correlation_spectrum(ring, 12)
    expect = np.zeros(13)
    expect[3] = n * A * A / (2 * (A * A + B * B))
    expect[5] = n * B * B / (2 * (A * A + B * B))
    np.testing.assert_allclose(s, expect, atol=1e-10)
    assert S.dominant_mode(s) == 3


def test_spectrum_is_the_power_spectrum_of_the_fluctuation():
    """Wiener-Khinchin: the transform of R_uu equals |FFT(du)|^2 / sum du^2
    per plane (numpy's FFT as the independent path)."""
    rng = np.random.default_rng(3)
    ring = rng.normal(size=(4, 60))
    s = S.correlation_spectrum(ring, 29)
    ref = np.zeros(30)
    for z in range(4):
        du = ring[z] - ring[z].mean()
        ref += np.abs(np.fft.fft(du)[:30]) ** 2 / np.sum(du * du)
    np.testing.assert_allclose(s, ref / 4, rtol=1e-10, atol=1e-12)


def test_transition_matrix_counts():
    """Columns are the current mode, rows the next one (the convention of
    the printed matrix, whose columns sum to 1)."""
    t = S.transition_matrix([1, 2, 1, 2, 1, 1, 3], 1, 3)
    np.testing.assert_allclose(t, np.array([[1 / 4, 2 / 4, 1 / 4], [1, 0, 0], [0, 0, 0]]).T)
    t2 = S.transition_matrix([1, 2, 1, 2, 1, 1, 3], 2, 3)
    np.testing.assert_allclose(t2, np.array([[2 / 3, 0, 1 / 3], [0.5, 0.5, 0], [0, 0, 0]]).T)
    with pytest.raises(IndexError):
        S.transition_matrix([1, 4], 1, 3)


def test_transition_matrix_of_a_markov_chain_and_the_ck_prediction():
    """A simulated 3-state Markov chain with a known column-stochastic T:
    the estimate is within sampling error, and the decimated series obey
    the Chapman-Kolmogorov relation |lambda(T_d)| = |lambda(T_1)|^d."""
    T = np.array([[0.90, 0.05, 0.10], [0.06, 0.90, 0.05], [0.04, 0.05, 0.85]])
    rng = np.random.default_rng(11)
    s, modes = 0, []
    for _ in range(200000):
        modes.append(s + 1)
        s = rng.choice(3, p=T[:, s])
    est = S.transition_matrix(modes, 1, 3)
    np.testing.assert_allclose(est, T, atol=0.01)
    for lam, pred in S.ck_eigenvalues(modes, 3, (1, 2, 4)):
        np.testing.assert_allclose(lam, pred, atol=0.02)
    lam_true = np.sort(np.abs(np.linalg.eigvals(T)))[::-1]
    np.testing.assert_allclose(S.ck_eigenvalues(modes, 3, (1,))[0][0], lam_true, atol=0.01)


def test_self_correlation_closed_forms():
    """Blocks of L equal modes cycling through all n modes: V_m is a periodic
    indicator of period n L, whose normalised autocovariance at lag tau <= L
    is ((L - tau)/(n L) - 1/n^2) / (1/n - 1/n^2) (exact for the full cycle
    when the averages run over whole periods: checked on a long series)."""
    n, L = 4, 10
    modes = [1 + (t // L) % n for t in range(n * L * 400)]
    f, mean = S.self_correlation(modes, n, L)
    tau = np.arange(L + 1)
    expect = ((L - tau) / (n * L) - 1 / n ** 2) / (1 / n - 1 / n ** 2)
    for m in range(n):
        np.testing.assert_allclose(f[m], expect, atol=2e-3)
    np.testing.assert_allclose(mean, expect, atol=2e-3)


def test_run_lengths():
    runs = S.run_lengths([2, 2, 1, 3, 3, 3, 2], 3)
    assert runs == {1: [1], 2: [2, 1], 3: [3]}
    assert S.decimate([1, 2, 3, 4, 5, 6, 7], 3) == [1, 4, 7]


def test_printed_transition_matrix_is_column_stochastic():
    """The convention of transition_matrix: the printed matrix's columns sum
    to 1 within its three-decimal rounding, its rows do not."""
    import json
    import os
    t = np.array(json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                             "transition_matrix_printed.json")))["T"])
    assert np.abs(t.sum(axis=0) - 1).max() <= 0.006
    assert np.abs(t.sum(axis=1) - 1).max() > 0.05
