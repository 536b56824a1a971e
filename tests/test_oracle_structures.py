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
    t = S.transition_matrix([1, 2, 1, 2, 1, 1, 3], 1, 3)
    np.testing.assert_allclose(t, [[1 / 4, 2 / 4, 1 / 4], [1, 0, 0], [0, 0, 0]])
    t2 = S.transition_matrix([1, 2, 1, 2, 1, 1, 3], 2, 3)
    np.testing.assert_allclose(t2, [[2 / 3, 0, 1 / 3], [0.5, 0.5, 0], [0, 0, 0]])
    with pytest.raises(IndexError):
        S.transition_matrix([1, 4], 1, 3)
