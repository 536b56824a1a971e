"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact
rational identities of the D3Q27 lattice, closed forms printed in the
appendix of arXiv:2405.12082 that must agree with each other, continuous
Maxwell-Boltzmann moments, conservation laws and symmetries.
"""
from fractions import Fraction
import itertools

import numpy as np
import pytest

CS2 = 1.0 / 3.0


@pytest.fixture(scope="module")
def O(oracle_mod):
    return oracle_mod


@pytest.fixture
def rng():
    """A fresh seeded generator per test: each test's random inputs are the
    same whatever ran before it (also across parallel workers)."""
    return np.random.default_rng(20240520)


# ------------------------------------------------------------------ lattice
def test_lattice_velocities_are_the_27_d3q27_vectors(O):
    """Appendix velocity set: 27 distinct vectors in {-1,0,1}^3 (the printed
    c_x row read with its missing comma restored)."""
    c, w, opp = O.lattice()
    assert c.shape == (27, 3)
    assert set(map(tuple, c)) == set(itertools.product((-1, 0, 1), repeat=3))
    assert tuple(c[0]) == (0, 0, 0)
    # ordering by shell: rest, 6 faces, 12 edges, 8 corners
    shells = (c * c).sum(1)
    assert list(shells) == [0] + [1] * 6 + [2] * 12 + [3] * 8


def test_weights_eq_omegas_and_isotropy(O):
    """Eq. (omegas): w_0 = 8/27, faces w_0/4, edges w_0/16, corners w_0/64;
    they sum to one and are isotropic to fourth order with c_s^2 = 1/3."""
    c, w, _ = O.lattice()
    shells = (c * c).sum(1)
    w0 = 8.0 / 27.0
    expect = np.select([shells == 0, shells == 1, shells == 2, shells == 3],
                       [w0, w0 / 4, w0 / 16, w0 / 64])
    np.testing.assert_allclose(w, expect, rtol=0, atol=1e-16)
    assert abs(w.sum() - 1.0) < 1e-15
    for a in range(3):
        assert abs((w * c[:, a]).sum()) < 1e-16
        for b in range(3):
            assert abs((w * c[:, a] * c[:, b]).sum() - CS2 * (a == b)) < 1e-15
    # fourth order: sum w c_x^2 c_y^2 = cs^4, sum w c_x^4 = 3 cs^4
    assert abs((w * c[:, 0] ** 2 * c[:, 1] ** 2).sum() - CS2 ** 2) < 1e-15
    assert abs((w * c[:, 0] ** 4).sum() - 3 * CS2 ** 2) < 1e-15


def test_opposite_map(O):
    c, _, opp = O.lattice()
    for i in range(27):
        assert np.all(c[opp[i]] == -c[i])
    assert sorted(opp) == list(range(27))


# ------------------------------------------------------------------ transform
def _exact_inverse(A):
    n = A.shape[0]
    M = [[Fraction(int(round(A[r, k]))) for k in range(n)] + [Fraction(int(r == k)) for k in range(n)]
         for r in range(n)]
    det = Fraction(1)
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        if piv != col:
            M[col], M[piv] = M[piv], M[col]
            det = -det
        d = M[col][col]
        det *= d
        M[col] = [v / d for v in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                fct = M[r][col]
                M[r] = [a - fct * b for a, b in zip(M[r], M[col])]
    return [[M[r][n + k] for k in range(n)] for r in range(n)], det


def test_moment_matrix_integer_invertible_and_inverse_exact(O):
    """Eq. (Mmatrix): the 27 raw moments form an invertible integer matrix
    with det = 3 * 2^32; the oracle's FP64 Gauss-Jordan inverse equals the
    exact rational inverse."""
    A = O.moment_matrix()
    assert np.all(A == np.round(A))
    Ainv_exact, det = _exact_inverse(A)
    assert det == 3 * 2 ** 32 or det == -3 * 2 ** 32
    Ai = O.moment_matrix_inverse()
    ex = np.array([[float(v) for v in row] for row in Ainv_exact])
    assert np.abs(Ai - ex).max() < 1e-15
    assert np.abs(A @ Ai - np.eye(27)).max() < 1e-14


def test_conserved_and_stress_rows(O):
    """Rows 0-3 of Eq. (Mmatrix) are mass and momentum, rows 4-8 the
    deviatoric second moments relaxed with omega in Eq. (lambda)."""
    c, _, _ = O.lattice()
    A = O.moment_matrix()
    cx, cy, cz = c[:, 0], c[:, 1], c[:, 2]
    np.testing.assert_array_equal(A[0], np.ones(27))
    np.testing.assert_array_equal(A[1:4], c.T)
    np.testing.assert_array_equal(A[4], cx * cy)
    np.testing.assert_array_equal(A[5], cx * cz)
    np.testing.assert_array_equal(A[6], cy * cz)
    np.testing.assert_array_equal(A[7], cx ** 2 - cy ** 2)
    np.testing.assert_array_equal(A[8], cx ** 2 - cz ** 2)


def test_sparse_duals_of_stress_moments(O):
    """Columns 4..8 of A^{-1} (the populations carrying one unit of a
    stress moment and nothing else) are sparse: +-1/4 on the xy/xz/yz edge
    links and 1/6, -1/3 on the face links.  Exact rational inversion gives
    the same columns."""
    c, _, _ = O.lattice()
    Ai = O.moment_matrix_inverse()
    edge = (np.abs(c).sum(1) == 2)
    face = (np.abs(c).sum(1) == 1)
    for k, (a, b) in zip((4, 5, 6), ((0, 1), (0, 2), (1, 2))):
        expect = np.where(edge & (c[:, 3 - a - b] == 0), 0.25 * c[:, a] * c[:, b], 0.0)
        np.testing.assert_allclose(Ai[:, k], expect, atol=1e-15)
    # d_7: -1/3 on the y faces, 1/6 on the x and z faces; d_8: -1/3 on the z faces
    d7 = np.where(face, np.where(c[:, 1] != 0, -1 / 3, 1 / 6), 0.0)
    d8 = np.where(face, np.where(c[:, 2] != 0, -1 / 3, 1 / 6), 0.0)
    np.testing.assert_allclose(Ai[:, 7], d7, atol=1e-15)
    np.testing.assert_allclose(Ai[:, 8], d8, atol=1e-15)


# ------------------------------------------------------------------ equilibrium
def _random_state(rng, umax=0.15):
    return 1.0 + rng.uniform(-0.05, 0.05), rng.uniform(-umax, umax, size=3)


def test_equilibrium_moments_match_printed_meq(O, rng):
    """A f^eq (Hermite-6 equilibrium, Eq. (BoltzmannEquilibriumDistribution))
    reproduces all 27 printed closed forms m_k^eq of the appendix."""
    A = O.moment_matrix()
    for _ in range(50):
        rho, u = _random_state(rng)
        np.testing.assert_allclose(A @ O.feq(rho, u), O.meq(rho, u), rtol=0, atol=2e-15)


def test_equilibrium_matches_continuous_maxwell_boltzmann_moments(O, rng):
    """Every lattice moment sum f^eq c_x^a c_y^b c_z^c with a, b, c <= 2 equals
    the Maxwell-Boltzmann moment rho prod mu_a(u), mu_0 = 1, mu_1 = u,
    mu_2 = u^2 + c_s^2 (the order the D3Q27 lattice supports)."""
    c, _, _ = O.lattice()
    for _ in range(20):
        rho, u = _random_state(rng, 0.2)
        f = O.feq(rho, u)
        for ex in itertools.product(range(3), repeat=3):
            lat = (f * np.prod([c[:, d] ** ex[d] for d in range(3)], axis=0)).sum()
            mb = rho
            for d in range(3):
                mb *= (1.0, u[d], u[d] ** 2 + CS2)[ex[d]]
            assert abs(lat - mb) < 1e-15 * 10, (ex, lat, mb)


def test_equilibrium_product_form(O, rng):
    """The sixth-order Hermite equilibrium on D3Q27 factorises per axis:
    f_i^eq = rho prod_a phi(c_ia, u_a), phi(0,u) = 2/3 - u^2,
    phi(+-1,u) = (1/3 +- u + u^2)/2 (exact, no truncation)."""
    c, _, _ = O.lattice()

    def phi(ci, u):
        return 2.0 / 3.0 - u * u if ci == 0 else (1.0 / 3.0 + ci * u + u * u) / 2.0

    for _ in range(20):
        rho, u = _random_state(rng, 0.3)
        prod = np.array([rho * phi(c[i, 0], u[0]) * phi(c[i, 1], u[1]) * phi(c[i, 2], u[2])
                         for i in range(27)])
        np.testing.assert_allclose(O.feq(rho, u), prod, rtol=1e-14, atol=1e-17)


def test_equilibrium_at_rest_is_weights(O):
    _, w, _ = O.lattice()
    np.testing.assert_allclose(O.feq(1.3, [0, 0, 0]), 1.3 * w, rtol=1e-15)


# ------------------------------------------------------------------ forcing
def _cstep_grad(fun, x, d, h=1e-30):
    xc = np.array(x, dtype=np.complex128)
    xc[d] += 1j * h
    return np.imag(fun(xc)) / h


def test_printed_forcing_moments_are_velocity_derivatives_of_meq(O, rng):
    """The printed R_k^MRT equal a . grad_u m_k^eq for all 27 k (derivative of
    the printed m^eq, taken by complex step)."""
    for _ in range(20):
        rho, u = _random_state(rng)
        a = rng.normal(0, 1e-3, size=3)
        dm = sum(a[d] * _cstep_grad(lambda uc: O.meq_complex(rho, uc), u, d) for d in range(3))
        np.testing.assert_allclose(O.rmrt(rho, u, a), dm, rtol=0, atol=1e-17)


def test_population_forcing_maps_to_printed_R(O, rng):
    """Population-space forcing F_i = a . grad_u f_i^eq has moments A F = R."""
    A = O.moment_matrix()
    for _ in range(20):
        rho, u = _random_state(rng)
        a = rng.normal(0, 1e-3, size=3)
        F = sum(a[d] * _cstep_grad(lambda uc: O.feq_complex(rho, uc), u, d) for d in range(3))
        np.testing.assert_allclose(A @ F, O.rmrt(rho, u, a), rtol=0, atol=1e-17)


# ------------------------------------------------------------------ collision
def _random_f(O, rng, amp=1e-2):
    rho, u = _random_state(rng)
    return O.feq(rho, u) * (1.0 + rng.uniform(-amp, amp, size=27))


def test_unforced_post_collision_moments(O, rng):
    """Appendix, unforced case: m*_k = m_k^eq except k = 4..8, where
    m*_k = (1 - omega) m_k + omega m_k^eq."""
    A = O.moment_matrix()
    _, w, _ = O.lattice()
    for omega in (0.6, 1.25, 1.9):
        for _ in range(10):
            f = _random_f(O, rng)
            m = A @ f
            rho = m[0]
            u = m[1:4] / rho
            ms = A @ O.collide(f, [0, 0, 0], omega)
            meq = O.meq(rho, u)
            expect = meq.copy()
            expect[4:9] = (1 - omega) * m[4:9] + omega * meq[4:9]
            np.testing.assert_allclose(ms, expect, rtol=0, atol=2e-15)


def test_collision_conserves_mass_and_adds_momentum_rho_a(O, rng):
    """Guo forcing: sum f* = sum f and sum c f* = sum c f + rho a."""
    c, _, _ = O.lattice()
    for _ in range(30):
        f = _random_f(O, rng)
        a = rng.normal(0, 1e-3, size=3)
        fs = O.collide(f, a, 1.0 / 0.53)
        assert abs(fs.sum() - f.sum()) < 2e-15
        np.testing.assert_allclose(c.T @ fs, c.T @ f + f.sum() * a, rtol=0, atol=1e-15)


def test_equilibrium_is_fixed_point_of_unforced_collision(O, rng):
    for _ in range(10):
        rho, u = _random_state(rng)
        feq = O.feq(rho, u)
        np.testing.assert_allclose(O.collide(feq, [0, 0, 0], 1.7), feq, rtol=0, atol=1e-15)


# ------------------------------------------------------------------ walls
def test_bouzidi_reduces_to_halfway_bounce_back_at_half(O):
    """Eq. (fbc1) at Delta = 1/2 is halfway bounce-back; Eq. (fbc2) at
    Delta -> 1/2 from below agrees (the scheme is continuous)."""
    assert O.bouzidi(0.5, 0.3, 0.7, 0.11) == 0.3
    below = O.bouzidi(0.5 - 1e-12, 0.3, 0.7, 0.11)
    assert abs(below - 0.3) < 1e-11
    # Delta = 1: average of reflected and own incoming population
    assert abs(O.bouzidi(1.0, 0.3, 0.7, 0.11) - (0.3 / 2 + 0.7 / 2)) < 1e-16
    # no second fluid node: falls back to bounce-back
    assert O.bouzidi(0.2, 0.3, 0.7, 0.11, has_ff=False) == 0.3


def test_wall_fraction_is_the_ray_circle_intersection(O):
    """Delta along +x from (x, y): (px + Delta)^2 + py^2 = R^2 in closed form;
    along a diagonal the point p + Delta (1, 1) lies on the circle; the
    fraction is in (0, 1] exactly for links that cross the wall."""
    cfg = O.make_config(nx=24, ny=24, nz=1, radius=10.0)
    c, _, _ = O.lattice()
    xc = yc = 11.5
    d_px = [i for i in range(27) if tuple(c[i]) == (1, 0, 0)][0]
    d_diag = [i for i in range(27) if tuple(c[i]) == (1, 1, 0)][0]
    mask = O.Pipe(cfg).fluid_mask()[0]
    n_cut = 0
    for y in range(24):
        for x in range(24):
            if not mask[y, x]:
                continue
            px, py = x - xc, y - yc
            if not mask[y, x + 1]:
                n_cut += 1
                delta = O.wall_fraction(cfg, x, y, d_px)
                assert abs(delta - (np.sqrt(100.0 - py * py) - px)) < 1e-12
                assert 0.0 < delta <= 1.0
            if not mask[y + 1, x + 1]:
                delta = O.wall_fraction(cfg, x, y, d_diag)
                assert abs((px + delta) ** 2 + (py + delta) ** 2 - 100.0) < 1e-9
                assert 0.0 < delta <= 1.0
    assert n_cut > 10


def test_halfway_streaming_is_a_permutation(O):
    """Pull streaming with halfway bounce-back and periodic wrap maps the
    post-collision populations one-to-one onto the new populations."""
    cfg = O.make_config(nx=14, ny=13, nz=5, radius=5.7, tau=0.8)
    p = O.Pipe(cfg)
    mask = p.fluid_mask()
    n = mask.size
    vals = np.zeros((27,) + mask.shape)
    ids = np.arange(27 * n, dtype=np.float64).reshape(vals.shape) + 1.0
    vals[:, mask] = ids[:, mask]
    p.set_f(vals, 0)
    p.stream_only()
    out = p.get_f()
    assert sorted(out[:, mask].ravel()) == sorted(vals[:, mask].ravel())


def test_mass_conserved_with_bounce_back_not_with_bouzidi(O):
    """Halfway bounce-back conserves mass (no drift beyond rounding, and none
    that grows with time); Bouzidi interpolation does not (it is not a
    permutation), so its mass drift grows."""
    drift = {}
    for wall in (0, 1):
        cfg = O.make_config(nx=20, ny=20, nz=6, radius=8.3, tau=0.7, accel_z=2e-5, wall=wall)
        p = O.Pipe(cfg)
        m0 = p.sums()[0]
        p.step(100)
        d1 = abs(p.sums()[0] / m0 - 1.0)
        p.step(400)
        d2 = abs(p.sums()[0] / m0 - 1.0)
        drift[wall] = (d1, d2)
    assert drift[0][0] < 1e-12 and drift[0][1] < 1e-12
    assert abs(drift[0][1] - drift[0][0]) < 1e-13
    assert drift[1][0] > 1e-10 and drift[1][1] > 5 * drift[1][0]


def test_periodic_box_momentum_grows_by_force_times_mass(O):
    """No wall: total mass is constant and total momentum grows by a * M per
    step, exactly (collision adds rho a at each node, streaming permutes).
    In FP64 the dense transforms of 20 steps at 210 nodes round each
    population to ~1e-16 relative, so the sums hold to 1e-13 of the mass."""
    rng = np.random.default_rng(20240521)  # this test's own input, whatever ran before
    cfg = O.make_config(nx=6, ny=5, nz=7, radius=0.0, tau=0.9, accel_z=3e-5)
    p = O.Pipe(cfg)
    f = p.get_f() * (1.0 + rng.uniform(-0.01, 0.01, size=p.get_f().shape))
    p.set_f(f, 0)
    s0 = p.sums()
    p.step(20)
    s1 = p.sums()
    tol = 1e-13 * s0[0]
    assert abs(s1[0] - s0[0]) < tol
    np.testing.assert_allclose(s1[1:3], s0[1:3], atol=tol)
    assert abs(s1[3] - (s0[3] + 20 * 3e-5 * s0[0])) < tol


# ------------------------------------------------------------------ trigger force
def _force_cfg(O):
    return O.make_config(nx=64, ny=64, nz=40, radius=30.0, tau=0.6, accel_z=1e-6, n_modes=6,
                         kz=3.0, kappa=0.5, l0_frac=0.2, l_frac=0.4, period=100.0,
                         force_off_step=10 ** 6)


def test_trigger_force_is_divergence_free(O, rng):
    """Eq. (TurbForce) is solenoidal; so is the sum of rotated modes."""
    cfg = _force_cfg(O)
    amps = rng.uniform(0.5, 1.5, size=12)
    h = 1e-4
    xc = yc = 31.5
    checked = 0
    for _ in range(200):
        r = rng.uniform(0.4 * 30 + 0.05, 0.8 * 30 - 0.05)
        th = rng.uniform(0, 2 * np.pi)
        x, y, z = xc + r * np.cos(th), yc + r * np.sin(th), rng.uniform(0, 40)
        div = 0.0
        for d in range(3):
            e = np.zeros(3)
            e[d] = h
            fp = O.trigger_shape(cfg, amps, x + e[0], y + e[1], z + e[2])
            fm = O.trigger_shape(cfg, amps, x - e[0], y - e[1], z - e[2])
            div += (fp[d] - fm[d]) / (2 * h)
        scale = np.abs(O.trigger_shape(cfg, amps, x, y, z)).max()
        assert abs(div) < 1e-6 * max(scale, 1e-12) + 1e-9
        checked += 1
    assert checked == 200


def test_trigger_force_vanishes_on_region_edges(O):
    """All three components vanish at r = R - l0 and r = R - l0 - l, and the
    force is zero outside that annulus."""
    cfg = _force_cfg(O)
    amps = np.ones(12)
    for r in (30 - 6.0, 30 - 6.0 - 12.0):
        for th in np.linspace(0, 2 * np.pi, 13):
            v = O.trigger_shape(cfg, amps, 31.5 + r * np.cos(th), 31.5 + r * np.sin(th), 7.3)
            assert np.abs(v).max() < 1e-12
    for r in (3.0, 25.0, 29.0):
        v = O.trigger_shape(cfg, amps, 31.5 + r, 31.5, 2.0)
        assert np.abs(v).max() == 0.0


def test_trigger_force_single_mode_structure(O):
    """Mode (k_theta = 2, cos) of Eq. (TurbForce): F_z ~ sin(k_z 2 pi z / L)
    cos(2 theta); the sin-phase mode is the cos mode rotated by pi/4."""
    cfg = _force_cfg(O)
    cos2 = np.zeros(12)
    cos2[2] = 1.0
    sin2 = np.zeros(12)
    sin2[3] = 1.0
    r, z = 18.0, 3.1
    for th in np.linspace(0, 2 * np.pi, 9):
        a = O.trigger_shape(cfg, cos2, 31.5 + r * np.cos(th), 31.5 + r * np.sin(th), z)
        b = O.trigger_shape(cfg, sin2, 31.5 + r * np.cos(th + np.pi / 4),
                            31.5 + r * np.sin(th + np.pi / 4), z)
        assert abs(a[2] - b[2]) < 1e-13
        # rotating the point rotates the in-plane vector
        ca, sa = np.cos(np.pi / 4), np.sin(np.pi / 4)
        np.testing.assert_allclose([ca * a[0] - sa * a[1], sa * a[0] + ca * a[1]], b[:2], atol=1e-13)
    a0 = O.trigger_shape(cfg, cos2, 31.5 + r, 31.5, z)
    a1 = O.trigger_shape(cfg, cos2, 31.5 + r, 31.5, z + 40.0 / 12.0)  # quarter kz-wavelength
    # F_z: sin(kz 2 pi z/L) -> cos after a quarter wavelength shift of the phase
    ph = 3 * 2 * np.pi * z / 40.0
    assert abs(a0[2] * np.cos(ph) - a1[2] * np.sin(ph)) < 1e-13
