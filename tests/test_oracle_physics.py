"""Physical pins of the FP64 oracle: closed-form flows the scheme must reproduce.

* shear-wave decay at the viscosity nu = c_s^2 (tau - 1/2) implied by
  omega = (nu/c_s^2 + 1/2)^-1 (appendix, after Eq. (lambda)), with second-order
  convergence and Galilean invariance of the decay rate;
* start-up and steady Hagen-Poiseuille flow in the pipe (the laminar
  reference profile u_z = a (R^2 - r^2) / (4 nu)), with halfway bounce-back
  on the staircase mask and with the Bouzidi wall of Eqs. (fbc1)-(fbc2).
"""
import numpy as np
import pytest
from scipy import special


@pytest.fixture(scope="module")
def O(oracle_mod):
    return oracle_mod


def _shear_wave_nu_error(O, N, tau, U0=0.0, amp=1e-4):
    cfg = O.make_config(nx=1, ny=1, nz=N, radius=0.0, tau=tau, accel_z=0.0)
    p = O.Pipe(cfg)
    f = np.zeros((27, N, 1, 1))
    for k in range(N):
        f[:, k, 0, 0] = O.feq(1.0, [amp * np.sin(2 * np.pi * k / N), 0.0, U0])
    p.set_f(f, 0)
    nu = (tau - 0.5) / 3.0
    kk = 2 * np.pi / N
    T = int(1.0 / (nu * kk * kk))
    z = np.arange(N)

    def amplitude():
        _, u = p.moments()
        return abs(np.sum(u[0, :, 0, 0] * np.exp(-2j * np.pi * z / N))) * 2 / N

    p.step(T // 4)
    a1, t1 = amplitude(), p.step_index
    p.step(T)
    a2, t2 = amplitude(), p.step_index
    return np.log(a1 / a2) / (kk * kk * (t2 - t1)) / nu - 1.0


def test_shear_wave_decay_gives_nu_of_tau(O):
    """u_x = U sin(2 pi z / N) decays as exp(-nu k^2 t) with nu = (tau-1/2)/3."""
    err = _shear_wave_nu_error(O, 64, 0.8)
    assert abs(err) < 2e-4
    err = _shear_wave_nu_error(O, 128, 0.51)
    assert abs(err) < 5e-4


def test_shear_wave_second_order_convergence(O):
    errs = [abs(_shear_wave_nu_error(O, N, 0.8)) for N in (16, 32, 64)]
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.9 < o < 2.1 for o in orders), orders


def test_shear_wave_galilean_invariance(O):
    """A background velocity U_z = 0.1 along the wave vector leaves the
    fitted viscosity unchanged to O(1e-5): the sixth-order equilibrium
    carries the velocity-dependent terms a truncated one would miss."""
    e0 = _shear_wave_nu_error(O, 64, 0.8, U0=0.0)
    e1 = _shear_wave_nu_error(O, 64, 0.8, U0=0.1)
    assert abs(e1 - e0) < 2e-5


def _poiseuille_series(r, t, R, nu, a, nterm=200):
    """Start-up flow in a pipe from rest (Szymanski): steady parabola minus a
    Bessel series in the zeros j_n of J_0."""
    jn = special.jn_zeros(0, nterm)
    s = 1.0 - r ** 2 / R ** 2
    for j in jn:
        s -= 8.0 * special.j0(j * r / R) / (j ** 3 * special.j1(j)) * np.exp(-j * j * nu * t / R ** 2)
    return a * R * R / (4.0 * nu) * s


def _poiseuille_error(O, wall, steps, nz=4):
    R, tau, a = 10.0, 0.8, 1e-6
    nu = (tau - 0.5) / 3.0
    cfg = O.make_config(nx=24, ny=24, nz=nz, radius=R, tau=tau, accel_z=a, wall=wall)
    p = O.Pipe(cfg)
    p.step(steps)
    _, u = p.moments()
    mask = p.fluid_mask()[0]
    yy, xx = np.mgrid[0:24, 0:24]
    r = np.hypot(xx - 11.5, yy - 11.5)[mask]
    exact = _poiseuille_series(r, steps, R, nu, a)
    uz = u[2, 0][mask]
    # the flow is z-invariant
    assert np.abs(u[2] - u[2, :1]).max() < 1e-18
    return np.sqrt(np.sum((uz - exact) ** 2) / np.sum(exact ** 2))


def test_poiseuille_startup_halfway_bounce_back(O):
    """Laminar pipe R = 10, tau = 0.8, a = 1e-6, from rest, 500 steps: the
    staircase halfway-bounce-back wall matches the start-up series within 5%
    (L2); the residual is the first-order geometric error of the mask."""
    assert _poiseuille_error(O, 0, 500) < 0.05


def test_poiseuille_startup_bouzidi(O):
    """Same flow with the interpolated wall of Eqs. (fbc1)-(fbc2): within 0.5%."""
    assert _poiseuille_error(O, 1, 500) < 0.005


def test_poiseuille_steady(O):
    """After 5000 steps (29 slowest e-folds) the profile is the steady
    parabola a (R^2 - r^2) / (4 nu)."""
    assert _poiseuille_error(O, 1, 5000, nz=2) < 0.005
    assert _poiseuille_error(O, 0, 5000, nz=2) < 0.05


def test_laminar_pipe_is_axisymmetric(O):
    """The cylinder mask has the symmetries of the square, so the flow does."""
    cfg = O.make_config(nx=24, ny=24, nz=3, radius=10.0, tau=0.8, accel_z=1e-6)
    p = O.Pipe(cfg)
    p.step(200)
    _, u = p.moments()
    uz = u[2, 0]
    tol = 1e-10 * np.abs(uz).max()  # equal up to summation order
    np.testing.assert_allclose(uz, uz.T, rtol=0, atol=tol)
    np.testing.assert_allclose(uz, uz[::-1, :], rtol=0, atol=tol)
    # in-plane velocity is odd under the mirror that flips its component
    ux, uy = u[0, 0], u[1, 0]
    np.testing.assert_allclose(ux, -ux[:, ::-1], rtol=0, atol=tol)
    np.testing.assert_allclose(uy, -uy[::-1, :], rtol=0, atol=tol)


def test_loglaw_start_reduces_to_the_wall_laws(O):
    """The oracle's log-law start (Section II.B initial condition), pinned on
    the paper's pipe section (300x300, R = 149.5, nu = 0.0032, u* = 0.00388)
    by what does not restate its formula:
    * in the viscous sublayer the mean velocity in wall units equals the
      wall distance in wall units (the no-slip law of the wall, u = u*^2
      delta / nu): a wrong viscosity, wall distance or u* scaling fails it;
    * in the log region U+ grows by 1/kappa per e-fold of delta+ with von
      Karman's kappa = 0.4 (a base-10 logarithm or the wrong branch fails);
    * the bulk Reynolds number 2 R u_b / nu of this start is within 10% of
      the printed Re ~ 5329.3 of the developed flow (tests/golden): the log
      law without a wake term sits a few percent below it (5041 here), a
      wrong scale by far more."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_scalars.json")))
    nu, ut, R = g["nu"], g["u_tau"], g["radius"]
    n = g["grid"][0]
    cfg = O.make_config(nx=n, ny=n, nz=1, radius=R, tau=3 * nu + 0.5, accel_z=0.0, init=1, u_tau=ut)
    p = O.Pipe(cfg)
    rho, u = p.moments()
    mask = p.fluid_mask()[0]
    yy, xx = np.mgrid[0:n, 0:n]
    r = np.hypot(xx - 0.5 * (n - 1), yy - 0.5 * (n - 1))[mask]
    uz = u[2, 0][mask]
    assert np.allclose(rho[0][mask], 1.0, atol=1e-12) and np.abs(u[:2, 0][:, mask]).max() < 1e-15
    dplus = (R - r) * ut / nu
    Uplus = uz / ut
    sub = dplus < 10.0
    assert sub.sum() > 100
    np.testing.assert_allclose(uz[sub], ut * ut * (R - r[sub]) / nu, rtol=1e-12)
    log = dplus > 30.0
    slope = np.polyfit(np.log(dplus[log]), Uplus[log], 1)[0]
    assert abs(slope - 1.0 / 0.4) < 1e-9
    ub = uz.mean()  # one node per unit area: the section average is the bulk velocity
    Re = 2 * R * ub / nu
    assert abs(Re / g["Re_bulk"] - 1.0) < 0.1, Re
