"""Pins of the oracle's discrete adjoint (gradient of the time-averaged
streamwise kinetic energy with respect to the trigger-force amplitudes).

Three independent routes must agree on a tiny pipe: the reverse sweep with
complex-step node Jacobians, the complex-step tangent of the whole run, and
central finite differences of the objective.
"""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def O(oracle_mod):
    return oracle_mod


def _tiny(O, wall):
    return O.make_config(nx=12, ny=12, nz=8, radius=5.0, tau=0.6, accel_z=1e-5, n_modes=2, kz=1.0,
                         kappa=0.5, l0_frac=0.2, l_frac=0.4, period=20.0, force_off_step=1000,
                         wall=wall, init=1, u_tau=0.01)


AMPS = np.array([1e-4, 2e-4, 3e-4, 1.5e-4])


@pytest.mark.parametrize("wall", [0, 1])
def test_adjoint_equals_tangent(O, wall):
    cfg = _tiny(O, wall)
    J1, g1 = O.adjoint_gradient(cfg, AMPS, 20, 40)
    J2, g2 = O.tangent_gradient(cfg, AMPS, 20, 40)
    assert abs(J1 - J2) < 1e-14 * abs(J2)
    assert np.abs(g1 - g2).max() < 1e-12 * np.abs(g2).max()


def test_adjoint_matches_central_differences(O):
    cfg = _tiny(O, 0)
    J, g = O.adjoint_gradient(cfg, AMPS, 20, 40)
    assert abs(J - O.objective(cfg, AMPS, 20, 40)) < 1e-15 * abs(J)
    eps = 1e-6
    fd = []
    for q in range(len(AMPS)):
        ap, am = AMPS.copy(), AMPS.copy()
        ap[q] += eps
        am[q] -= eps
        fd.append((O.objective(cfg, ap, 20, 40) - O.objective(cfg, am, 20, 40)) / (2 * eps))
    fd = np.array(fd)
    assert np.abs(g - fd).max() < 1e-7 * np.abs(fd).max()


def test_gradient_vanishes_when_force_is_off(O):
    """With the trigger force switched off from step 0 the objective does not
    depend on the amplitudes."""
    cfg = _tiny(O, 0)
    cfg.force_off_step = 0
    J, g = O.adjoint_gradient(cfg, AMPS, 5, 10)
    assert np.all(g == 0.0)
