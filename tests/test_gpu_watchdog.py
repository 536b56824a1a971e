"""The failure watchdog of lbm_diagnostics (needs an MI355X): non-finite
populations and relative mass drift beyond a limit return LBM_ENAN.

The halfway bounce-back conserves mass to rounding (FP64 storage: 3e-13
relative over 300 steps of the laminar pipe driven at a = 1e-4, in the
oracle), the interpolated wall of Eqs. (fbc1)/(fbc2) does not (4e-8), so a
limit of 1e-10 passes one and stops the other."""
import numpy as np
import pytest

import lbm_inputs as LI

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_12082_amd as P
    P.lib()
    return P


def _laminar(wall):
    return dict(LI.preset("laminar"), storage=2, wall=wall, nz=8, accel_z=1e-4)


def test_mass_drift_limit(P, oracle_mod):
    O = oracle_mod
    tol = 1e-10
    # the oracle's own drift over the same steps: the interpolated wall leaks
    # mass well above the limit, the bounce-back stays far below it
    drift = {}
    for wall in (0, 1):
        o = O.Pipe(O.make_config(**_laminar(wall)))
        m0 = o.sums()[0]
        o.step(300)
        drift[wall] = abs(o.sums()[0] - m0) / m0
    assert drift[0] < 1e-2 * tol < tol < drift[1]
    for wall in (0, 1):
        p = P.Pipe(_laminar(wall))
        p.set_watchdog(tol)
        p.diagnostics(raise_on_nan=True)  # reference mass
        p.step(300)
        if wall == 0:
            p.diagnostics(raise_on_nan=True)
        else:
            with pytest.raises(P.LbmError, match="mass drift"):
                p.diagnostics(raise_on_nan=True)
            # a state write resets the reference: the next call passes
            g = p.populations()
            p.set_populations(g, p.step_index)
            p.diagnostics(raise_on_nan=True)
            p.set_watchdog(0.0)  # off
            p.step(300)
            p.diagnostics(raise_on_nan=True)


def test_non_finite_and_bad_limit(P):
    p = P.Pipe(_laminar(0))
    with pytest.raises(P.LbmError):
        p.set_watchdog(-1.0)
    with pytest.raises(P.LbmError):
        p.set_watchdog(float("nan"))
    g = p.populations()
    g[0, 3, 2, 11, 11] = float("nan")
    p.set_populations(g, 0)
    d = p.diagnostics()  # returns the sums; the non-finite count is set
    assert d[0, 4] >= 1
    with pytest.raises(P.LbmError, match="non-finite"):
        p.diagnostics(raise_on_nan=True)
