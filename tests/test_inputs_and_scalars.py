"""Seeded input generator and the paper's printed scalars (Section II.B)."""
import json
import math
import os

import numpy as np

import lbm_inputs as LI

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_scalars.json")


def test_splitmix64_reference_outputs():
    """SplitMix64 from state 0 (published reference sequence)."""
    s, outs = 0, []
    for _ in range(3):
        s, z = LI.splitmix64(s)
        outs.append(z)
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_amplitudes_seeded_and_bounded():
    a = LI.amplitudes(0, 6, 0.00388, 1206.0)
    b = LI.amplitudes(0, 6, 0.00388, 1206.0)
    c = LI.amplitudes(1, 6, 0.00388, 1206.0)
    assert a.shape == (12,) and np.array_equal(a, b) and not np.array_equal(a, c)
    unit = LI.amplitude_unit(0.00388, 1206.0)
    assert np.all(a >= 0) and np.all(a < 0.05 * unit)


def test_paper_scalars_are_consistent():
    """Section II.B: Re_tau = u* R / nu, delta_x+ = u*/nu, T^LET = R/u*,
    L/R, and the bulk Reynolds number, all mutually consistent."""
    g = json.load(open(GOLDEN))
    nu, ut, R = g["nu"], g["u_tau"], g["radius"]
    assert abs(ut * R / nu - g["Re_tau"]) < 0.05
    assert abs(ut / nu - g["delta_x_plus"]) < 0.001
    assert abs(R / ut - g["T_LET"]) < 1.0
    assert abs(g["grid"][2] / R - g["L_over_R"]) < 0.005
    assert abs(LI.BULK_OVER_UTAU - g["Re_bulk"] / (2 * g["Re_tau"])) < 1e-12
    # forcing period T ~ 0.052 T^LET ~ 2004 steps
    assert abs(g["T_over_TLET"] * g["T_LET"] - 2004) < 1.0
    # omega = (nu/cs^2 + 1/2)^-1: tau = 3 nu + 1/2
    assert abs(1.0 / (nu / (1 / 3) + 0.5) - 1.0 / (3 * nu + 0.5)) < 1e-15


def test_presets_follow_the_paper_relations():
    """u* = sqrt(h R / 2) and tau = 3 nu + 1/2 in every turbulent preset."""
    for name in ("turbulent", "precision_ref", "batched", "adjoint"):
        c = LI.preset(name)
        nu = (c["tau"] - 0.5) / 3.0
        assert abs(math.sqrt(c["accel_z"] * c["radius"] / 2) - c["u_tau"]) < 1e-15
        assert abs(c["period"] - round(0.052 * c["radius"] / c["u_tau"])) == 0
        if name in ("turbulent", "precision_ref"):
            assert abs(c["u_tau"] * 90.0 / nu - 181.3) < 1e-9
    t = LI.preset("turbulent")
    assert (t["nx"], t["ny"], t["nz"], t["radius"]) == (192, 192, 1152, 90.0)
    # the paper's own pipe, Section II.B
    g = json.load(open(GOLDEN))
    p = LI.preset("paper")
    nu = (p["tau"] - 0.5) / 3.0
    assert [p["nx"], p["ny"], p["nz"]] == g["grid"] and p["radius"] == g["radius"] and p["wall"] == 1
    assert abs(nu - g["nu"]) < 1e-15 and p["u_tau"] == g["u_tau"]
    assert abs(math.sqrt(p["accel_z"] * p["radius"] / 2) - g["u_tau"]) < 1e-15
    assert p["period"] == round(g["T_over_TLET"] * g["T_LET"])
    assert p["force_off_step"] == 3 * g["T_LET"] and p["steps"] == 30 * g["T_LET"]
    assert (p["kz"], p["kappa"], p["l0_frac"], p["l_frac"]) == (g["kz"], g["kappa"], g["l0_over_R"], g["l_over_R"])
    a = LI.preset_amplitudes(p)
    assert a.shape == (1, 2 * g["ktheta"]) and a[0, 2 * (g["ktheta"] - 1)] == g["A0"] * p["accel_z"]
    assert np.count_nonzero(a) == 1
    assert LI.preset("batched")["batch"] == 64


def test_deviation_generators_agree():
    """The full-field (numpy and torch) and pointwise generators give the same
    float32 values, so both sides of a parity test see identical inputs."""
    import torch
    shape = (5, 4, 3)
    a = LI.random_deviations(17, shape)
    b = LI.random_deviations_torch(17, shape, device="cpu").numpy()
    assert np.array_equal(a, b)
    rng = np.random.default_rng(0)
    i = rng.integers(0, 27, 50)
    flat = rng.integers(0, 60, 50)
    c = LI.random_deviations_at(17, shape, i, flat)
    assert np.array_equal(c, a.reshape(27, -1)[i, flat])
