"""Closed forms of the validation harness (no GPU): Washburn's law in the
forms of Eqs. (47), (48) and (49)-(51), the area error of Sec. IV.A and the
Laplace fit."""
import math

import numpy as np
import pytest

from paper_2407_10914_amd import validation as V

KW = dict(L=100.0, r=5.0, mu_w=1.0 / 6.0, mu_nw=1.0 / 30.0, dP=0.0, gamma=1.0 / 45.0, theta_deg=40.0)


def test_eq48_solves_eq47():
    t = np.linspace(0.0, 5e4, 11)
    for dP in (0.0, 0.004):
        kw = dict(KW, dP=dP)
        z = V.washburn_z(t, **kw)
        lhs = z * z * (kw["mu_w"] - kw["mu_nw"]) / 2.0 + kw["mu_nw"] * kw["L"] * z
        rhs = kw["r"] ** 2 / 8.0 * (dP + 2 * kw["gamma"] * math.cos(math.radians(kw["theta_deg"])) / kw["r"]) * t
        assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)
        # the inverse
        assert np.allclose(V.washburn_time(z, **kw), t, rtol=1e-10, atol=1e-8)


def test_eq49_is_eq48_in_scaled_variables():
    kw = KW
    t = np.linspace(0.0, 4e4, 9)
    z = V.washburn_z(t, **kw)
    dm = kw["mu_w"] - kw["mu_nw"]
    t_star = kw["gamma"] * t / (dm * kw["L"])  # Eq. (51)
    zs = V.washburn_scaled(t_star, r_over_L=kw["r"] / kw["L"], mu_w=kw["mu_w"], mu_nw=kw["mu_nw"],
                           dP_r2_over_2Lgamma=kw["dP"] * kw["r"] ** 2 / (2 * kw["L"] * kw["gamma"]),
                           theta_deg=kw["theta_deg"])
    assert np.allclose(zs, z / kw["L"], rtol=1e-12, atol=1e-14)  # Eq. (50)


def test_equal_viscosities_give_the_linear_law_and_the_limit_agrees():
    kw = dict(KW, mu_w=0.1, mu_nw=0.1, dP=0.002)
    t = np.linspace(0, 1e4, 5)
    z = V.washburn_z(t, **kw)
    assert np.allclose(np.diff(z, 2), 0.0, atol=1e-12)
    near = V.washburn_z(t, **dict(kw, mu_w=0.1 * (1 + 1e-7)))
    assert np.allclose(near, z, rtol=1e-5)


def test_washburn_short_time_and_neutral_pressure_limits():
    # neutral wetting without a pressure difference: nothing moves
    assert np.abs(V.washburn_z([0, 100, 1000], **dict(KW, theta_deg=90.0))).max() < 1e-10
    # at short times the non-wetting column dominates: z ~ drive t / (mu_nw L)
    t = 1e-3
    drive = KW["r"] ** 2 / 8 * 2 * KW["gamma"] * math.cos(math.radians(KW["theta_deg"])) / KW["r"]
    assert V.washburn_z(t, **KW) == pytest.approx(drive * t / (KW["mu_nw"] * KW["L"]), rel=1e-6)


def test_area_error():
    t = np.linspace(0, 10, 101)
    assert V.area_error(t, t ** 2, t ** 2) == 0.0
    # z = 1.1 t against z = t: areas differ by 10 %
    assert V.area_error(t, 1.1 * t, t) == pytest.approx(0.1, rel=1e-12)


def test_laplace_fit_recovers_slope_and_radius_from_volume():
    R = np.array([10.0, 15.0, 20.0, 30.0])
    dp = 0.022 * 2 / R + 1e-5
    s, c = V.laplace_fit(dp, R)
    assert s == pytest.approx(0.022, rel=1e-12) and c == pytest.approx(1e-5, rel=1e-9)
    assert V.drop_radius_from_volume(4 / 3 * math.pi * 12.5 ** 3) == pytest.approx(12.5, rel=1e-14)
