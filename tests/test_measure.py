"""Geometric observables of Sec. III.B (Eqs. 45-46) and Sec. IV.A read from a
phase field, pinned to closed forms: circular caps of known angle, synthetic
diffuse caps and fronts whose interface position is known exactly."""
import math

import numpy as np
import pytest

from paper_2407_10914_amd import measure as M


@pytest.mark.parametrize("theta", [15.0, 30.0, 60.0, 90.0, 120.0, 150.0, 165.0])
def test_cap_angle_of_an_exact_circular_cap(theta):
    R = 20.0
    t = math.radians(theta)
    b, h = 2.0 * R * math.sin(t), R * (1.0 - math.cos(t))
    assert M.cap_angle(b, h) == pytest.approx(theta, abs=1e-10)


def test_half_disc_is_ninety_degrees_and_bad_input_is_rejected():
    assert M.cap_angle(10.0, 5.0) == pytest.approx(90.0, abs=1e-12)
    with pytest.raises(ValueError):
        M.cap_angle(0.0, 1.0)


def test_crossings_interpolate_linearly():
    assert M.crossings([1.0, -1.0]) == [0.5]
    assert M.crossings([3.0, -1.0, -2.0, 2.0]) == pytest.approx([0.75, 2.5])
    assert M.crossings([1.0, 2.0], positions=[4.0, 5.0]) == []


@pytest.mark.parametrize("theta", [45.0, 90.0, 135.0])
def test_base_and_height_of_a_diffuse_cap(theta):
    """A tanh profile (width 2) around a circle that meets the halfway wall
    y = 0.5 at angle theta: the base on the first fluid row is the circle's
    chord there, the height its top above the wall (to the error of linear
    interpolation across a diffuse interface, here below 0.01)."""
    R, wall, xc = 15.0, 0.5, 40.0
    yc = wall - R * math.cos(math.radians(theta))
    ny, nx = 40, 80
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    phi = np.tanh(0.5 * (R - np.hypot(xx - xc, yy - yc)))
    b, h = M.drop_base_height(phi, wall=wall)
    chord = 2.0 * math.sqrt(R * R - (1.0 - yc) ** 2)
    assert b == pytest.approx(chord, abs=0.02)
    assert h == pytest.approx(yc + R - wall, abs=0.02)
    # the angle from the first fluid row differs from theta by O(1/R)
    assert M.drop_angle(phi, wall=wall) == pytest.approx(theta, abs=4.0)


def test_front_on_the_axis_and_from_the_volume():
    nz, ny, nx = 60, 9, 9
    z0 = 23.4
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    phi = np.tanh(z0 - z) * np.ones((nz, ny, nx))
    assert M.front_on_axis(phi, axis=0) == pytest.approx(z0, abs=0.02)
    sharp = np.where(z < 23, 1.0, -1.0) * np.ones((nz, ny, nx))
    fluid = np.ones((nz, ny, nx), dtype=bool)
    assert M.front_from_volume(sharp, fluid, area=ny * nx) == pytest.approx(23.0, abs=1e-12)

