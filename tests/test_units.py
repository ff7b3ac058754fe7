"""Lattice <-> physical units (Sec. II.E, Eqs. 40-44) against the worked
examples the paper prints (tests/golden/units_worked_examples.json: Sec. III.C
m_o = 1e-15, t_o = 1e-6/30, gamma_lbm = 1/45; Sec. IV.B m_o = 2.16e-13,
t_o = 1.2e-6, gamma_lbm = 2/15)."""
import json
import os

import pytest

from paper_2407_10914_amd.units import Units, lattice_viscosity

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = json.load(open(os.path.join(HERE, "golden", "units_worked_examples.json")))["cases"]


@pytest.mark.parametrize("c", CASES, ids=[c["name"] for c in CASES])
def test_worked_example(c):
    nu = lattice_viscosity(c["tau"])
    u = Units.from_physics(c["a_o"], c["rho_phys"], c["nu_phys"], nu, rho_lbm=c["rho_lbm"])
    p = c["printed"]
    assert nu == pytest.approx(p["nu_lbm"], rel=1e-14)
    assert u.m_o == pytest.approx(p["m_o"], rel=1e-12)
    assert u.t_o == pytest.approx(p["t_o"], rel=1e-12)
    assert u.tension_to_lbm(c["gamma_phys"]) == pytest.approx(p["gamma_lbm"], rel=1e-12)
    assert u.tension_to_phys(p["gamma_lbm"]) == pytest.approx(c["gamma_phys"], rel=1e-12)


def test_pressure_round_trip_and_scale():
    u = Units(a_o=6e-6, m_o=2.16e-13, t_o=1.2e-6)
    # Eq. (43): 1 m.u./(l.u. t.u.^2) = m_o / (a_o t_o^2) Pa
    assert u.pressure_to_phys(1.0) == pytest.approx(2.16e-13 / (6e-6 * 1.44e-12), rel=1e-14)
    assert u.pressure_to_lbm(u.pressure_to_phys(0.0123)) == pytest.approx(0.0123, rel=1e-14)
    # a Laplace pressure converts as sigma / R does (Eq. 43 / Eq. 44 = 1 / a_o)
    assert u.pressure_to_phys(0.01 / 20.0) == pytest.approx(u.tension_to_phys(0.01) / (20.0 * u.a_o), rel=1e-14)
