"""Lattice <-> physical units (Sec. II.E, Eqs. 40-44).

Results are scaled by a length unit a_o, a mass unit m_o and a time unit t_o:
a_o = l_phys / x_lbm (Eq. 40), m_o = rho_phys a_o^3 / rho_lbm (Eq. 41),
t_o = nu_lbm a_o^2 / nu_phys (Eq. 42); a pressure scales by m_o / (a_o t_o^2)
(Eq. 43) and an interfacial tension by m_o / t_o^2 (Eq. 44).  The lattice
viscosity of a relaxation time is nu = (tau - 1/2)/3 (Eq. 13).  Host
arithmetic only: this converts inputs and reported observables and is not on
the time step.
"""
from __future__ import annotations

from dataclasses import dataclass


def lattice_viscosity(tau: float) -> float:
    """nu_lbm = (tau - 1/2) / 3 in l.u.^2/t.u. (Eq. 13)."""
    return (tau - 0.5) / 3.0


@dataclass(frozen=True)
class Units:
    """The three scales of Sec. II.E (SI per lattice unit)."""

    a_o: float  # m / l.u.
    m_o: float  # kg / m.u.
    t_o: float  # s / t.u.

    @classmethod
    def from_physics(cls, l_phys: float, rho_phys: float, nu_phys: float, nu_lbm: float,
                     x_lbm: float = 1.0, rho_lbm: float = 1.0) -> "Units":
        a_o = l_phys / x_lbm                      # Eq. (40)
        m_o = rho_phys * a_o ** 3 / rho_lbm       # Eq. (41)
        t_o = nu_lbm * a_o ** 2 / nu_phys         # Eq. (42)
        return cls(a_o, m_o, t_o)

    def pressure_to_phys(self, p_lbm: float) -> float:
        """Pa from m.u./(l.u. t.u.^2), Eq. (43)."""
        return p_lbm * self.m_o / (self.a_o * self.t_o ** 2)

    def pressure_to_lbm(self, p_phys: float) -> float:
        return p_phys * self.a_o * self.t_o ** 2 / self.m_o

    def tension_to_phys(self, gamma_lbm: float) -> float:
        """N/m from m.u./t.u.^2, Eq. (44)."""
        return gamma_lbm * self.m_o / self.t_o ** 2

    def tension_to_lbm(self, gamma_phys: float) -> float:
        return gamma_phys * self.t_o ** 2 / self.m_o

    def velocity_to_phys(self, u_lbm: float) -> float:
        """m/s from l.u./t.u."""
        return u_lbm * self.a_o / self.t_o

    def time_to_phys(self, steps: float) -> float:
        """s from a number of time steps."""
        return steps * self.t_o
