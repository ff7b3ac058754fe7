"""The drainage/imbibition protocol on the GPU.

* A fixed schedule (drainage stages, a spontaneous stage at zero pressure
  difference, the switch to water injection of Eqs. 37-38, a forced stage)
  on a small rock, for both pressure drives, against the oracle running the
  same schedule: bitwise in FP64, including the slab observables that the
  protocol reads (S_w and the mass saturation of the porous region).
* The protocol driver itself on a 64^3 rock: drainage lowers the wetting
  saturation of the sample, forced imbibition raises it again.
"""
import numpy as np
import pytest

import oracle as O
from cases import rel
from paper_2407_10914_amd import inputs
from parity_helpers import TOL64, compare_macro, say

pytestmark = pytest.mark.gpu


def _small_rock(n=24, buffer=3):
    case = inputs.grf_rock(n=n, corr=4.0, porosity=0.3, seed=2412, buffer=buffer)
    kw = dict(dim=3, periodic=case.periodic, tau_r=1.0, tau_b=0.6, sigma=0.01, beta=0.95, scheme=1,
              theta_deg=30.0, bc=1, rho_in=1.0, rho_out=1.0, zeta_r=1.0, collision=1)
    return case, kw


@pytest.mark.parametrize("drive", ["type1", "type2"])
def test_fixed_schedule_fp64_against_the_oracle(drive):
    from paper_2407_10914_amd.protocol import Driver
    from paper_2407_10914_amd.sim import Sim

    case, kw = _small_rock()
    nz = case.solid.shape[0]
    g = Sim(case.solid, precision="f64", **kw)
    g.set_phase(case.phi0)
    o = O.OracleSim(case.solid, **kw)
    o.set_phase(case.phi0)
    dg = Driver(g, drive, nz)

    class OrcAdapter:
        def set_pressure(self, a, b):
            o.set_pressure(a, b)

        def set_body_force(self, gg):
            o.set_body_force(gg)

    do = Driver(OrcAdapter(), drive, nz)
    region = (2, 3, nz - 3)
    fluid = case.solid == 0
    for phase, drho, n in (("drainage", 0.02, 150), ("drainage", 0.05, 150), ("spontaneous", 0.0, 100),
                           ("switch", None, 0), ("forced", 0.04, 150)):
        if phase == "switch":
            g.switch_inlet(0.0)
            o.switch_inlet(0.0)
            continue
        dg.apply(drho)
        do.apply(drho)
        g.step(n)
        o.step(n)
        a, b = g.observe(slab=region), o.observe(slab=region)
        say(f"{drive} {phase} drho {drho}: S_w {a['sat_w']:.6f} / {b['sat_w']:.6f}")
        for k in ("sat_w", "sat_nw_mass", "mass_r", "mass_b", "n_fluid", "vol_r"):
            assert abs(a[k] - b[k]) <= 1e-12 * max(1.0, abs(b[k])), (phase, k, a[k], b[k])
    compare_macro(g, o, fluid, TOL64, f"protocol schedule {drive}")


def test_protocol_driver_on_a_64_rock():
    from paper_2407_10914_amd import protocol

    sim, case, region = protocol.rock_run(64, "type1", buffer=4)
    st = protocol.run_protocol(sim, drive="type1", region=region, length=case.solid.shape[0],
                               drainage=(0.02, 0.06), spontaneous=(0.0,), forced=(0.06,), check=500, window=3,
                               tol=3e-3, min_steps=2000, max_steps=12000, log=lambda m: say(m))
    sw = [s.s_w for s in st]
    say("S_w per stage:", sw)
    assert sw[0] < 0.999 and sw[1] < sw[0]  # oil invades, more at the higher pressure
    assert sw[-1] > sw[1]  # water comes back when it is injected
    # the inlet plane holds water after the switch
    ph = sim.field("phi")
    fl = case.solid == 0
    assert np.all(ph[0][fl[0]] == -1.0)
