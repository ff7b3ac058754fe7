"""Quasi-static drainage and imbibition of a porous sample (Sec. IV.B).

The sample starts saturated with the wetting fluid b (water).  The protocol
then runs three phases, each a list of pressure stages, and advances every
stage until the wetting saturation of the porous region stops changing:

1. primary drainage: the non-wetting fluid r (oil) is injected at z = 0 and
   the pressure difference between inlet and outlet is raised stage by stage;
   the last drainage saturation is the irreducible wetting saturation S_w,irr;
2. spontaneous imbibition: the pressure difference is lowered back to zero
   while oil is still injected;
3. forced imbibition: the inlet switches to water (Eqs. 37-38, a library
   call on the device state) and the pressure difference is raised again;
   the capillary pressure is then counted negative.

The pressure difference is imposed by one of the two implementations of
Sec. II.C: Type-I, Zou-He densities rho_in = rho_out + drho at the open
faces (Appendix B); Type-II, equal densities at both faces and a body force
g = drho / (3 L) along z (Eq. 36) that gives the same mean gradient over the
sample length L.  The capillary pressure of a stage is P_c = drho / 3 (Eq.
23 with c = 1), positive while oil is injected, negative while water is.

S_w is the node count of phi < 0 over the fluid nodes of the porous region
(the buffer layers excluded), as Sec. IV.B defines it; the mass saturation
sum rho^r / sum rho of the region is reported beside it.  Every number comes
from the device reductions (cg_lbm_observe_slab); the host only schedules
stages.  Steady state: S_w changes by less than `tol` over `window`
consecutive checks `check` steps apart (and at least `min_steps` steps), or
the stage stops at `max_steps` and is marked unconverged.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time


@dataclasses.dataclass
class Stage:
    phase: str  # "drainage", "spontaneous", "forced"
    drho: float  # density difference imposed (Type-I) or its body-force equivalent (Type-II)
    p_c: float  # capillary pressure of the stage, lattice units
    steps: int
    s_w: float
    s_nw_mass: float
    converged: bool
    history: list  # (step, S_w) at every check


# Pressure stages of the default protocol (density differences).  The entry
# pressure of the synthetic rock is about 2 sigma cos(theta) / r with pore
# radii of 3-5 voxels: drho ~ 0.01-0.02 for sigma = 0.01, theta = 30 deg.
DRAINAGE = (0.005, 0.01, 0.015, 0.02, 0.03, 0.045, 0.06)
SPONTANEOUS = (0.03, 0.015, 0.0)
FORCED = (0.01, 0.02, 0.04, 0.06)


class Driver:
    """Applies the pressure difference of a stage to a run (Sim)."""

    def __init__(self, sim, drive: str, length: int, rho_out: float = 1.0):
        if drive not in ("type1", "type2"):
            raise ValueError("drive must be 'type1' or 'type2'")
        self.sim, self.drive, self.length, self.rho_out = sim, drive, length, rho_out

    def apply(self, drho: float):
        if self.drive == "type1":
            self.sim.set_pressure(self.rho_out + drho, self.rho_out)
        else:
            self.sim.set_body_force((0.0, 0.0, drho / (3.0 * self.length)))


def settle(sim, region, *, check, window, tol, min_steps, max_steps):
    """Steps until S_w of the region is steady; returns (steps, obs, converged,
    history)."""
    hist = []
    steps = 0
    obs = None
    while steps < max_steps:
        sim.step(check)
        steps += check
        obs = sim.observe(slab=(2, region[0], region[1]), check=False)
        if obs["nan_count"] > 0:
            raise FloatingPointError(f"non-finite state after {sim.time} steps")
        hist.append((sim.time, obs["sat_w"]))
        if steps >= min_steps and len(hist) > window:
            recent = [h[1] for h in hist[-(window + 1):]]
            if max(recent) - min(recent) < tol:
                return steps, obs, True, hist
    return steps, obs, False, hist


def run_protocol(sim, *, drive, region, length, drainage=DRAINAGE, spontaneous=SPONTANEOUS, forced=FORCED,
                 check=1000, window=3, tol=2e-3, min_steps=4000, max_steps=40000, log=None, on_stage=None):
    """Runs the three phases on `sim` (a Sim with Zou-He faces on z, injecting
    the non-wetting fluid, zeta_r = 1).  Returns the list of Stage records;
    on_stage(records) is called after every stage."""
    drv = Driver(sim, drive, length)
    out = []

    def stage(phase, drho, sign):
        drv.apply(drho)
        steps, obs, conv, hist = settle(sim, region, check=check, window=window, tol=tol, min_steps=min_steps,
                                        max_steps=max_steps)
        st = Stage(phase, drho, sign * drho / 3.0, steps, obs["sat_w"], obs["sat_nw_mass"], conv, hist)
        out.append(st)
        if on_stage:
            on_stage(out)
        if log:
            log(f"{phase:12s} drho {drho:.4f} P_c {st.p_c:+.5f}: S_w {st.s_w:.4f} S_nw(mass) {st.s_nw_mass:.4f} "
                f"after {steps} steps{'' if conv else ' (max steps)'}")

    for d in drainage:
        stage("drainage", d, +1.0)
    for d in spontaneous:
        stage("spontaneous", d, +1.0)
    sim.switch_inlet(0.0)  # Eqs. (37)-(38): water is injected from now on
    for d in forced:
        stage("forced", d, -1.0)
    return out


def summary(stages):
    d = [s for s in stages if s.phase == "drainage"]
    sp = [s for s in stages if s.phase == "spontaneous"]
    fo = [s for s in stages if s.phase == "forced"]
    return {"S_w_irr": d[-1].s_w if d else None, "S_w_spontaneous": sp[-1].s_w if sp else None,
            "S_w_final": fo[-1].s_w if fo else None,
            "steps": sum(s.steps for s in stages), "all_converged": all(s.converged for s in stages)}


def rock_run(n, drive, precision="f32", theta=30.0, sigma=0.01, buffer=10, seed=None):
    """The synthetic-rock workload (the benchmark's rock at edge n) set up for
    the protocol: Scheme-I at theta, MRT, tau_r = 1.0 (oil), tau_b = 0.6
    (water), oil injected at z = 0."""
    from . import inputs
    from .sim import Sim

    case = inputs.grf_rock(n=n, corr=8.0, porosity=0.22, seed=inputs.MASTER_SEED if seed is None else seed,
                           buffer=buffer)
    kw = dict(dim=3, periodic=case.periodic, tau_r=1.0, tau_b=0.6, sigma=sigma, beta=0.95, scheme=1,
              theta_deg=theta, bc=1, rho_in=1.0, rho_out=1.0, zeta_r=1.0, collision=1)
    sim = Sim(case.solid, precision=precision, **kw)
    sim.set_phase(case.phi0)
    region = (buffer, case.solid.shape[0] - buffer)
    return sim, case, region


def main(argv=None):
    ap = argparse.ArgumentParser(description="drainage / imbibition protocol on the synthetic rock (Sec. IV.B)")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--drive", choices=("type1", "type2", "both"), default="both")
    ap.add_argument("--check", type=int, default=1000)
    ap.add_argument("--max-steps", type=int, default=40000)
    ap.add_argument("--min-steps", type=int, default=4000)
    ap.add_argument("--tol", type=float, default=2e-3)
    ap.add_argument("--json", default=None, help="write the stage records here")
    a = ap.parse_args(argv)
    import torch

    torch.cuda.set_device(0)
    res = {}
    workload = (f"synthetic rock {a.n}^3, porosity 0.22, sigma 0.01, theta 30 deg Scheme-I, MRT FP32, "
                f"tau_r 1.0 tau_b 0.6; steady when S_w moves < {a.tol} over {3 * a.check} steps, "
                f"{a.min_steps}-{a.max_steps} steps per stage")

    def dump(partial=None):
        if a.json:
            body = dict(res)
            if partial:
                body.update(partial)
            with open(a.json, "w") as f:
                json.dump({"workload": workload, "results": body}, f)

    for drive in (("type1", "type2") if a.drive == "both" else (a.drive,)):
        t0 = time.perf_counter()
        sim, case, region = rock_run(a.n, drive)
        stages = run_protocol(sim, drive=drive, region=region, length=case.solid.shape[0], check=a.check,
                              max_steps=a.max_steps, min_steps=a.min_steps, tol=a.tol,
                              log=lambda m: print(f"[{drive}] {m}", file=sys.stderr, flush=True),
                              on_stage=lambda st: dump({drive: {"partial": True,
                                                                "stages": [dataclasses.asdict(x) for x in st]}}))
        res[drive] = {"summary": summary(stages), "stages": [dataclasses.asdict(s) for s in stages],
                      "fluid_nodes": sim.info()["fluid"], "wall_s": round(time.perf_counter() - t0, 1)}
        print(f"[{drive}] {res[drive]['summary']}", file=sys.stderr, flush=True)
        del sim
        torch.cuda.empty_cache()
        dump()
    dump()
    print(json.dumps({k: v["summary"] for k, v in res.items()}))


if __name__ == "__main__":
    main()
