"""Helpers of the GPU parity tests: one run on each side from the same seeded
case, and the two comparisons (whole-run FP64, per-step FP32)."""
import sys

import numpy as np

import oracle as O
from cases import rel

TOL64 = 1e-12
TOL32 = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu(case, kw, precision, **extra):
    from paper_2407_10914_amd.sim import Sim

    s = Sim(case.solid, precision=precision, **kw, **extra)
    s.set_phase(case.phi0)
    return s


def orc(case, kw, eps="f64"):
    o = O.OracleSim(case.solid, eps=eps, **kw)
    o.set_phase(case.phi0)
    return o


def compare_macro(g, o, fluid, tol, tag):
    gm = dict(rho_r=g.field("rho_r"), rho_b=g.field("rho_b"), u=g.field("u"))
    om = o.macro()
    out = {k: rel(gm[k], om[k], fluid) for k in ("rho_r", "rho_b", "u")}
    say(tag, {k: f"{v:.3e}" for k, v in out.items()})
    for k, v in out.items():
        assert v <= tol, (tag, k, v)
    return out


def fp32_step_from(g, case, kw, tag, before=None):
    """Export the GPU FP32 state exactly, take one oracle step from it and one
    GPU step, compare (1e-6 relative per field).  `before(o)` may change the
    oracle's parameters the same way the GPU run's were changed."""
    fr, fb = g.populations()
    o = O.OracleSim(case.solid, eps="f32", **kw)
    o.set_state(fr, fb)
    if before is not None:
        before(o)
    g.step(1)
    o.step(1)
    return compare_macro(g, o, case.solid == 0, TOL32, tag)


def outlet_mixed(phi, fluid):
    """Number of outlet-plane fluid nodes with |phi| < 0.9."""
    return int((np.abs(phi[-1][fluid[-1]]) < 0.9).sum())
