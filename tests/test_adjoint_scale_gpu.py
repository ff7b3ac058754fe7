"""The adjoint at the size of the drainage workload it is specified for: the
128^3 Gaussian-random-field rock (porosity 0.22, z periodic, non-wetting
fluid in the inlet buffer, per-voxel contact angle 40 deg on the solid, body
force 1e-5 along z), objective = non-wetting mass saturation of the rock
region, checkpoints every 100 steps.

What holds at this size, measured:

* The step is a piecewise smooth map: the guards of Eq. 27 (|C| <= eps_c)
  and of the Scheme-I secant switch branch as the angle changes, so
  J(theta) has small kinks.  Over 2000 steps central differences do not
  converge as h -> 0 (the two one-sided differences differ by up to 30 % at
  h = 1e-4 deg); with h = 0.01 - 0.1 deg, above the kink scale, they agree
  with the adjoint (the exact derivative of the map with its branches held
  fixed) to about 2e-4, and dJ/dg_z to 3e-5 (h = 1 % of g).
* FP32 against FP64: over 500 steps J to ~3e-6 and the gradients to 1e-4;
  over 2000 steps the two trajectories themselves drift apart (J by ~2e-5)
  through the invasion events of the drainage, and their gradients differ
  by ~5e-3 (dJ/dtheta) and ~2e-2 (the field): reported, not held to 1e-4.
"""
import numpy as np
import pytest

from paper_2407_10914_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

K = 100


def _case():
    case, th = inputs.drainage_rock(n=128)
    kw = dict(dim=3, periodic=case.periodic, tau_r=1.0, tau_b=0.6, sigma=0.01, beta=0.95, scheme=1,
              theta_deg=40.0, collision=1, g=(0.0, 0.0, 1e-5))
    return case, th, kw


class Runs:
    def __init__(self, case, th, kw, prec):
        from paper_2407_10914_amd.sim import Sim

        self.case, self.th = case, th
        self.s = Sim(case.solid, precision=prec, theta_field=th, **kw)
        self.nz, self.buf = case.solid.shape[0], case.meta["buffer"]
        self.ones = (case.solid == 1).astype(float)

    def adjoint(self, steps):
        self.s.set_wetting(theta_field=self.th)
        self.s.set_body_force((0.0, 0.0, 1e-5))
        self.s.set_phase(self.case.phi0)
        r = self.s.adjoint("saturation", n_steps=steps, checkpoint_every=K, lo=self.buf, hi=self.nz - self.buf,
                           field_grad=True)
        return dict(J=r["J"], dth=r["dJ_dtheta"], dgz=float(r["dJ_dg"][2]), field=r["dJ_dtheta_field"].cpu().numpy())

    def J(self, steps, shift=0.0, gz=1e-5):
        self.s.set_wetting(theta_field=self.th + shift * self.ones)
        self.s.set_body_force((0.0, 0.0, gz))
        self.s.set_phase(self.case.phi0)
        self.s.step(steps)
        return self.s.observe(slab=(2, self.buf, self.nz - self.buf))["sat_nw_mass"]

    def close(self):
        del self.s
        torch.cuda.empty_cache()


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def test_adjoint_128_fp32_against_fp64_over_500_steps():
    case, th, kw = _case()
    r64 = Runs(case, th, kw, "f64")
    a64 = r64.adjoint(500)
    j0 = r64.J(500)
    fd_g = (r64.J(500, gz=1.01e-5) - r64.J(500, gz=0.99e-5)) / 2e-7
    fd_th = [(r64.J(500, h) - r64.J(500, -h)) / (2 * h) for h in (0.01, 0.03, 0.1)]
    r64.close()
    r32 = Runs(case, th, kw, "f32")
    a32 = r32.adjoint(500)
    r32.close()
    fdiff = np.linalg.norm(a32["field"] - a64["field"]) / np.linalg.norm(a64["field"])
    e_th = sorted(rel(a64["dth"], f) for f in fd_th)
    print(f"128^3 x 500: J {a64['J']:.12e} (forward {j0:.12e}); dtheta {a64['dth']:.9e} fd {fd_th} "
          f"rel {e_th}; dgz {a64['dgz']:.9e} fd {fd_g:.9e} rel {rel(a64['dgz'], fd_g):.2e}", flush=True)
    print(f"128^3 x 500 FP32 vs FP64: J {rel(a32['J'], a64['J']):.2e} dtheta {rel(a32['dth'], a64['dth']):.2e} "
          f"dgz {rel(a32['dgz'], a64['dgz']):.2e} field {fdiff:.2e}", flush=True)
    assert rel(a64["J"], j0) <= 1e-13
    assert rel(float(a64["field"].sum()), a64["dth"]) <= 1e-10
    assert rel(a64["dgz"], fd_g) <= 1e-4
    assert e_th[1] <= 3e-4  # the median of the three step sizes
    assert rel(a32["J"], a64["J"]) <= 1e-5
    assert rel(a32["dth"], a64["dth"]) <= 1e-4
    assert rel(a32["dgz"], a64["dgz"]) <= 1e-4
    assert fdiff <= 1e-4


def test_adjoint_128_over_2000_steps_against_central_differences():
    case, th, kw = _case()
    r64 = Runs(case, th, kw, "f64")
    a64 = r64.adjoint(2000)
    fd_th = (r64.J(2000, 0.03) - r64.J(2000, -0.03)) / 0.06
    fd_g = (r64.J(2000, gz=1.01e-5) - r64.J(2000, gz=0.99e-5)) / 2e-7
    r64.close()
    r32 = Runs(case, th, kw, "f32")
    a32 = r32.adjoint(2000)
    r32.close()
    fdiff = np.linalg.norm(a32["field"] - a64["field"]) / np.linalg.norm(a64["field"])
    print(f"128^3 x 2000: dtheta {a64['dth']:.9e} fd(h=0.03) {fd_th:.9e} rel {rel(a64['dth'], fd_th):.2e}; "
          f"dgz {a64['dgz']:.9e} fd {fd_g:.9e} rel {rel(a64['dgz'], fd_g):.2e}", flush=True)
    print(f"128^3 x 2000 FP32 vs FP64: J {rel(a32['J'], a64['J']):.2e} dtheta {rel(a32['dth'], a64['dth']):.2e} "
          f"dgz {rel(a32['dgz'], a64['dgz']):.2e} field {fdiff:.2e}", flush=True)
    assert rel(a64["dth"], fd_th) <= 5e-4
    assert rel(a64["dgz"], fd_g) <= 1e-4
    assert rel(a32["J"], a64["J"]) <= 1e-4
