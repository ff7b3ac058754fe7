"""Pins of the oracle's discrete derivative (forward mode on dual numbers).

The derivative of an objective of the state after n steps along the contact
angle (global or per-voxel field) or the body force is checked against
central finite differences of the oracle's own forward runs (which converge
to it at second order in the step), against linearity in the direction, and
against the identity that a uniform angle field moved uniformly is the global
angle moved.  These are the references for the GPU adjoint."""
import numpy as np
import pytest

import oracle as O
from paper_2407_10914_amd import inputs


def slug_2d():
    nx, ny = 24, 10
    solid = np.zeros((1, ny, nx), np.uint8)
    solid[0, 0, :] = 1
    solid[0, -1, :] = 1
    xx = np.arange(nx)[None, None, :] * np.ones((1, ny, 1))
    phi0 = np.where((xx >= 6) & (xx < 14), 1.0, -1.0)
    kw = dict(dim=2, periodic=(1, 0, 0), tau_r=1.0, tau_b=0.8, sigma=0.01, beta=0.7, scheme=1, theta_deg=60.0,
              collision=0, g=(2e-5, 0, 0))
    return solid, phi0, kw


def tiny_rock(scheme):
    c = inputs.grf_rock(n=14, nz=20, corr=3.0, porosity=0.35, seed=77, buffer=3)
    solid = c.solid
    nz = solid.shape[0]
    zz = np.arange(nz)[:, None, None] * np.ones(solid.shape)
    phi0 = np.where(zz < 3, 1.0, -1.0)
    kw = dict(dim=3, periodic=(0, 0, 1), tau_r=1.0, tau_b=0.6, sigma=0.01, beta=0.95, scheme=scheme,
              theta_deg=40.0, collision=1, g=(0, 0, 1e-4))
    return solid, phi0, kw


def run(solid, phi0, kw, steps, obj, axis, lo, hi, field=None, **over):
    k = dict(kw)
    k.update(over)
    s = O.OracleSim(solid, theta_field=field, **k)
    s.set_phase(phi0)
    s.step(steps)
    return s.objective(obj, axis=axis, lo=lo, hi=hi)


def central(f, h):
    return (f(h) - f(-h)) / (2 * h)


@pytest.mark.parametrize("obj,lo,hi", [("red_volume", 10, 20), ("sat_nw", 10, 20), ("flux", 5, 0)])
@pytest.mark.parametrize("seed", ["theta", "gx"])
def test_tangent_matches_central_differences_2d(obj, lo, hi, seed):
    solid, phi0, kw = slug_2d()
    steps = 40
    o = O.OracleSim(solid, **kw)
    J, dJ = o.tangent(phi0, objective=obj, n_steps=steps, seed=seed, axis=0, lo=lo, hi=hi)
    assert J == run(solid, phi0, kw, steps, obj, 0, lo, hi)
    if seed == "theta":
        f = lambda h: run(solid, phi0, kw, steps, obj, 0, lo, hi, theta_deg=60.0 + h)
        hs = (1e-2, 1e-3)
    else:
        f = lambda h: run(solid, phi0, kw, steps, obj, 0, lo, hi, g=(2e-5 + h, 0, 0))
        hs = (2e-7, 2e-8)
    errs = [abs(central(f, h) - dJ) / abs(dJ) for h in hs]
    assert errs[1] < 1e-6, errs


@pytest.mark.parametrize("scheme", [1, 2])
def test_tangent_field_matches_central_differences_3d(scheme):
    solid, phi0, kw = tiny_rock(scheme)
    nz = solid.shape[0]
    steps = 30
    th = np.where(solid == 1, 40.0, 0.0)
    dirn = np.where(solid == 1, np.random.default_rng(5).standard_normal(solid.shape), 0.0)
    o = O.OracleSim(solid, theta_field=th, **kw)
    J, dJ = o.tangent(phi0, objective="sat_nw", n_steps=steps, seed="theta_field", theta_dir=dirn, lo=3,
                      hi=nz - 3)
    f = lambda h: run(solid, phi0, kw, steps, "sat_nw", 2, 3, nz - 3, field=th + h * dirn)
    e1 = abs(central(f, 1e-3) - dJ) / abs(dJ)
    e2 = abs(central(f, 1e-4) - dJ) / abs(dJ)
    # second-order convergence of the differences onto the tangent
    assert e2 < 1e-5 and e2 < 0.05 * e1, (e1, e2)


@pytest.mark.parametrize("scheme", [1, 2])
def test_tangent_body_force_3d(scheme):
    solid, phi0, kw = tiny_rock(scheme)
    nz = solid.shape[0]
    steps = 30
    o = O.OracleSim(solid, **kw)
    J, dJ = o.tangent(phi0, objective="sat_nw", n_steps=steps, seed="gz", lo=3, hi=nz - 3)
    f = lambda h: run(solid, phi0, kw, steps, "sat_nw", 2, 3, nz - 3, g=(0, 0, 1e-4 + h))
    e1 = abs(central(f, 1e-8) - dJ) / abs(dJ)
    e2 = abs(central(f, 1e-9) - dJ) / abs(dJ)
    assert e2 < 1e-5, (e1, e2)


@pytest.mark.parametrize("scheme", [1, 2])
def test_uniform_field_direction_equals_global_angle(scheme):
    solid, phi0, kw = tiny_rock(scheme)
    nz = solid.shape[0]
    th = np.where(solid == 1, 40.0, 0.0)
    o = O.OracleSim(solid, **kw)
    Jg, dg = o.tangent(phi0, objective="red_volume", n_steps=20, seed="theta", lo=3, hi=nz - 3)
    of = O.OracleSim(solid, theta_field=th, **kw)
    Jf, df = of.tangent(phi0, objective="red_volume", n_steps=20, seed="theta_field",
                        theta_dir=(solid == 1).astype(float), lo=3, hi=nz - 3)
    assert abs(Jf - Jg) <= 1e-12 * abs(Jg)
    assert abs(df - dg) <= 1e-10 * abs(dg)


def test_tangent_is_linear_in_the_direction():
    solid, phi0, kw = tiny_rock(1)
    nz = solid.shape[0]
    th = np.where(solid == 1, 40.0, 0.0)
    rng = np.random.default_rng(11)
    d1 = np.where(solid == 1, rng.standard_normal(solid.shape), 0.0)
    d2 = np.where(solid == 1, rng.standard_normal(solid.shape), 0.0)
    o = O.OracleSim(solid, theta_field=th, **kw)
    t = [o.tangent(phi0, objective="sat_nw", n_steps=15, seed="theta_field", theta_dir=d, lo=3, hi=nz - 3)[1]
         for d in (d1, d2, 2.0 * d1 - 3.0 * d2)]
    assert abs(t[2] - (2.0 * t[0] - 3.0 * t[1])) <= 1e-10 * (abs(t[0]) + abs(t[1]))


def outlet_tube(zeta_r=0.25):
    """Short Type-I tube whose red slug sits against the outlet, so the
    outlet plane holds mixed phase from the first steps (chi^s strictly
    between 0 and 1, Eqs. B.12-B.18 with Eq. 39), with mixed injection at the
    inlet (Eq. B.1)."""
    c = inputs.tube(nx=10, ny=10, nz=14, radius=3.5, wet_len=4)
    z = np.arange(14)[:, None, None]
    phi0 = np.where((z >= 7) & (z < 13), 1.0, -1.0) * np.ones(c.solid.shape)
    kw = dict(dim=3, periodic=c.periodic, tau_r=1.0, tau_b=0.7, sigma=0.02, beta=0.95, scheme=2, theta_deg=60.0,
              bc=1, rho_in=1.04, rho_out=1.0, zeta_r=zeta_r, collision=1)
    return c.solid, phi0, kw


@pytest.mark.parametrize("obj,lo,hi", [("sat_nw", 0, 14), ("red_volume", 10, 14), ("flux", 13, 0), ("flux", 0, 0)])
@pytest.mark.parametrize("seed", ["theta", "rho_in", "rho_out"])
def test_tangent_through_the_zou_he_faces(obj, lo, hi, seed):
    """The derivative through the inlet and outlet faces (Appendix B) and the
    upstream phase of the outlet (Eq. 39), for objectives that include the face
    layers, against central differences of the oracle's own runs."""
    solid, phi0, kw = outlet_tube()
    steps = 20
    o = O.OracleSim(solid, **kw)
    J, dJ = o.tangent(phi0, objective=obj, n_steps=steps, seed=seed, axis=2, lo=lo, hi=hi)
    assert J == run(solid, phi0, kw, steps, obj, 2, lo, hi)
    base = {"theta": ("theta_deg", 60.0, (1e-2, 1e-3)), "rho_in": ("rho_in", 1.04, (1e-4, 1e-5)),
            "rho_out": ("rho_out", 1.0, (1e-4, 1e-5))}[seed]
    name, v0, hs = base
    f = lambda h: run(solid, phi0, kw, steps, obj, 2, lo, hi, **{name: v0 + h})
    errs = [abs(central(f, h) - dJ) / abs(dJ) for h in hs]
    assert errs[1] < 1e-6, errs


def test_rho_seeds_need_zou_he_faces():
    solid, phi0, kw = slug_2d()
    o = O.OracleSim(solid, **kw)
    with pytest.raises(Exception):
        o.tangent(phi0, objective="sat_nw", n_steps=2, seed="rho_in", axis=0, lo=0, hi=24)
