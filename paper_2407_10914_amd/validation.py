"""The paper's validation setups, run on the device (Secs. III.A, III.B, IV.A).

* Laplace law (Sec. III.A): red drops of several radii in a fully periodic
  128^3 box of blue fluid, tau_r = 1.0, tau_b = 0.6 (viscosity ratio 5),
  sigma = 1/45.  At steady state the pressure jump across each drop (mean
  rho/3 over phi > 0.9 minus over phi < -0.9, Eq. 23) is plotted against 2/R
  (R from the red volume); the slope of the least-squares line is the
  simulated interfacial tension, compared with the input (the paper: 0.45 %).
* Static contact angle (Sec. III.B): a red drop of radius 30 on the lower
  plate of a channel 201 x 102 x 201 (plates at y = 0 and y = 101, periodic
  along x and z), same fluids; after relaxation the angle is read from the
  drop's base and height (Eqs. 45-46) on the two vertical mid-planes, by
  the device (cg_lbm_drop_shape), and compared with the input angle through
  fluid b, for Scheme-I and Scheme-II.
* Capillary filling (Sec. IV.A): a tube of radius 5 in a 12 x 12 x 101 box,
  wetting fluid b (tau_b = 1.0) displacing the non-wetting fluid r
  (tau_r = 0.6, viscosity ratio M = 1/5), sigma = 1/45, b injected at the
  inlet with equal pressures (Case-I, spontaneous imbibition at theta < 90)
  or at theta = 90 with a pressure difference by Type-I Zou-He densities or
  the Type-II body force (Case-II).  The interface starts from a pre-run at
  neutral wetting (b in the first layers); the tip position on the axis is
  compared with Washburn's law, Eq. (48) (Eq. 49 in the scaled variables of
  Eqs. 50-51), shifted in time so that it starts at the measured initial
  position, by the area error of the paper: |int z_lbm dt - int z dt| /
  int z dt.

The sweeps of one setup run together as one batch (cg_batch_*).  The host
only sets up, schedules and fits; every field value comes from device
reductions.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

# ------------------------------------------------------------ closed forms


def washburn_z(t, *, L, r, mu_w, mu_nw, dP, gamma, theta_deg):
    """Tip position z(t) of a wetting fluid filling a tube of length L and
    radius r from z = 0 at t = 0 (Eq. 48; Eq. 47 solved for z).  mu_w, mu_nw:
    dynamic viscosities of the wetting (invading) and non-wetting fluids;
    dP: inlet minus outlet pressure; gamma: interfacial tension.  For
    mu_w = mu_nw Eq. 47 is linear in z."""
    t = np.asarray(t, dtype=np.float64)
    drive = (r * r / 8.0) * (dP + 2.0 * gamma * math.cos(math.radians(theta_deg)) / r)
    dm = mu_w - mu_nw
    if dm == 0.0:
        return drive * t / (mu_nw * L)
    a = L * mu_nw / dm
    return -a + np.sqrt(a * a + (dP * r * r / 2.0 + r * gamma * math.cos(math.radians(theta_deg))) * t / (2.0 * dm))


def washburn_time(z, *, L, r, mu_w, mu_nw, dP, gamma, theta_deg):
    """Time at which Eq. (47) puts the tip at z (the inverse of washburn_z)."""
    drive = (r * r / 8.0) * (dP + 2.0 * gamma * math.cos(math.radians(theta_deg)) / r)
    return (z * z * (mu_w - mu_nw) / 2.0 + mu_nw * L * z) / drive


def washburn_scaled(t_star, *, r_over_L, mu_w, mu_nw, dP_r2_over_2Lgamma, theta_deg):
    """Eq. (49): z* = z/L as a function of t* = gamma t / ((mu_w - mu_nw) L)
    (Eqs. 50-51), for mu_w != mu_nw."""
    a = mu_nw / (mu_w - mu_nw)
    return -a + np.sqrt(a * a + 0.5 * (dP_r2_over_2Lgamma + r_over_L * math.cos(math.radians(theta_deg)))
                        * np.asarray(t_star, dtype=np.float64))


def area_error(t, z_sim, z_ref):
    """Relative difference of the areas under two curves on the same times
    (the error measure of Sec. IV.A), trapezoidal rule."""
    t = np.asarray(t, dtype=np.float64)
    a = np.trapezoid(np.asarray(z_sim, dtype=np.float64), t)
    b = np.trapezoid(np.asarray(z_ref, dtype=np.float64), t)
    return abs(a - b) / abs(b)


def laplace_fit(dp, radius):
    """Least-squares line dp = s * (2/R) + c (3D Laplace law): returns the
    slope s (the simulated interfacial tension) and the intercept c."""
    x = 2.0 / np.asarray(radius, dtype=np.float64)
    y = np.asarray(dp, dtype=np.float64)
    A = np.vstack([x, np.ones_like(x)]).T
    (s, c), *_ = np.linalg.lstsq(A, y, rcond=None)
    return float(s), float(c)


def drop_radius_from_volume(vol):
    """Radius of the sphere of the given volume."""
    return (3.0 * vol / (4.0 * math.pi)) ** (1.0 / 3.0)


# ---------------------------------------------------------- device runs


def _batch(sims):
    from .sim import Batch

    return Batch(sims)


def laplace_sweep(n=128, radii=(10.0, 14.0, 18.0, 22.0, 26.0, 30.0), steps=40000, sigma=1.0 / 45.0, tau_r=1.0,
                  tau_b=0.6, beta=0.95, precision="f32", log=None):
    # 40000 steps: the largest drop relaxes on the viscous time R^2/nu, about
    # 27000 steps at R = 30 (at 10000 its pressure jump is still moving)
    from . import inputs
    from .sim import Sim

    sims = []
    for R in radii:
        c = inputs.drop_periodic((n, n, n), R)
        s = Sim(c.solid, dim=3, periodic=c.periodic, tau_r=tau_r, tau_b=tau_b, sigma=sigma, beta=beta,
                collision=1, precision=precision)
        s.set_phase(c.phi0)
        sims.append(s)
    b = _batch(sims)
    hist = []
    done = 0
    for frac in (0.8, 1.0):
        b.step(int(steps * frac) - done)
        done = int(steps * frac)
        b.sync()
        hist.append([s.observe() for s in sims])
    rows = []
    for R0, o_prev, o in zip(radii, hist[0], hist[1]):
        R = drop_radius_from_volume(o["vol_r"])
        dp = o["p_in"] - o["p_out"]
        dp_prev = o_prev["p_in"] - o_prev["p_out"]
        rows.append(dict(R0=R0, R=R, dp=dp, sigma_drop=dp * R / 2.0, dp_change_last_20pct=abs(dp - dp_prev) / abs(dp),
                         u_max=o["u_max"]))
        if log:
            log(f"laplace R0 {R0:.0f}: R {R:.3f} dp {dp:.6e} sigma_drop {dp * R / 2:.6e}")
    s_fit, c_fit = laplace_fit([r["dp"] for r in rows], [r["R"] for r in rows])
    return dict(setup=f"{n}^3 periodic, tau_r {tau_r} tau_b {tau_b}, sigma {sigma:.6g}, beta {beta}, {steps} steps, "
                      f"{precision}", sigma_input=sigma, sigma_fit=s_fit, intercept=c_fit,
                error_pct=abs(s_fit - sigma) / sigma * 100.0, drops=rows)


def angle_sweep(thetas=(30.0, 45.0, 60.0, 75.0, 90.0, 105.0, 120.0, 135.0, 150.0), schemes=(1, 2),
                shape=(201, 102, 201), radius=30.0, steps=20000, sigma=1.0 / 45.0, tau_r=1.0, tau_b=0.6,
                beta=0.95, precision="f32", log=None):
    from . import inputs
    from .sim import Sim

    nx, ny, nz = shape
    out = []
    for scheme in schemes:
        sims = []
        for th in thetas:
            c = inputs.sessile_box(nx, ny, nz, radius)
            s = Sim(c.solid, dim=3, periodic=c.periodic, tau_r=tau_r, tau_b=tau_b, sigma=sigma, beta=beta,
                    scheme=scheme, theta_deg=th, collision=1, precision=precision)
            s.set_phase(c.phi0)
            sims.append(s)
        b = _batch(sims)
        chunk = 5000
        for k in range(0, steps, chunk):
            b.step(min(chunk, steps - k))
            b.sync()
            if log:
                log(f"angle scheme {scheme}: {min(steps, k + chunk)} of {steps} steps")
        for th, s in zip(thetas, sims):
            d1 = s.drop_shape(base_axis=0, wall_axis=1, slice=nz // 2, wall=0.5, row=1)
            d2 = s.drop_shape(base_axis=2, wall_axis=1, slice=nx // 2, wall=0.5, row=1)
            sim_b = 180.0 - 0.5 * (d1["theta_deg"] + d2["theta_deg"])
            out.append(dict(scheme=scheme, theta_input=th, theta_sim=sim_b, error=th - sim_b,
                            base=[d1["base"], d2["base"]], height=[d1["height"], d2["height"]]))
            if log:
                log(f"angle scheme {scheme} theta {th:.0f}: simulated {sim_b:.2f} (error {th - sim_b:+.2f})")
        del b
        del sims
    return dict(setup=f"channel {nx}x{ny}x{nz}, plates at y = 0 and {ny - 1}, drop radius {radius}, tau_r {tau_r} "
                      f"tau_b {tau_b}, sigma {sigma:.6g}, {steps} steps, {precision}", runs=out)


def _tube_front(s, nx, ny):
    """Mean first phi = 0 crossing along z on the four grid lines around the
    tube axis (the axis of an even box lies between grid lines)."""
    xs = []
    for x in (nx // 2 - 1, nx // 2):
        for y in (ny // 2 - 1, ny // 2):
            c = s.line_crossings(2, (x, y, 0), max_points=1)
            if c:
                xs.append(c[0])
    return float(np.mean(xs)) if xs else float("nan")


def washburn_runs(cases=None, shape=(12, 12, 101), radius=5.0, sigma=1.0 / 45.0, tau_w=1.0, tau_nw=0.6,
                  beta=0.95, pre_steps=4000, max_steps=300000, every=500, z_stop=0.9, precision="f32",
                  log=None):
    """Case-I / Case-II capillary filling.  cases: list of dicts with keys
    scheme, theta, drive ("none", "type1", "type2") and dP (lattice pressure
    difference)."""
    from . import inputs
    from .sim import Sim
    from .units import lattice_viscosity

    nx, ny, nz = shape
    L = nz - 1
    if cases is None:
        cases = [dict(scheme=s, theta=t, drive="none", dP=0.0) for s in (1, 2) for t in (30.0, 45.0, 60.0, 75.0)]
        cases += [dict(scheme=2, theta=90.0, drive=d, dP=p) for d in ("type1", "type2") for p in (0.004, 0.008)]
    sims = []
    for cs in cases:
        c = inputs.tube(nx=nx, ny=ny, nz=nz, radius=radius, wet_len=2)
        kw = dict(dim=3, periodic=c.periodic, tau_r=tau_nw, tau_b=tau_w, sigma=sigma, beta=beta,
                  scheme=cs["scheme"], theta_deg=90.0, bc=1, rho_in=1.0, rho_out=1.0, zeta_r=0.0, collision=1)
        s = Sim(c.solid, precision=precision, **kw)
        s.set_phase(c.phi0)
        sims.append(s)
    # pre-run at neutral wetting and equal pressures: a settled meniscus near
    # the inlet (the initial state of Sec. IV.A)
    b = _batch(sims)
    b.step(pre_steps)
    b.sync()
    for cs, s in zip(cases, sims):
        # the run's own angle and drive from now on
        s.set_wetting(cs["theta"])
        if cs["drive"] == "type1":
            s.set_pressure(1.0 + 3.0 * cs["dP"], 1.0)
        elif cs["drive"] == "type2":
            s.set_body_force((0.0, 0.0, cs["dP"] / L))
    z0 = [_tube_front(s, nx, ny) for s in sims]
    t0 = sims[0].time
    series = [[(0, z)] for z in z0]
    active = [True] * len(sims)
    while any(active) and sims[0].time - t0 < max_steps:
        b.step(every)
        b.sync()
        for k, s in enumerate(sims):
            if not active[k]:
                continue
            z = _tube_front(s, nx, ny)
            series[k].append((s.time - t0, z))
            if not (z < z_stop * L):
                active[k] = False
    mu_w, mu_nw = lattice_viscosity(tau_w), lattice_viscosity(tau_nw)
    out = []
    for cs, ser in zip(cases, series):
        t = np.array([p[0] for p in ser], dtype=np.float64)
        z = np.array([p[1] for p in ser], dtype=np.float64)
        ok = np.isfinite(z)
        t, z = t[ok], z[ok]
        kw = dict(L=L, r=radius, mu_w=mu_w, mu_nw=mu_nw, dP=cs["dP"], gamma=sigma, theta_deg=cs["theta"])
        tshift = washburn_time(z[0], **kw)
        za = washburn_z(t + tshift, **kw)
        err = area_error(t, z, za)
        rec = dict(cs, z_init=float(z[0]), z_init_star=float(z[0] / L), t_end=float(t[-1]), z_end=float(z[-1]),
                   area_error_pct=100.0 * err, points=int(len(t)))
        out.append(rec)
        if log:
            log(f"washburn {cs}: z0 {z[0]:.2f} -> {z[-1]:.2f} in {t[-1]:.0f} steps, area error {100 * err:.2f} %")
    return dict(setup=f"tube radius {radius} in {nx}x{ny}x{nz}, tau_w {tau_w} tau_nw {tau_nw} (M = "
                      f"{mu_nw / mu_w:.3g}), sigma {sigma:.6g}, pre-run {pre_steps} steps at 90 deg, {precision}",
                mu_w=mu_w, mu_nw=mu_nw, L=L, runs=out)


def main(argv=None):
    ap = argparse.ArgumentParser(description="the paper's validation setups on the device")
    ap.add_argument("which", choices=("laplace", "angle", "washburn", "all"))
    ap.add_argument("--json", default=None)
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--steps", type=int, default=None,
                    help="steps of the Laplace and contact-angle runs (default 40000 and 20000)")
    ap.add_argument("--schemes", default=None,
                    help="wetting schemes of the contact-angle sweep, e.g. 1,2,3 (3: fictitious density, Eq. 24)")
    a = ap.parse_args(argv)
    extra = {} if a.steps is None else {"steps": a.steps}
    angle_extra = dict(extra)
    if a.schemes:
        angle_extra["schemes"] = tuple(int(x) for x in a.schemes.split(","))
    import torch

    torch.cuda.set_device(0)
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    res = {}
    for w in (("laplace", "angle", "washburn") if a.which == "all" else (a.which,)):
        t0 = time.perf_counter()
        if w == "laplace":
            res[w] = laplace_sweep(precision=a.precision, log=log, **extra)
        elif w == "angle":
            res[w] = angle_sweep(precision=a.precision, log=log, **angle_extra)
        else:
            res[w] = washburn_runs(precision=a.precision, log=log)
        res[w]["wall_s"] = round(time.perf_counter() - t0, 1)
        torch.cuda.empty_cache()
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
