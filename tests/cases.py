"""Shared case definitions for the parity tests: the same seeded input and the
same parameters handed to the GPU run (paper_2407_10914_amd.sim.Sim) and to
the CPU oracle (oracle.OracleSim)."""
import numpy as np

from paper_2407_10914_amd import inputs


def c1_sessile_2d():
    c = inputs.sessile_2d()
    kw = dict(dim=2, periodic=c.periodic, tau_r=1.0, tau_b=1.0, sigma=0.005, beta=0.7, scheme=1, theta_deg=60.0,
              collision=0)
    return c, kw


def c2_tube(scheme=1, theta=45.0, drive="type1", nz=400, radius=10.0, wet_len=40, beta=0.95):
    c = inputs.tube(nz=nz, radius=radius, wet_len=wet_len)
    kw = dict(dim=3, periodic=c.periodic, tau_r=1.0, tau_b=1.0, sigma=1.0 / 45.0, beta=beta, scheme=scheme,
              theta_deg=theta, bc=1, zeta_r=0.0, collision=1)
    if drive == "type1":
        kw.update(rho_in=1.01, rho_out=1.0)
    elif drive == "type2":
        kw.update(rho_in=1.0, rho_out=1.0, g=(0.0, 0.0, 0.01 / (3.0 * (nz - 1))))
    else:
        kw.update(rho_in=1.0, rho_out=1.0)
    return c, kw


def drop_3d(n=20, R=6.0, tau_r=1.0, tau_b=0.6, sigma=0.02, beta=0.95):
    c = inputs.drop_periodic((n, n, n), R)
    kw = dict(dim=3, periodic=c.periodic, tau_r=tau_r, tau_b=tau_b, sigma=sigma, beta=beta, collision=1)
    return c, kw


def rock(n=48, nz=None, seed=2409, buffer=4, theta=30.0, drive="type1", scheme=1):
    c = inputs.grf_rock(n=n, nz=nz, corr=4.0, porosity=0.22, seed=seed, buffer=buffer)
    kw = dict(dim=3, periodic=c.periodic, tau_r=1.0, tau_b=0.6, sigma=0.01, beta=0.95, scheme=scheme,
              theta_deg=theta, bc=1, zeta_r=1.0, collision=1)
    if drive == "type1":
        kw.update(rho_in=1.02, rho_out=1.0)
    else:
        kw.update(rho_in=1.0, rho_out=1.0, g=(0.0, 0.0, 1e-5))
    return c, kw


def rel(a, b, mask=None):
    """||a - b||_2 / ||b||_2 over the mask (fluid nodes)."""
    a = np.asarray(a)
    b = np.asarray(b)
    if mask is not None:
        if a.ndim > mask.ndim:
            a = a[..., mask] if a.shape[-mask.ndim:] == mask.shape else a
            b = b[..., mask] if b.shape[-mask.ndim:] == mask.shape else b
        else:
            a, b = a[mask], b[mask]
    den = np.linalg.norm(b.ravel())
    num = np.linalg.norm((a - b).ravel())
    return num / den if den > 0 else num


def sessile_3d(edge, theta, scheme, sigma=1.0 / 45.0, beta=0.95):
    c = inputs.sessile_3d(edge=edge)
    kw = dict(dim=3, periodic=c.periodic, tau_r=1.0, tau_b=1.0, sigma=sigma, beta=beta, scheme=scheme,
              theta_deg=theta, collision=1)
    return c, kw


def outlet_slug(nz=40, radius=6.0, slug=(24, 34), scheme=2, theta=70.0, drho=0.05, zeta_r=0.0, n=16):
    """A red slug in a blue-filled tube, pushed out through the Zou-He outlet
    by a Type-I pressure difference: the outlet plane holds mixed phase
    (chi^s strictly between 0 and 1, Eqs. B.12-B.18 with Eq. 39) for a few
    hundred steps from about step 300."""
    c = inputs.tube(nx=n, ny=n, nz=nz, radius=radius, wet_len=8)
    z = np.arange(nz)[:, None, None]
    c.phi0 = np.where((z >= slug[0]) & (z < slug[1]), 1.0, -1.0) * np.ones_like(c.phi0)
    kw = dict(dim=3, periodic=c.periodic, tau_r=1.0, tau_b=1.0, sigma=1.0 / 45.0, beta=0.95, scheme=scheme,
              theta_deg=theta, bc=1, rho_in=1.0 + drho, rho_out=1.0, zeta_r=zeta_r, collision=1)
    return c, kw
