"""Seeded synthetic inputs: geometries and initial colour fields.

This module holds no arithmetic of the lattice Boltzmann method itself; it only
builds voxel images (1 = solid) and initial phase fields that both the GPU path
and the CPU oracle take as input.  Every array is returned in (nz, ny, nx)
order, x fastest in memory; 2D cases have nz = 1.

Workloads follow the paper's setups where the paper fixes them:
  * sessile drop on a wall (static contact-angle test, Sec. III.B),
  * circular capillary tube with an invading wetting fluid (Washburn tests,
    Sec. IV.A),
  * a porous rock with solid side walls and ten pure-fluid layers at both ends
    (Sec. IV.B).  The Bentheimer micro-CT image used there is not available, so
    a seeded Gaussian random field thresholded to the target porosity, with the
    connected pore cluster that spans inlet to outlet kept, stands in for it.
"""
from __future__ import annotations

import dataclasses
import functools
import os

import numpy as np

MASTER_SEED = 2407


@dataclasses.dataclass
class Case:
    """A geometry plus initial phase field."""

    solid: np.ndarray  # uint8 (nz, ny, nx), 1 = solid
    phi0: np.ndarray  # float64 (nz, ny, nx), +1 red, -1 blue
    periodic: tuple  # (px, py, pz)
    dim: int
    meta: dict

    @property
    def shape(self):
        return self.solid.shape


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def sessile_2d(nx=64, ny=32, radius=12.0, cx=32.0) -> Case:
    """D2Q9 sessile drop: solid rows y = 0 and y = ny-1, periodic in x, red
    half-disc of the given radius centred at (cx, 0.5) (the halfway wall), blue
    elsewhere."""
    solid = np.zeros((1, ny, nx), np.uint8)
    solid[0, 0, :] = 1
    solid[0, ny - 1, :] = 1
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    red = ((x - cx) ** 2 + (y - 0.5) ** 2 < radius**2) & (y >= 1) & (y <= ny - 2)
    phi = np.where(red, 1.0, -1.0)[None]
    return Case(solid, phi, (1, 0, 0), 2, dict(kind="sessile_2d", nx=nx, ny=ny, radius=radius, cx=cx))


def drop_periodic(shape, radius, dim=None) -> Case:
    """Free red drop of the given radius centred in a fully periodic box of
    blue fluid (Laplace-law test, Sec. III.A)."""
    if len(shape) == 2:
        shape = (1,) + tuple(shape)
    nz, ny, nx = shape
    dim = dim or (2 if nz == 1 else 3)
    zz, yy, xx = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    c = [(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0]
    r2 = (xx - c[0]) ** 2 + (yy - c[1]) ** 2
    if dim == 3:
        r2 = r2 + (zz - c[2]) ** 2
    phi = np.where(r2 < radius**2, 1.0, -1.0)
    solid = np.zeros(shape, np.uint8)
    per = (1, 1, 1) if dim == 3 else (1, 1, 0)
    return Case(solid, phi, per, dim, dict(kind="drop", radius=radius))


def channel_2d(nx=8, ny=18) -> Case:
    """Plane channel: solid rows y = 0 and y = ny-1, periodic in x, all red."""
    solid = np.zeros((1, ny, nx), np.uint8)
    solid[0, 0, :] = 1
    solid[0, ny - 1, :] = 1
    phi = np.ones((1, ny, nx))
    return Case(solid, phi, (1, 0, 0), 2, dict(kind="channel_2d"))


def channel_3d(nx=4, ny=12, nz=4) -> Case:
    """3D plane channel: solid planes y = 0 and y = ny-1, periodic in x and z."""
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    phi = np.ones((nz, ny, nx))
    return Case(solid, phi, (1, 0, 1), 3, dict(kind="channel_3d"))


def tube(nx=24, ny=24, nz=400, radius=10.0, wet_len=40, periodic_z=False) -> Case:
    """Circular capillary along z: fluid where (x-xc)^2 + (y-yc)^2 < r^2 with the
    axis at the box centre; wetting fluid b fills z < wet_len, non-wetting red
    the rest (Washburn setup, Sec. IV.A)."""
    zz, yy, xx = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    xc, yc = (nx - 1) / 2.0, (ny - 1) / 2.0
    fluid = (xx - xc) ** 2 + (yy - yc) ** 2 < radius**2
    solid = (~fluid).astype(np.uint8)
    phi = np.where(zz < wet_len, -1.0, 1.0)
    return Case(solid, phi, (0, 0, 1 if periodic_z else 0), 3,
                dict(kind="tube", radius=radius, wet_len=wet_len))


def sessile_box(nx, ny, nz, radius) -> Case:
    """Channel with solid planes y = 0 and y = ny-1, periodic in x and z, a red
    hemisphere of the given radius on the floor at the centre of the x-z
    plane, blue elsewhere (static contact-angle setup of Sec. III.B, whose
    domain is 102 lattice points between the plates and 201 x 201 along
    them)."""
    zz, yy, xx = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    cx, cz = nx / 2.0, nz / 2.0
    red = ((xx - cx) ** 2 + (yy - 0.5) ** 2 + (zz - cz) ** 2 < radius**2) & (yy >= 1) & (yy <= ny - 2)
    phi = np.where(red, 1.0, -1.0)
    return Case(solid, phi, (1, 0, 1), 3, dict(kind="sessile_box", radius=radius))


def sessile_3d(edge=64, radius=None) -> Case:
    """Cubic box with solid planes y = 0 and y = edge-1, periodic in x and z, a
    red hemisphere of radius 0.25*edge on the floor at the box centre."""
    radius = 0.25 * edge if radius is None else radius
    n = edge
    zz, yy, xx = np.mgrid[0:n, 0:n, 0:n].astype(np.float64)
    solid = np.zeros((n, n, n), np.uint8)
    solid[:, 0, :] = 1
    solid[:, n - 1, :] = 1
    c = n / 2.0
    red = ((xx - c) ** 2 + (yy - 0.5) ** 2 + (zz - c) ** 2 < radius**2) & (yy >= 1) & (yy <= n - 2)
    phi = np.where(red, 1.0, -1.0)
    return Case(solid, phi, (1, 0, 1), 3, dict(kind="sessile_3d", edge=edge, radius=radius))


def _gaussian_field(n: int, corr: float, seed: int) -> np.ndarray:
    """Periodic Gaussian random field: white noise filtered in Fourier space by a
    Gaussian kernel of standard deviation corr/sqrt(2), i.e. covariance
    exp(-r^2 / (2 corr^2))."""
    rng = _rng(seed)
    noise = rng.standard_normal((n, n, n))
    k = np.fft.fftfreq(n) * 2.0 * np.pi
    kr = np.fft.rfftfreq(n) * 2.0 * np.pi
    s = corr / np.sqrt(2.0)
    kz, ky, kx = np.meshgrid(k, k, kr, indexing="ij")
    filt = np.exp(-0.5 * s * s * (kx * kx + ky * ky + kz * kz))
    field = np.fft.irfftn(np.fft.rfftn(noise) * filt, s=(n, n, n), axes=(0, 1, 2))
    return field


def _spanning_fluid(fluid: np.ndarray, buffer: int) -> np.ndarray:
    """Keep the 6-connected fluid component(s) that touch both buffer slabs."""
    from scipy import ndimage

    lab, _ = ndimage.label(fluid)
    nz = fluid.shape[0]
    lo = np.unique(lab[:buffer][fluid[:buffer]])
    hi = np.unique(lab[nz - buffer:][fluid[nz - buffer:]])
    keep = np.intersect1d(lo, hi)
    keep = keep[keep > 0]
    return np.isin(lab, keep)


def grf_rock(n=256, corr=8.0, porosity=0.22, seed=MASTER_SEED, buffer=10, tol=0.002,
             nz=None) -> Case:
    """Synthetic rock: seeded Gaussian random field (correlation length `corr`),
    pore = field above a threshold, rock region z in [buffer, nz-buffer),
    `buffer` pure-fluid layers at both ends, 1-voxel solid walls on the x and y
    faces, only the pore cluster spanning both buffers kept, threshold adjusted
    until the rock-region porosity is within `tol` of the target.  Initially
    wetting-saturated (phi = -1)."""
    nz = n if nz is None else nz
    cache = _cache_path("rock", n, nz, corr, porosity, seed, buffer)
    if cache and os.path.exists(cache):
        solid = np.load(cache)
    else:
        solid = _grf_rock_solid(n, nz, corr, porosity, seed, buffer, tol)
        if cache:
            try:
                np.save(cache, solid)
            except OSError:
                pass
    phi = -np.ones(solid.shape)
    rock = solid[buffer:nz - buffer, 1:-1, 1:-1]
    por = 1.0 - rock.mean()
    return Case(solid, phi, (0, 0, 0), 3,
                dict(kind="grf_rock", n=n, nz=nz, corr=corr, porosity=float(por), seed=seed, buffer=buffer))


def _cache_path(*key):
    d = os.environ.get("CGLBM_CACHE", os.path.join(os.environ.get("TMPDIR", "/tmp"), "cglbm_inputs"))
    try:
        os.makedirs(d, exist_ok=True)
    except OSError:
        return None
    return os.path.join(d, "_".join(str(k) for k in key) + ".npy")


def _grf_rock_solid(n, nz, corr, porosity, seed, buffer, tol):
    m = max(n, nz)
    field = _gaussian_field(m, corr, seed)[:nz, :n, :n]
    interior = field[buffer:nz - buffer, 1:n - 1, 1:n - 1]
    flat = np.sort(interior.ravel())

    def build(raw_por):
        thr = flat[min(len(flat) - 1, max(0, int(round((1.0 - raw_por) * len(flat)))))]
        fluid = np.zeros((nz, n, n), bool)
        fluid[buffer:nz - buffer, 1:n - 1, 1:n - 1] = interior > thr
        fluid[:buffer, 1:n - 1, 1:n - 1] = True
        fluid[nz - buffer:, 1:n - 1, 1:n - 1] = True
        fluid = _spanning_fluid(fluid, buffer)
        por = fluid[buffer:nz - buffer, 1:n - 1, 1:n - 1].mean()
        return fluid, por

    lo, hi = porosity, min(0.95, porosity + 0.3)
    raw = porosity
    fluid, por = build(raw)
    for _ in range(40):
        if abs(por - porosity) <= tol:
            break
        if por < porosity:
            lo = raw
        else:
            hi = raw
        raw = 0.5 * (lo + hi)
        fluid, por = build(raw)
    return (~fluid).astype(np.uint8)


def drainage_rock(n=128, corr=8.0, porosity=0.22, seed=MASTER_SEED, buffer=10, theta=40.0, nz=None):
    """Body-force drainage through the synthetic rock (the adjoint workload):
    the rock of grf_rock with the z axis periodic (the two ten-layer buffers
    meet), non-wetting red in the inlet buffer z < buffer and wetting blue
    elsewhere, and a per-voxel contact-angle field that is `theta` degrees on
    every solid voxel.  Returns (case, theta_field)."""
    c = grf_rock(n=n, corr=corr, porosity=porosity, seed=seed, buffer=buffer, nz=nz)
    nzz = c.solid.shape[0]
    zz = np.arange(nzz)[:, None, None] * np.ones(c.solid.shape)
    phi = np.where(zz < buffer, 1.0, -1.0)
    theta_field = np.where(c.solid == 1, float(theta), 0.0)
    meta = dict(c.meta, kind="drainage_rock", theta=float(theta))
    return Case(c.solid, phi, (0, 0, 1), 3, meta), theta_field


@functools.lru_cache(maxsize=None)
def contact_angles(count=64, seed=MASTER_SEED):
    """Per-run contact angles of the batched sweep: theta_k ~ U[15, 165] deg
    drawn from seed + k."""
    return tuple(float(_rng(seed + k).uniform(15.0, 165.0)) for k in range(count))


def sweep_edges(count=64, seed=MASTER_SEED):
    """Per-run cubic box edges of the batched sweep, drawn from {48, 64, 96, 128}."""
    choices = np.array([48, 64, 96, 128])
    return tuple(int(choices[_rng(seed + 1000 + k).integers(0, 4)]) for k in range(count))


def random_state_perturbation(shape, q, seed, scale=1e-3):
    """Small seeded perturbation field (q, *shape) for parity tests that start
    away from rest."""
    return scale * _rng(seed).standard_normal((q,) + tuple(shape))
