"""Degenerate geometries and rejected inputs on the GPU path.

Degenerate cases of the method: a fluid node with no fluid neighbour (every
link bounces back, every stencil neighbour is a solid boundary point), a
channel one voxel wide, and a two-node slit; each runs in FP64 against the
oracle (1e-12, the bar of the double build) and conserves the colour masses.
Geometries the method cannot take are rejected by cg_lbm_create with a
message (these checks need the device to be selected first, hence the GPU
mark)."""
import numpy as np
import pytest

import oracle as O
from cases import rel

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _pair(solid, phi0, kw, steps):
    from paper_2407_10914_amd.sim import Sim

    g = Sim(solid, precision="f64", **kw)
    g.set_phase(phi0)
    o = O.OracleSim(solid, **kw)
    o.set_phase(phi0)
    a = g.observe()
    g.step(steps)
    o.step(steps)
    b = g.observe()
    fluid = solid == 0
    om = o.macro()
    for k in ("rho_r", "rho_b", "u"):
        e = rel(g.field(k), om[k], fluid)
        assert e <= TOL64, (k, e)
    for k in ("mass_r", "mass_b"):
        assert abs(b[k] - a[k]) <= 1e-12 * max(1.0, abs(a[k])), (k, a[k], b[k])
    return g, o


def _kw(**extra):
    kw = dict(dim=3, periodic=(1, 1, 1), tau_r=1.0, tau_b=0.6, sigma=0.02, beta=0.9, scheme=1, theta_deg=60.0,
              collision=1)
    kw.update(extra)
    return kw


@pytest.mark.parametrize("scheme", [1, 2])
def test_isolated_fluid_node(scheme):
    solid = np.ones((5, 5, 5), dtype=np.uint8)
    solid[2, 2, 2] = 0
    phi0 = np.zeros(solid.shape)
    phi0[2, 2, 2] = 0.3
    _pair(solid, phi0, _kw(scheme=scheme, g=(1e-4, 0.0, 0.0)), 30)


def test_channel_one_voxel_wide_with_body_force():
    solid = np.ones((3, 3, 32), dtype=np.uint8)
    solid[1, 1, :] = 0
    phi0 = np.where(np.arange(32) < 16, 1.0, -1.0)[None, None, :] * np.ones(solid.shape)
    _pair(solid, phi0, _kw(g=(1e-5, 0.0, 0.0)), 60)


def test_two_node_slit():
    solid = np.ones((4, 16, 16), dtype=np.uint8)
    solid[1:3, :, :] = 0
    yy, xx = np.meshgrid(np.arange(16), np.arange(16), indexing="ij")
    phi0 = np.where((xx - 8) ** 2 + (yy - 8) ** 2 < 16, 1.0, -1.0)[None] * np.ones(solid.shape)
    _pair(solid, phi0, _kw(scheme=2, theta_deg=120.0), 60)


@pytest.mark.parametrize("what, words", [
    ("all_solid", "no fluid voxel"),
    ("wall_face", "neither periodic nor open"),
    ("outlet", "upstream"),
])
def test_create_rejects_geometries_the_method_cannot_take(what, words):
    from paper_2407_10914_amd.lib import CgError
    from paper_2407_10914_amd.sim import Sim

    kw = _kw()
    solid = np.zeros((6, 6, 6), dtype=np.uint8)
    if what == "all_solid":
        solid[:] = 1
    elif what == "wall_face":
        kw["periodic"] = (0, 1, 1)  # fluid on the x faces, which are walls
    else:
        solid[:, 0, :] = 1
        solid[:, -1, :] = 1
        solid[:, :, 0] = 1
        solid[:, :, -1] = 1
        solid[-2, 2, 2] = 1  # outlet voxel (2, 2) has a solid voxel upstream
        kw.update(periodic=(0, 0, 0), bc=1, rho_in=1.01, rho_out=1.0)
    with pytest.raises(CgError, match=words):
        Sim(solid, precision="f32", **kw)


def _sphere_pack(n, period=32, radius=11):
    x = np.arange(n, dtype=np.int32)
    d = ((x % period) - period // 2) ** 2
    return (d[:, None, None] + d[None, :, None] + d[None, None, :] < radius**2).astype(np.uint8)


def test_largest_lattice_below_the_index_limit():
    """512^3 voxels, 111.7 M fluid nodes (a periodic packing of spheres, FP32
    MRT, Scheme-I, body force): fluid nodes times Q lies just below 2^31, the
    16-byte normal grid spans 2^31 bytes, and the device holds about 54 GB.
    The run keeps both colour masses to 1e-6 over 50 steps with a finite
    state, reading a pull table that mixes 8-bit waves and fallback waves.
    512^3 = 2^27 voxels is also the largest box (the per-node word holds a
    27-bit voxel index): cg_lbm_create refuses 528^3, and 512^3 with smaller
    spheres (more than 2^31 / 19 fluid nodes)."""
    from paper_2407_10914_amd.sim import Sim

    kw = dict(dim=3, periodic=(1, 1, 1), tau_r=1.0, tau_b=0.6, sigma=0.01, beta=0.95, scheme=1, theta_deg=60.0,
              g=(0.0, 0.0, 1e-5), precision="f32", collision="mrt")
    for geom, words in ((_sphere_pack(528, period=48, radius=10), "2^27 voxels"),
                        (_sphere_pack(512, radius=8), "32-bit")):
        with pytest.raises(Exception) as e:
            Sim(geom, **kw)
        print(str(e.value), flush=True)
        assert words in str(e.value)
    del geom
    n = 512
    solid = _sphere_pack(n)
    x = np.arange(n)
    phi = np.where((x[:, None, None] < 64) & (solid == 0), 1.0, -1.0)
    s = Sim(solid, **kw)
    inf = s.info()
    print({k: inf[k] for k in ("fluid", "state_bytes", "device_bytes", "pull_waves", "pull_waves_8bit")}, flush=True)
    assert inf["fluid"] * 19 < 2**31 and inf["fluid"] > 100_000_000
    assert 0 < inf["pull_waves_8bit"] < inf["pull_waves"]
    s.set_phase(phi)
    a = s.observe()
    s.step(50)
    b = s.observe()
    assert b["nan_count"] == 0
    for k in ("mass_r", "mass_b"):
        assert abs(b[k] / a[k] - 1.0) < 1e-6, (k, a[k], b[k])
