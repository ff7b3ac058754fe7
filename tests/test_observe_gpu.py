"""Observables on the device against the oracle and against the host-side
measurement of an exported field.

* Interface points along grid lines (the phi = 0 crossings that Sec. III.B
  reads the drop's base and height from, and the tube front of Sec. IV.A):
  the device scan gives exactly what measure.crossings gives on the exported
  phase field, and on an FP64 run exactly what it gives on the oracle's field.
* The sessile-drop shape of Eqs. (45)-(46) from the device equals
  measure.drop_base_height on the same field.
* Flux per colour, mass saturation and the other reductions against the
  oracle; a non-finite population makes cg_lbm_observe fail with
  CG_EUNSTABLE.
"""
import numpy as np
import pytest

from cases import c1_sessile_2d, c2_tube, sessile_3d
from parity_helpers import gpu, orc, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_line_crossings_equal_the_host_scan_of_the_exported_field(precision):
    from paper_2407_10914_amd import measure

    case, kw = sessile_3d(32, 60.0, 2)
    g = gpu(case, kw, precision)
    g.step(400)
    ph = g.field("phi")  # (z, y, x)
    nz, ny, nx = ph.shape
    checked = 0
    for z in (nz // 2, nz // 2 + 3):
        for y in (1, 4, 8):
            got = g.line_crossings(0, (0, y, z))
            want = measure.crossings(ph[z, y, :])
            assert got == want, (z, y, got, want)
            checked += len(want)
        for x in (nx // 2, nx // 2 - 2):
            got = g.line_crossings(1, (x, 0, z), lo=1)
            want = measure.crossings(ph[z, 1:, x], np.arange(1, ny))
            assert got == want
            # a line between two columns
            got = g.line_crossings(1, (x, 0, z), lo=1, blend=0.3, blend_axis=0)
            col = 0.7 * ph[z, 1:, x] + 0.3 * ph[z, 1:, x + 1]
            want = measure.crossings(col, np.arange(1, ny))
            assert got == want
            checked += len(want)
    assert checked >= 10
    # at most max_points come back, the count is still total
    assert len(g.line_crossings(0, (0, 1, nz // 2), max_points=1)) == 1


def test_drop_shape_and_front_from_the_device():
    from paper_2407_10914_amd import measure

    case, kw = c1_sessile_2d()
    g = gpu(case, kw, "f64")
    o = orc(case, kw)
    g.step(2000)
    o.step(2000)
    d = g.drop_shape(base_axis=0, wall_axis=1, wall=0.5, row=1)
    b, h = measure.drop_base_height(g.field("phi")[0], wall=0.5, row=1)
    ob, oh = measure.drop_base_height(o.macro()["phi"][0], wall=0.5, row=1)
    say("C1 drop (device):", d, "host:", b, h, "oracle:", ob, oh)
    assert d["base"] == b == ob and d["height"] == h == oh
    assert abs(d["theta_deg"] - measure.cap_angle(b, h)) < 1e-12
    # 3D drop, slice through its centre
    case, kw = sessile_3d(32, 120.0, 2)
    g = gpu(case, kw, "f32")
    g.step(600)
    z = case.solid.shape[0] // 2
    d = g.drop_shape(0, 1, slice=z)
    b, h = measure.drop_base_height(g.field("phi")[z], wall=0.5, row=1)
    assert d["base"] == b and d["height"] == h
    # front on the axis of a tube
    case, kw = c2_tube(scheme=1, theta=45.0, drive="type1", nz=40, radius=6.0, wet_len=12)
    g = gpu(case, kw, "f64")
    g.step(200)
    ph = g.field("phi")
    at = (case.solid.shape[2] // 2, case.solid.shape[1] // 2, 0)
    assert g.front(2, at) == measure.front_on_axis(ph, axis=0, line=(at[1], at[0]))


def test_line_queries_outside_the_box_are_refused():
    from paper_2407_10914_amd.lib import CgError

    case, kw = c1_sessile_2d()
    g = gpu(case, kw, "f64")
    for bad in (dict(axis=2, at=(0, 0, 0)), dict(axis=0, at=(0, 99, 0)), dict(axis=0, at=(0, 1, 0), hi=1000),
                dict(axis=1, at=(63, 0, 0), blend=0.5, blend_axis=0), dict(axis=0, at=(0, 1, 0), blend=1.0)):
        with pytest.raises(CgError):
            g.line_crossings(**bad)
    with pytest.raises(CgError):
        g.drop_shape(0, 1, row=20)  # no drop on that row


def test_flux_per_colour_and_saturations_against_the_oracle():
    case, kw = c2_tube(scheme=2, theta=45.0, drive="type1", nz=40, radius=6.0, wet_len=12)
    kw = dict(kw, zeta_r=0.25)
    g = gpu(case, kw, "f64")
    o = orc(case, kw)
    g.step(150)
    o.step(150)
    for plane in (0, 11, 20, 39):
        a, b = g.observe(axis=2, plane=plane), o.observe(axis=2, plane=plane)
        for k in ("flux_t", "flux_r", "flux_b", "sat_nw_mass", "sat_w", "vol_b", "p_in", "p_out", "n_in",
                  "n_out", "nan_count"):
            assert abs(a[k] - b[k]) <= 1e-12 * max(1.0, abs(b[k])), (plane, k, a[k], b[k])
        assert abs(a["flux_r"] + a["flux_b"] - a["flux_t"]) <= 1e-12 * max(1e-12, abs(a["flux_t"]))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_non_finite_state_is_reported_unstable(precision):
    from paper_2407_10914_amd.lib import CG_EUNSTABLE, CgError

    case, kw = c2_tube(scheme=1, theta=45.0, drive="type1", nz=24, radius=6.0, wet_len=8)
    g = gpu(case, kw, precision)
    g.step(5)
    snap = g.save()  # the checkpoint a driver rolls back to
    ref = gpu(case, kw, precision)
    ref.step(5)
    ref.step(4)
    fr, fb = g.populations()
    z, y, x = 12, case.solid.shape[1] // 2, case.solid.shape[2] // 2
    assert case.solid[z, y, x] == 0
    fr[3, z, y, x] = np.nan
    g.set_state(fr, fb)
    with pytest.raises(CgError) as e:
        g.observe()
    assert e.value.status == CG_EUNSTABLE
    o = g.observe(check=False)
    assert o["nan_count"] >= 1
    # the step keeps running; the value spreads and stays reported
    g.step(3)
    with pytest.raises(CgError):
        g.observe()
    # roll back to the checkpoint: the run continues as if nothing happened
    g.load(snap)
    g.step(4)
    a, b = g.populations(), ref.populations()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert g.observe()["nan_count"] == 0
