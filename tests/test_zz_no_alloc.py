"""cg_lbm_observe_noalloc (the observables for callers that cannot allocate)
against cg_lbm_observe: the same kernels over the same state, so the same
numbers; two calls in a row, the second on a smaller run; the refusal of a
run above the documented limit; called through the C ABI."""
import ctypes as C

import numpy as np
import pytest

from cases import c2_tube, sessile_3d

pytestmark = pytest.mark.gpu


def _sim(case, kw, precision):
    from paper_2407_10914_amd.sim import Sim

    s = Sim(case.solid, precision=precision, **kw)
    s.set_phase(case.phi0)
    return s


def _noalloc(s, axis=-1, plane=0):
    from paper_2407_10914_amd import lib as L

    o = L.Observables()
    rc = L.load().cg_lbm_observe_noalloc(s._h, axis, plane, C.byref(o))
    return rc, o.as_dict()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_observables_equal_the_allocating_call(precision):
    big_case, big_kw = sessile_3d(40, 60.0, 1)
    small_case, small_kw = c2_tube(scheme=2, theta=45.0, drive="type1", nz=24, radius=6.0, wet_len=8)
    big, small = _sim(big_case, big_kw, precision), _sim(small_case, small_kw, precision)
    assert small.info()["fluid"] < big.info()["fluid"]
    big.step(37)
    small.step(23)
    for s, axis, plane in ((big, 1, 5), (small, 2, 11)):  # the second call: a smaller input
        rc, got = _noalloc(s, axis, plane)
        assert rc == 0
        want = s.observe(axis=axis, plane=plane)
        for k, v in want.items():
            assert abs(got[k] - v) <= 1e-12 * max(1.0, abs(v)), (k, got[k], v)
        assert got == want  # same kernels, same order: identical in practice
    # and again on the first run after the second used the array
    rc, got = _noalloc(big, 1, 5)
    assert rc == 0 and got == big.observe(axis=1, plane=5)


def test_noalloc_refuses_runs_above_its_limit():
    from paper_2407_10914_amd import lib as L

    n = 224  # 11.2 M fluid nodes in a periodic box: above 8,947,456
    solid = np.zeros((n, n, n), np.uint8)
    from paper_2407_10914_amd.sim import Sim

    s = Sim(solid, dim=3, periodic=(1, 1, 1), precision="f32", collision=1)
    rc, _ = _noalloc(s)
    assert rc == L.CG_EINVAL
    assert b"8947456" in L.load().cg_last_error()
    del s
