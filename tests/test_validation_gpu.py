"""The validation harness of the paper's setups, at reduced sizes (the full
setups run from `python -m paper_2407_10914_amd.validation`): the harness
runs on the device and its numbers are physically sane."""
import numpy as np
import pytest

from parity_helpers import say

pytestmark = pytest.mark.gpu


def test_laplace_sweep_small():
    from paper_2407_10914_amd import validation as V

    r = V.laplace_sweep(n=64, radii=(10.0, 14.0, 18.0), steps=3000, log=say)
    say("laplace 64^3:", r["sigma_fit"], r["error_pct"])
    assert all(d["dp"] > 0 for d in r["drops"])
    assert r["error_pct"] < 10.0
    for d in r["drops"]:
        assert abs(d["sigma_drop"] / r["sigma_input"] - 1.0) < 0.15


def test_angle_sweep_small():
    from paper_2407_10914_amd import validation as V

    r = V.angle_sweep(thetas=(60.0, 120.0), schemes=(2,), shape=(64, 34, 64), radius=10.0, steps=4000, log=say)
    for run in r["runs"]:
        assert abs(run["error"]) < 12.0, run
    assert r["runs"][0]["theta_sim"] < 90.0 < r["runs"][1]["theta_sim"]


def test_washburn_short_tube():
    from paper_2407_10914_amd import validation as V

    cases = [dict(scheme=2, theta=45.0, drive="none", dP=0.0), dict(scheme=2, theta=90.0, drive="type1", dP=0.004),
             dict(scheme=2, theta=90.0, drive="type2", dP=0.004)]
    r = V.washburn_runs(cases=cases, shape=(12, 12, 41), pre_steps=1000, max_steps=30000, every=500, log=say)
    for run in r["runs"]:
        assert run["z_end"] > run["z_init"] + 5.0, run
        assert np.isfinite(run["area_error_pct"]) and run["area_error_pct"] < 50.0, run
