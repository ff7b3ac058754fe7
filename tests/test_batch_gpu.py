"""Batched persistent launches: every run of a batch advances exactly as it
does on its own (bitwise in double precision; in single precision to the
rounding of the same arithmetic), with or without the captured graph, before
and after autotuning; and every run of a batch against its own oracle run
(FP64: 1e-12, bitwise in practice; FP32: the one-step protocol from the
batch's state), including two runs at the smallest edge of the batched
contact-angle sweep (48^3, Scheme-I and Scheme-II) and a periodic drop
without walls."""
import numpy as np
import pytest

import oracle as O
from cases import c2_tube, drop_3d, rel, sessile_3d
from parity_helpers import TOL32, TOL64, compare_macro, say

pytestmark = pytest.mark.gpu


def _runs(precision, specs):
    from paper_2407_10914_amd.sim import Sim

    out = []
    for case, kw in specs:
        s = Sim(case.solid, precision=precision, **kw)
        s.set_phase(case.phi0)
        out.append((case, s))
    return out


def _specs(sweep=False):
    # uneven sizes, both schemes, angles on both sides of 90 degrees, and one
    # run with Zou-He faces; with sweep, two runs of the batched sweep's
    # smallest edge and a periodic drop without any solid voxel (a run whose
    # solid-boundary stages have no point)
    out = [sessile_3d(16, 40.0, 1), sessile_3d(20, 120.0, 2), sessile_3d(13, 75.0, 2),
           c2_tube(scheme=1, theta=45.0, drive="type1", nz=24, radius=6.0, wet_len=8)]
    if sweep:
        out += [sessile_3d(48, 25.0, 1), sessile_3d(48, 150.0, 2), drop_3d(n=14, R=4.5)]
    return out


def _fields(s):
    return [s.field("rho_r"), s.field("rho_b"), s.field("u")]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("graph", [True, False])
def test_batch_matches_individual_runs(precision, graph):
    from paper_2407_10914_amd.sim import Batch

    specs = _specs()
    solo = _runs(precision, specs)
    batched = _runs(precision, specs)
    b = Batch([s for _, s in batched])
    b.set_graph(graph)
    for n in (1, 6, 5):  # first step from the host state, then even and odd counts
        b.step(n)
        for _, s in solo:
            s.step(n)
    b.sync()
    for (case, s1), (_, s2) in zip(solo, batched):
        assert s1.time == s2.time == 12
        fluid = case.solid == 0
        for a, c in zip(_fields(s1), _fields(s2)):
            r = rel(c, a, fluid)
            if precision == "f64":
                assert r == 0.0, r
            else:
                assert r <= 1e-6, r


def test_batch_autotune_keeps_results(tmp_path, monkeypatch):
    from paper_2407_10914_amd.sim import Batch

    monkeypatch.setenv("CGLBM_TUNE_CACHE", str(tmp_path / "tune.txt"))
    specs = _specs()
    solo = _runs("f64", specs)
    batched = _runs("f64", specs)
    b = Batch([s for _, s in batched])
    rep = b.tune(reps=2)
    print(rep, flush=True)
    info = b.info()
    assert all(bs in (64, 128, 256) for bs in info["block"])
    assert (tmp_path / "tune.txt").exists()
    b.step(9)  # tune took the first step
    for _, s in solo:
        s.step(10)
    b.sync()
    for (case, s1), (_, s2) in zip(solo, batched):
        fluid = case.solid == 0
        for a, c in zip(_fields(s1), _fields(s2)):
            assert rel(c, a, fluid) == 0.0
    # a second batch over the same class reads the cached choice
    b2 = Batch([s for _, s in batched])
    assert b2.info()["block"] == info["block"] and b2.info()["grid"] == info["grid"]


def test_run_stepped_alone_between_batch_steps():
    from paper_2407_10914_amd.sim import Batch

    specs = _specs()[:2]
    solo = _runs("f64", specs)
    batched = _runs("f64", specs)
    b = Batch([s for _, s in batched])
    b.step(4)
    batched[0][1].step(3)  # one run advances on its own
    b.step(4)
    b.sync()
    solo[0][1].step(11)
    solo[1][1].step(8)
    for (case, s1), (_, s2) in zip(solo, batched):
        assert s1.time == s2.time
        fluid = case.solid == 0
        for a, c in zip(_fields(s1), _fields(s2)):
            assert rel(c, a, fluid) == 0.0


def test_batch_observe_reports_each_run():
    """cg_batch_observe(i) after queued batch steps gives what the run's own
    cg_lbm_observe gives, and what the run stepped alone gives (FP64: exactly)."""
    from paper_2407_10914_amd.sim import Batch

    specs = _specs()
    solo = _runs("f64", specs)
    batched = _runs("f64", specs)
    b = Batch([s for _, s in batched])
    b.step(7)
    for _, s in solo:
        s.step(7)
    for k, ((case, s1), (_, s2)) in enumerate(zip(solo, batched)):
        ob = b.observe(k)
        assert ob == s2.observe()
        o1 = s1.observe()
        for key in ("step", "mass_r", "mass_b", "sat_nw_mass", "vol_r", "u_max"):
            assert ob[key] == o1[key], (k, key, ob[key], o1[key])
    with pytest.raises(Exception):
        b.observe(len(specs))


@pytest.mark.parametrize("graph", [True, False])
def test_batch_runs_against_their_oracle_runs_fp64(graph):
    from paper_2407_10914_amd.sim import Batch

    specs = _specs(sweep=True)
    batched = _runs("f64", specs)
    b = Batch([s for _, s in batched])
    b.set_graph(graph)
    orcs = []
    for case, kw in specs:
        o = O.OracleSim(case.solid, **kw)
        o.set_phase(case.phi0)
        orcs.append(o)
    for n in (1, 6, 7):
        b.step(n)
        for o in orcs:
            o.step(n)
    b.sync()
    for k, ((case, s), o) in enumerate(zip(batched, orcs)):
        assert s.time == 14
        compare_macro(s, o, case.solid == 0, TOL64, f"batch run {k} vs oracle t=14")


def test_batch_runs_against_their_oracle_runs_fp32_per_step():
    from paper_2407_10914_amd.sim import Batch

    specs = _specs(sweep=True)
    batched = _runs("f32", specs)
    b = Batch([s for _, s in batched])
    b.step(1)
    b.step(30)
    b.sync()
    orcs = []
    for (case, kw), (_, s) in zip(specs, batched):
        fr, fb = s.populations()
        o = O.OracleSim(case.solid, eps="f32", **kw)
        o.set_state(fr, fb)
        orcs.append(o)
    b.step(1)  # one batched step from the exported state
    b.sync()
    for k, ((case, s), o) in enumerate(zip(batched, orcs)):
        o.step(1)
        compare_macro(s, o, case.solid == 0, TOL32, f"batch run {k} fp32 31->32")


def test_odd_step_counts_reuse_the_two_captured_graphs():
    """One graph per starting parity, captured once: odd step counts neither
    drop nor re-capture them, and the runs stay bitwise with solo runs."""
    from paper_2407_10914_amd.sim import Batch

    specs = _specs()
    solo = _runs("f64", specs)
    batched = _runs("f64", specs)
    b = Batch([s for _, s in batched])
    total = 0
    for n in (1, 3, 5, 7, 2, 9, 4):
        b.step(n)
        total += n
    b.sync()
    assert b.graph_captures <= 2, b.graph_captures
    for _, s in solo:
        s.step(total)
    for (case, s1), (_, s2) in zip(solo, batched):
        assert s1.time == s2.time == total
        for a, c in zip(_fields(s1), _fields(s2)):
            assert rel(c, a, case.solid == 0) == 0.0


def test_parameter_changes_reach_batched_runs():
    """A new body force and new Zou-He densities set on a run that belongs to a
    batch apply from the batch's next step (bitwise as the run stepped alone
    with the same changes, and as the oracle)."""
    from paper_2407_10914_amd.sim import Batch

    specs = _specs()
    batched = _runs("f64", specs)
    b = Batch([s for _, s in batched])
    orcs = []
    for case, kw in specs:
        o = O.OracleSim(case.solid, **kw)
        o.set_phase(case.phi0)
        orcs.append(o)
    b.step(5)
    for o in orcs:
        o.step(5)
    b.sync()
    g = (0.0, 3e-5, 0.0)
    batched[0][1].set_body_force(g)
    orcs[0].set_body_force(g)
    batched[3][1].set_pressure(1.03, 0.99)
    orcs[3].set_pressure(1.03, 0.99)
    b.step(6)
    for o in orcs:
        o.step(6)
    b.sync()
    for k, ((case, s), o) in enumerate(zip(batched, orcs)):
        compare_macro(s, o, case.solid == 0, TOL64, f"batch run {k} after parameter changes")
