"""Checkpoint/resume, state import and kernel timing through the C ABI.

A run restored from a snapshot continues bit for bit as the run that saved
it (both precisions, the snapshot carrying the time step); a snapshot does
not load into a run of another geometry or precision; canonical populations
exported from an FP64 run and imported into a fresh one (host or device
buffers) continue bit for bit; the Scheme-I line option LITERAL agrees with
the oracle as the default rule does; the kernel timers count every launch of
the kernels they are set for, and their durations fit inside the stream time
of the steps they time.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle as O
from cases import c2_tube, rel, rock

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sim(case, kw, precision):
    from paper_2407_10914_amd.sim import Sim

    s = Sim(case.solid, precision=precision, **kw)
    s.set_phase(case.phi0)
    return s


def _same(a, b):
    fa, fb = a.populations(), b.populations()
    return np.array_equal(fa[0], fb[0]) and np.array_equal(fa[1], fb[1])


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_snapshot_resume_is_bitwise(precision):
    case, kw = rock(n=32, buffer=4)
    _say("rock32 snapshot", precision)
    a = _sim(case, kw, precision)
    a.step(40)
    snap = a.save()
    t0 = a.time
    a.step(25)
    # another handle of the same geometry, elsewhere in time, takes the snapshot
    b = _sim(case, kw, precision)
    b.step(3)
    b.load(snap)
    assert b.time == t0
    b.step(25)
    assert b.time == a.time
    assert _same(a, b)
    # the saving handle itself, rewound
    a.load(snap)
    a.step(25)
    assert _same(a, b)


def test_snapshot_from_another_run_is_rejected():
    from paper_2407_10914_amd import lib as L

    case, kw = rock(n=32, buffer=4)
    # the same box and fluid node count with one fluid voxel and one solid
    # voxel of the rock region exchanged: equal buffer sizes, so only the
    # fingerprint tells the runs apart
    sol = case.solid.copy()
    inner = sol[8:32, 1:-1, 1:-1]  # rock region, away from the wall faces
    f = np.argwhere(inner == 0)[0] + (8, 1, 1)
    w = np.argwhere(inner == 1)[-1] + (8, 1, 1)
    sol[tuple(f)], sol[tuple(w)] = 1, 0
    other = dataclasses.replace(case, solid=sol)
    assert (sol == 0).sum() == (case.solid == 0).sum()
    kw2 = kw
    a = _sim(case, kw, "f64")
    snap = a.save()
    for prec, c, k in (("f32", case, kw), ("f64", other, kw2)):
        b = _sim(c, k, prec)
        with pytest.raises(L.CgError) as e:
            b.load(snap)
        _say(prec, str(e.value))
        assert "snapshot" in str(e.value)
        # the run is left as it was and still steps
        b.step(2)


@pytest.mark.parametrize("device", [False, True])
def test_exported_fp64_state_resumes_bitwise(device):
    case, kw = c2_tube(scheme=1, theta=45.0, drive="type1", nz=40, wet_len=12)
    a = _sim(case, kw, "f64")
    a.step(30)
    fr, fb = a.populations(device=device)
    b = _sim(case, kw, "f64")
    b.set_state(fr, fb)
    a.step(20)
    b.step(20)
    assert _same(a, b)


def test_exported_fp32_state_resumes_to_single_precision():
    case, kw = rock(n=32, buffer=4)
    fluid = case.solid == 0
    a = _sim(case, kw, "f32")
    a.step(30)
    fr, fb = a.populations()
    b = _sim(case, kw, "f32")
    b.set_state(fr, fb)
    a.step(10)
    b.step(10)
    for k in ("rho_r", "rho_b", "u"):
        r = rel(b.field(k), a.field(k), fluid)
        _say(k, f"{r:.3e}")
        assert r <= 1e-6, (k, r)


def test_scheme1_literal_line_rule_fp64_against_the_oracle():
    case, kw = c2_tube(scheme=1, theta=135.0, drive="type2", nz=40, wet_len=12)
    kw = dict(kw, s1_line=1)
    fluid = case.solid == 0
    g = _sim(case, kw, "f64")
    o = O.OracleSim(case.solid, eps="f64", **kw)
    o.set_phase(case.phi0)
    g.step(120)
    o.step(120)
    om = o.macro()
    for k in ("rho_r", "rho_b", "u"):
        r = rel(g.field(k), om[k], fluid)
        _say(k, f"{r:.3e}")
        assert r <= 1e-12, (k, r)


def test_kernel_timing_counts_every_launch():
    case, kw = rock(n=32, buffer=4)
    s = _sim(case, kw, "f32")
    s.set_timing("all")
    s.step(5)
    t = s.kernel_times()
    _say(t)
    for k in ("k_phase", "k_sb_phi", "k_normal", "k_sb_n", "k_main"):
        assert t[k][0] == 5 and t[k][1] > 0.0, (k, t[k])
    assert t["k_curv"][0] == 0
    s.reset_timing()
    assert all(c == 0 for c, _ in s.kernel_times().values())
    s.set_timing(["k_main"])
    s.step(2)
    t = s.kernel_times()
    assert t["k_main"][0] == 2 and t["k_phase"][0] == 0
    s.set_timing(None)
    s.step(1)
    assert s.kernel_times()["k_main"][0] == 2


def test_kernel_timers_fit_inside_the_stream_time():
    """The timers' events belong to the dispatches: over timed steps on one
    stream the kernels run one after another, so their summed durations fit
    inside the elapsed time of the same steps measured around them.  (On
    small grids the host's launch rate, not the kernels, sets that time.)"""
    import torch

    case, kw = rock(n=96, buffer=4)
    s = _sim(case, kw, "f32")
    s.step(3)
    s.sync()
    s.set_timing("all")
    s.reset_timing()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    s.step(20)
    e1.record(st)
    s.sync()
    torch.cuda.synchronize()
    wall = e0.elapsed_time(e1)
    t = s.kernel_times()
    s.set_timing(None)
    busy = sum(ms for _, ms in t.values())
    _say(f"kernels {busy:.4f} ms inside {wall:.4f} ms", t)
    assert t["k_main"][0] == 20 and t["k_phase"][0] == 20
    assert 0.1 * wall <= busy <= wall
