"""The neighbour table the pull reads changes where the source indices come
from, never a result.  Three tables exist: one byte per link with a base per
wave of 64 nodes (waves whose offsets spread over more than 252 nodes fall
back to the next table), two bytes per link with a base per tile of 256
nodes, and plain int32 indices.  On a 40^3 rock the 8-bit table has waves
that fall back, so the default run reads two tables at once.

FP64: each table, run against the oracle, must agree bit for bit over a
whole run (Type-I Zou-He inlet and outlet, Scheme-I wetting: every kind of
link, bounce-back and open face included).  FP32: the three tables give
identical bits.  A batch that mixes the tables steps every run as it steps
alone.
"""
import sys

import numpy as np
import pytest

import oracle as O
from cases import rel, rock

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sim(case, kw, precision, table):
    from paper_2407_10914_amd.sim import Sim

    s = Sim(case.solid, precision=precision, pull_table=table, **kw)
    s.set_phase(case.phi0)
    return s


def _check_info(s, table):
    inf = s.info()
    _say("table", table, {k: inf[k] for k in ("pull_bits", "pull_fallback_bits", "pull_waves", "pull_waves_8bit")})
    if table in (0, 8):
        assert inf["pull_bits"] == 8
        # the case must hold waves on both sides of the fallback
        assert 0 < inf["pull_waves_8bit"] < inf["pull_waves"]
        assert inf["pull_fallback_bits"] == 16
    else:
        assert inf["pull_bits"] == table
        assert inf["pull_fallback_bits"] == 0
        assert inf["pull_waves_8bit"] == 0


@pytest.mark.parametrize("table", [0, 16, 32])
def test_fp64_rock_bitwise_against_the_oracle_for_every_pull_table(table):
    case, kw = rock(n=40, buffer=4)
    fluid = case.solid == 0
    _say("rock40 fp64 pull_table", table)
    g = _sim(case, kw, "f64", table)
    _check_info(g, table)
    o = O.OracleSim(case.solid, eps="f64", **kw)
    o.set_phase(case.phi0)
    g.step(40)
    o.step(40)
    om = o.macro()
    for k in ("rho_r", "rho_b", "u"):
        gv = g.field(k)
        err = rel(gv, om[k], fluid)
        _say(k, f"{err:.3e}")
        assert err == 0.0, (k, err)


def test_results_do_not_depend_on_the_pull_table_alone_or_batched():
    from paper_2407_10914_amd.sim import Batch

    case, kw = rock(n=40, buffer=4)
    runs = {t: _sim(case, kw, "f32", t) for t in (0, 16, 32)}
    for t, s in runs.items():
        _check_info(s, t)
        s.step(30)
    ref = runs[0].populations()
    for t in (16, 32):
        assert np.array_equal(runs[t].populations(), ref), t
    # a batch of runs that read different tables steps each run as it does
    # alone (FP64: bit for bit)
    single = _sim(case, kw, "f64", 0)
    single.step(20)
    parts = [_sim(case, kw, "f64", t) for t in (0, 16, 32)]
    b = Batch(parts)
    b.step(20)
    b.sync()
    for t, s in zip((0, 16, 32), parts):
        for k in ("rho_r", "rho_b", "u"):
            assert np.array_equal(s.field(k), single.field(k)), (t, k)
    b.close()
