"""Host logic of the drainage/imbibition protocol (no GPU): stage order, the
fluid switch between the imbibition phases, the two pressure drives, the
steady-state rule and the summary, on a stand-in run whose saturation
relaxes towards a value set by the applied pressure."""
import pytest

from paper_2407_10914_amd import protocol


class FakeSim:
    def __init__(self):
        self.time = 0
        self.sw = 1.0
        self.target = 1.0
        self.calls = []

    def _target(self, drho, water):
        if water:
            return min(1.0, 0.6 + 4.0 * drho)
        return max(0.3, 1.0 - 10.0 * max(0.0, drho - 0.004))

    def set_pressure(self, rin, rout):
        self.calls.append(("pressure", rin, rout))
        self.drho = rin - rout
        self.target = self._target(self.drho, self.water)

    def set_body_force(self, g):
        self.calls.append(("force", tuple(g)))
        self.drho = g[2] * 3.0 * self.length
        self.target = self._target(self.drho, self.water)

    def switch_inlet(self, z):
        self.calls.append(("switch", z))
        self.water = z == 0.0

    def step(self, n):
        self.time += n
        for _ in range(n // 100):
            self.sw += 0.2 * (self.target - self.sw)

    def observe(self, slab=None, check=True):
        assert slab[0] == 2
        return {"sat_w": self.sw, "sat_nw_mass": 1.0 - self.sw, "nan_count": 0.0}


@pytest.mark.parametrize("drive", ["type1", "type2"])
def test_protocol_phases_switch_and_steady_rule(drive):
    s = FakeSim()
    s.water = False
    s.length = 50
    st = protocol.run_protocol(s, drive=drive, region=(5, 45), length=50, drainage=(0.01, 0.03, 0.05),
                               spontaneous=(0.02, 0.0), forced=(0.02, 0.05), check=200, window=3, tol=1e-4,
                               min_steps=1000, max_steps=20000)
    assert [x.phase for x in st] == ["drainage"] * 3 + ["spontaneous"] * 2 + ["forced"] * 2
    kinds = [c[0] for c in s.calls]
    assert kinds.count("switch") == 1 and s.calls[kinds.index("switch")] == ("switch", 0.0)
    assert kinds.index("switch") == 5  # after the last spontaneous stage, before the forced ones
    if drive == "type1":
        assert all(c[0] == "pressure" and c[2] == 1.0 for c in s.calls if c[0] != "switch")
    else:
        assert all(c[0] == "force" for c in s.calls if c[0] != "switch")
        assert s.calls[0][1][2] == pytest.approx(0.01 / (3 * 50))
    assert all(x.converged for x in st)
    # each stage settled near its target; drainage lowers S_w, imbibition raises it
    assert st[2].s_w < st[1].s_w < st[0].s_w
    assert st[-1].s_w > st[2].s_w
    assert all(x.p_c > 0 for x in st[:4]) and st[4].p_c == 0.0
    assert all(x.p_c < 0 for x in st[5:])
    sm = protocol.summary(st)
    assert sm["S_w_irr"] == st[2].s_w and sm["S_w_final"] == st[-1].s_w and sm["all_converged"]


def test_stage_stops_at_max_steps_and_reports_it():
    s = FakeSim()
    s.water = False
    s.length = 50
    s.step = lambda n: (setattr(s, "time", s.time + n), setattr(s, "sw", s.sw - 0.01))
    st = protocol.run_protocol(s, drive="type1", region=(5, 45), length=50, drainage=(0.05,), spontaneous=(),
                               forced=(), check=100, tol=1e-4, min_steps=200, max_steps=1000)
    assert len(st) == 1 and not st[0].converged and st[0].steps == 1000
