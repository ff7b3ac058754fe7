"""Run life cycle on the device: creating and destroying runs gives back every
byte of device memory, through PyTorch's caching allocator and through plain
hipMalloc, with everything a run can own switched on (graph replay, a batch,
snapshots, the allocation-free observables, an adjoint with its checkpoint
and work memory).  And a fluid at rest in a rock stays at rest."""
import gc

import numpy as np
import pytest

from cases import c2_tube, rock
from parity_helpers import gpu, orc, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _exercise(precision, torch_alloc, adjoint):
    from paper_2407_10914_amd import inputs
    from paper_2407_10914_amd.sim import Batch, Sim

    case, kw = c2_tube(scheme=1, theta=60.0, drive="type1", nz=24, radius=6.0, wet_len=8)
    s = Sim(case.solid, precision=precision, torch_alloc=torch_alloc, **kw)
    s.set_phase(case.phi0)
    s.set_graph(True)
    s.step(6)
    s.observe()
    snap = s.save()
    s.load(snap)
    b = Batch([s])
    b.step(3)
    b.sync()
    b.close()
    s.close()
    if adjoint:
        c, th = inputs.drainage_rock(n=24, corr=4.0, buffer=3, seed=2412)
        a = Sim(c.solid, dim=3, periodic=c.periodic, tau_r=1.0, tau_b=0.6, sigma=0.01, beta=0.95, scheme=1,
                theta_deg=40.0, theta_field=th, collision=1, g=(0.0, 0.0, 1e-5), precision=precision,
                torch_alloc=torch_alloc)
        a.set_phase(c.phi0)
        a.adjoint("saturation", n_steps=20, checkpoint_every=5, lo=3, hi=c.solid.shape[0] - 3, field_grad=True)
        a.close()


def _settle():
    torch.cuda.synchronize()
    gc.collect()
    torch.cuda.empty_cache()
    torch.cuda.synchronize()


def test_create_and_destroy_return_device_memory():
    _settle()
    base = torch.cuda.memory_allocated()
    frees = []
    for rep in range(3):
        for precision in ("f32", "f64"):
            for torch_alloc in (True, False):
                _exercise(precision, torch_alloc, adjoint=(rep == 0 or torch_alloc))
        _settle()
        assert torch.cuda.memory_allocated() == base, rep
        frees.append(torch.cuda.mem_get_info()[0])
    say(f"free device memory after each round: {[f >> 20 for f in frees]} MiB")
    # once the runtime's own structures exist, further rounds leave nothing behind
    assert abs(frees[2] - frees[1]) <= 8 << 20


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_fluid_at_rest_stays_at_rest(precision):
    """One fluid filling a rock, no drive, wetting on: no gradient of the
    phase anywhere, so nothing may move; the oracle keeps the rest state
    exactly and so does the device."""
    case, kw = rock(n=24, buffer=3, drive="type2", scheme=1)
    kw = dict(kw, g=(0.0, 0.0, 0.0), bc=0, periodic=(0, 0, 1))
    phi = -np.ones_like(case.phi0)
    g = gpu(case, kw, precision)
    g.set_phase(phi)
    rho0 = g.field("rho_r") + g.field("rho_b")  # sum_i w_i rho_o: 1 up to the rounding of the weights
    g.step(40)
    o = orc(case, kw, eps=precision)
    o.set_phase(phi)
    o.step(40)
    fluid = case.solid == 0
    om = o.macro()
    u, ou = g.field("u"), om["u"]
    rho = g.field("rho_r") + g.field("rho_b")
    orho = om["rho_r"] + om["rho_b"]
    say(f"{precision}: max |u| {np.abs(u[:, fluid]).max():.2e} (oracle {np.abs(ou[:, fluid]).max():.2e}), "
        f"max |rho - rho(t=0)| {np.abs(rho - rho0)[fluid].max():.2e}, max |rho - 1| {np.abs(rho[fluid] - 1).max():.2e}")
    assert np.abs(ou[:, fluid]).max() == 0.0
    assert np.abs(u[:, fluid]).max() == 0.0
    assert np.array_equal(rho[fluid], rho0[fluid])
    if precision == "f64":
        assert np.array_equal(rho[fluid], orho[fluid])
    assert np.abs(rho[fluid] - 1.0).max() <= 1e-15
