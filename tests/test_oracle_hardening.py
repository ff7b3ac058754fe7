"""CPU hardening of the checker and of the host set-up code.

* Visiting order: every per-voxel loop of the oracle's step visits the voxels
  in a seeded random permutation (and the face loops their (x, y) positions
  in the induced order).  A stage reads only what earlier stages wrote, so
  the state after a run must be bit for bit the state of the natural order;
  an in-place update that read a neighbour's new value would break this.
  The same holds for the number of OpenMP threads.
* Sanitizers: the oracle (g++) and the host set-up code of the library
  (the host pass of its HIP source) are built with AddressSanitizer and
  UndefinedBehaviorSanitizer, any report fatal, and driven through every
  entry point on small geometries by the programs in tests/sanitize/.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O

import cases

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _run(case, kw, steps, perm_seed=None, threads=None, pressure=None, switch=None):
    o = O.OracleSim(case.solid, **kw)
    o.set_phase(case.phi0)
    if perm_seed is not None:
        o.set_visit_order(np.random.default_rng(perm_seed).permutation(case.solid.size))
    prev = O.set_threads(threads) if threads else None
    try:
        o.step(steps // 2)
        if pressure:
            o.set_pressure(*pressure)
        if switch is not None:
            o.switch_inlet(switch)
        o.step(steps - steps // 2)
    finally:
        if prev:
            O.set_threads(prev)
    return o


def _cases():
    out = []
    c, kw = cases.c1_sessile_2d()
    out.append(("2d-sessile-bgk-scheme1", c, kw, 40, {}))
    c, kw = cases.outlet_slug(nz=24, radius=4.0, slug=(10, 18), n=10, zeta_r=0.25)
    out.append(("tube-outlet-mixed-injection", c, kw, 40, dict(pressure=(1.03, 1.0), switch=1.0)))
    c, kw = cases.rock(n=16, buffer=3, scheme=2, drive="type2")
    rng = np.random.default_rng(11)
    kw = dict(kw, theta_field=np.where(c.solid == 1, rng.uniform(20.0, 160.0, c.solid.shape), 0.0))
    out.append(("rock-mrt-scheme2-theta-field", c, kw, 20, {}))
    c, kw = cases.rock(n=16, buffer=3, scheme=3, theta=50.0)
    out.append(("rock-fictitious-density", c, kw, 20, {}))
    c, kw = cases.rock(n=16, buffer=3, scheme=1, theta=120.0)
    kw = dict(kw, collision=0)
    out.append(("rock-bgk-scheme1", c, kw, 20, {}))
    return out


CASES = _cases()


@pytest.mark.parametrize("name,case,kw,steps,extra", CASES, ids=[c[0] for c in CASES])
def test_shuffled_visiting_order_gives_the_same_state(name, case, kw, steps, extra):
    ref = _run(case, kw, steps, **extra)
    fr0, fb0 = ref.get_state()
    for seed in (1, 2):
        o = _run(case, kw, steps, perm_seed=seed, **extra)
        fr, fb = o.get_state()
        assert np.array_equal(fr, fr0) and np.array_equal(fb, fb0), f"{name}: order {seed} changed the state"
    assert np.isfinite(fr0).all() and np.abs(fr0).sum() > 0


def test_thread_count_gives_the_same_state():
    name, case, kw, steps, extra = CASES[2]
    a = _run(case, kw, steps, threads=1, **extra).get_state()
    b = _run(case, kw, steps, threads=7, perm_seed=5, **extra).get_state()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_visit_order_must_be_a_permutation():
    c, kw = cases.drop_3d(n=6, R=2.0)
    o = O.OracleSim(c.solid, **kw)
    bad = np.arange(c.solid.size)
    bad[3] = 4
    with pytest.raises(Exception):
        o.set_visit_order(bad)
    with pytest.raises(ValueError):
        o.set_visit_order(np.arange(5))


# ---------------------------------------------------------------- sanitizers

SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1:detect_stack_use_after_return=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def _build(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, "build failed:\n" + " ".join(cmd) + "\n" + r.stderr[-4000:]


def _exec(exe, cwd):
    r = subprocess.run([exe], cwd=cwd, capture_output=True, text=True, timeout=600, env=SAN_ENV)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out[-6000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _build(["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
            "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "oracle"),
            os.path.join(ROOT, "oracle", "cg_oracle.cpp"), os.path.join(HERE, "sanitize", "oracle_driver.cpp"),
            "-o", exe], str(tmp_path))
    out = _exec(exe, str(tmp_path))
    assert "oracle driver: all checks passed" in out, out


def _hipcc():
    c = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    return c if os.path.exists(c) else shutil.which("hipcc")


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_host_setup_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The host set-up code (voxel classes, smoothing, wall normals, angles,
    pull tables) is compiled by the host pass only, sanitizers on that pass."""
    csrc = os.path.join(ROOT, "paper_2407_10914_amd", "csrc")
    objs = []
    for src in (os.path.join(csrc, "setup.cpp"), os.path.join(HERE, "sanitize", "setup_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _build([_hipcc(), "-x", "hip", "--cuda-host-only", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                "-ffp-contract=off", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all", "-I", csrc, "-I", os.path.join(ROOT, "include"),
                "-c", src, "-o", obj], str(tmp_path))
        objs.append(obj)
    exe = str(tmp_path / "setup_san")
    clang = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang++")
    _build([clang, "-fsanitize=address,undefined", "-fno-sanitize-recover=all", *objs, "-lpthread", "-o", exe],
           str(tmp_path))
    out = _exec(exe, str(tmp_path))
    assert "setup driver: all checks passed" in out, out
