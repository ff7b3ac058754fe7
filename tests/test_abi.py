"""The C-ABI library loads and exports every symbol include/cg_lbm.h declares
(no compute call: this runs without a GPU), and the product package does not
reach the oracle."""
import ast
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cg_lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(cg_[a-z_0-9]+)\s*\(", src))
    return sorted(n for n in names if not n.endswith("_fn"))


def test_header_declares_the_boundary_calls():
    names = _declared()
    for required in ("cg_lbm_create", "cg_lbm_step", "cg_lbm_observe", "cg_lbm_destroy", "cg_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2407_10914_amd import lib as L

    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libcglbm.so not built")
    so = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(so, n)]
    assert not missing, missing
    assert set(_declared()) <= set(L.EXPORTS)


def test_library_reports_bad_arguments_without_a_gpu():
    from paper_2407_10914_amd import lib as L

    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libcglbm.so not built")
    so = L.load()
    h = ctypes.c_void_p()
    # NULL geometry is rejected before any device call
    rc = so.cg_lbm_create(None, 1.0, 1.0, 0.0, 0.5, None, None, None, ctypes.byref(h))
    assert rc == L.CG_EINVAL
    assert b"geometry" in so.cg_last_error()


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2407_10914_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if not f.endswith(".py"):
                continue
            tree = ast.parse(open(os.path.join(dirpath, f)).read())
            for node in ast.walk(tree):
                if isinstance(node, ast.Import):
                    assert all(not a.name.startswith("oracle") for a in node.names), f
                if isinstance(node, ast.ImportFrom):
                    assert not (node.module or "").startswith("oracle"), f


def _create(L, so, *, dim=3, shape=(6, 6, 6), tau=(1.0, 1.0), sigma=0.01, beta=0.7, scheme=1, theta=60.0,
            bc=None, precision=None, collision=None):
    import numpy as np

    nz, ny, nx = shape
    solid = np.zeros(shape, dtype=np.uint8)
    geo = L.Geometry(dim, nx, ny, nz, solid.ctypes.data_as(ctypes.c_void_p), (ctypes.c_uint8 * 3)(1, 1, 1))
    wet = L.Wetting(scheme, theta, None, 0)
    opt = L.Options()
    so.cg_options_default(ctypes.byref(opt), L.CG_FP32 if precision is None else precision)
    if collision is not None:
        opt.collision = collision
    h = ctypes.c_void_p()
    rc = so.cg_lbm_create(ctypes.byref(geo), tau[0], tau[1], sigma, beta, ctypes.byref(wet),
                          None if bc is None else ctypes.byref(bc), ctypes.byref(opt), ctypes.byref(h))
    return rc, so.cg_last_error()


@pytest.mark.parametrize("case, code, words", [
    (dict(tau=(0.5, 1.0)), "CG_EINVAL", b"tau"),
    (dict(tau=(1.0, 0.3)), "CG_EINVAL", b"tau"),
    (dict(beta=1.5), "CG_EINVAL", b"beta"),
    (dict(sigma=float("nan")), "CG_EINVAL", b"sigma"),
    (dict(scheme=4), "CG_EINVAL", b"scheme"),
    (dict(theta=0.0), "CG_EINVAL", b"theta"),
    (dict(theta=180.0), "CG_EINVAL", b"theta"),
    (dict(dim=2, shape=(1, 6, 6), collision=1), "CG_EUNSUPPORTED", b"MRT"),
    (dict(precision=7), "CG_EINVAL", b"precision"),
])
def test_create_rejects_invalid_parameters_before_any_device_call(case, code, words):
    """Parameter checks of cg_lbm_create run before the device is touched, so
    they hold on a machine without a GPU; each names what it rejects."""
    from paper_2407_10914_amd import lib as L

    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libcglbm.so not built")
    so = L.load()
    rc, msg = _create(L, so, **case)
    assert rc == getattr(L, code), (rc, msg)
    assert words in msg, msg


def test_create_rejects_a_zou_he_face_in_2d_and_a_bad_colour_fraction():
    from paper_2407_10914_amd import lib as L

    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libcglbm.so not built")
    so = L.load()
    bc = L.BC(L.CG_BC_ZOUHE, 1.01, 1.0, 1.5, (ctypes.c_double * 3)(0.0, 0.0, 0.0))
    rc, msg = _create(L, so, bc=bc)
    assert rc == L.CG_EINVAL and b"zeta_r" in msg, msg
    bc = L.BC(L.CG_BC_ZOUHE, 1.01, 1.0, 1.0, (ctypes.c_double * 3)(0.0, 0.0, 0.0))
    rc, msg = _create(L, so, dim=2, shape=(1, 6, 6), collision=0, bc=bc)
    assert rc == L.CG_EUNSUPPORTED and b"Zou-He" in msg, msg


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes mirror of a header struct has the C size and the C offset
    of each field (compiled with the host C compiler from include/cg_lbm.h)."""
    import shutil
    import subprocess

    from paper_2407_10914_amd import lib as L

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"cg_geometry": L.Geometry, "cg_wetting": L.Wetting, "cg_bc": L.BC, "cg_options": L.Options,
               "cg_observables": L.Observables, "cg_info": L.Info, "cg_adjoint_spec": L.AdjointSpec,
               "cg_gradients": L.Gradients}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "cg_lbm.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    c = {}
    for ln in out:
        if ln:
            s, f, v = ln.split()
            c[(s, f)] = int(v)
    src_h = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "cg_lbm.h")).read(), flags=re.S)
    for body, cname in re.findall(r"typedef struct\s*\{(.*?)\}\s*(cg_[a-z_]+)\s*;", src_h, flags=re.S):
        if cname not in mirrors:
            continue
        declared = []
        for decl in body.split(";"):
            parts = [p.strip() for p in decl.split(",") if p.strip()]
            for p in parts:
                tok = re.sub(r"\[.*?\]", "", p).replace("*", " ").split()
                declared.append(tok[-1])
        assert declared == [f[0] for f in mirrors[cname]._fields_], cname
    for cname, py in mirrors.items():
        assert c[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert c[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])
