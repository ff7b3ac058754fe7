"""ctypes binding of libcglbm.so (the C ABI of include/cg_lbm.h).

Argument marshalling only: every step of the time step runs in the HIP
library.  PyTorch supplies device memory (its caching allocator, through the
library's allocator callbacks) and the stream.  Importing this module fails
loudly when the library is not built: there is no other compute path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcglbm.so")

CG_OK, CG_EINVAL, CG_ENOMEM, CG_EHIP, CG_EUNSTABLE, CG_EUNSUPPORTED, CG_ESTATE = 0, -1, -2, -3, -4, -5, -6
CG_FP32, CG_FP64 = 0, 1
CG_BGK, CG_MRT = 0, 1
CG_BC_NONE, CG_BC_ZOUHE = 0, 1
FIELDS = {"rho_r": (0, 1), "rho_b": (1, 1), "phi": (2, 1), "u": (3, 3), "f_r": (4, "q"), "f_b": (5, "q"),
          "n": (6, 3), "C": (7, 3), "kappa": (8, 1), "force": (9, 3)}

# Every symbol include/cg_lbm.h declares.
EXPORTS = ("cg_options_default", "cg_lbm_create", "cg_lbm_destroy", "cg_last_error", "cg_lbm_set_phase",
           "cg_lbm_set_state", "cg_lbm_step", "cg_lbm_sync", "cg_lbm_time", "cg_lbm_observe",
           "cg_lbm_get_field", "cg_lbm_info", "cg_lbm_snapshot_bytes", "cg_lbm_save", "cg_lbm_load",
           "cg_lbm_set_timing", "cg_lbm_kernel_times", "cg_lbm_reset_timing", "cg_lbm_set_graph",
           "cg_lbm_graph_captures", "cg_batch_create",
           "cg_batch_destroy", "cg_batch_step", "cg_batch_sync", "cg_batch_set_graph", "cg_batch_tune",
           "cg_batch_info", "cg_batch_observe", "cg_lbm_set_wetting", "cg_lbm_set_body_force", "cg_lbm_adjoint",
           "cg_lbm_tune", "cg_lbm_set_pressure", "cg_lbm_switch_inlet", "cg_lbm_line_crossings",
           "cg_lbm_drop_shape", "cg_batch_graph_captures", "cg_stream_probe", "cg_lbm_observe_noalloc",
           "cg_lbm_observe_slab")

OBJECTIVES = {"saturation": 0, "red_volume": 1, "flux": 2}


class CgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"cg_lbm error {status}: {msg}")
        self.status = status


class Geometry(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("solid", C.c_void_p),
                ("periodic", C.c_uint8 * 3)]


class Wetting(C.Structure):
    _fields_ = [("scheme", C.c_int), ("theta_deg", C.c_double), ("theta_field_deg", C.c_void_p),
                ("scheme1_line", C.c_int)]


class BC(C.Structure):
    _fields_ = [("type", C.c_int), ("rho_in", C.c_double), ("rho_out", C.c_double), ("zeta_r", C.c_double),
                ("g", C.c_double * 3)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("collision", C.c_int), ("rho0", C.c_double), ("eps_c", C.c_double),
                ("eps_f", C.c_double), ("eps_v", C.c_double), ("device", C.c_int), ("stream", C.c_void_p),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", C.c_void_p), ("block", C.c_int),
                ("pull_table", C.c_int)]


class Observables(C.Structure):
    _fields_ = [("step", C.c_int64)] + [(n, C.c_double) for n in (
        "mass_r", "mass_b", "n_fluid", "sat_w", "sat_nw_mass", "flux_t", "flux_r", "flux_b", "vol_r", "vol_b",
        "p_in", "p_out", "n_in", "n_out", "u_max", "nan_count")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [(n, C.c_int) for n in ("dim", "q", "nx", "ny", "nz", "precision", "collision")] + \
               [(n, C.c_int64) for n in ("voxels", "fluid", "fluid_boundary", "solid_boundary", "inlet", "outlet",
                                         "state_bytes", "device_bytes")] + \
               [("pull_bits", C.c_int), ("pull_fallback_bits", C.c_int), ("pull_waves", C.c_int64),
                ("pull_waves_8bit", C.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Line(C.Structure):
    _fields_ = [("axis", C.c_int), ("at", C.c_int * 3), ("lo", C.c_int), ("hi", C.c_int), ("blend_axis", C.c_int),
                ("blend", C.c_double)]


class Drop(C.Structure):
    _fields_ = [("base", C.c_double), ("height", C.c_double), ("radius", C.c_double), ("theta_deg", C.c_double),
                ("n_base_points", C.c_int)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class AdjointSpec(C.Structure):
    _fields_ = [("objective", C.c_int), ("axis", C.c_int), ("lo", C.c_int), ("hi", C.c_int),
                ("n_steps", C.c_int64), ("checkpoint_every", C.c_int64), ("delta", C.c_double)]


class Gradients(C.Structure):
    _fields_ = [("J", C.c_double), ("dJ_dtheta", C.c_double), ("dJ_dg", C.c_double * 3),
                ("dJ_dtheta_field", C.c_void_p), ("ms_forward", C.c_double), ("ms_reverse", C.c_double),
                ("work_bytes", C.c_int64), ("dJ_drho_in", C.c_double), ("dJ_drho_out", C.c_double)]


_LIB = None


def load():
    """Load libcglbm.so; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (or python -m "
                          "paper_2407_10914_amd.build)")
    # PyTorch ships its own HIP runtime with the same SONAME; load it first so
    # that the library binds to that one copy and torch-allocated device
    # memory and streams are valid in both.
    import torch  # noqa: F401

    L = C.CDLL(LIB_PATH)
    p, i, d, i64 = C.c_void_p, C.c_int, C.c_double, C.c_int64
    L.cg_options_default.argtypes = [C.POINTER(Options), i]
    L.cg_options_default.restype = None
    L.cg_lbm_create.argtypes = [C.POINTER(Geometry), d, d, d, d, C.POINTER(Wetting), C.POINTER(BC),
                                C.POINTER(Options), C.POINTER(p)]
    L.cg_lbm_destroy.argtypes = [p]
    L.cg_lbm_destroy.restype = None
    L.cg_last_error.restype = C.c_char_p
    L.cg_lbm_set_phase.argtypes = [p, p]
    L.cg_lbm_set_state.argtypes = [p, p, p, i]
    L.cg_lbm_step.argtypes = [p, i64]
    L.cg_lbm_sync.argtypes = [p]
    L.cg_lbm_time.argtypes = [p]
    L.cg_lbm_time.restype = i64
    L.cg_lbm_observe.argtypes = [p, i, i, C.POINTER(Observables)]
    L.cg_lbm_observe_noalloc.argtypes = [p, i, i, C.POINTER(Observables)]
    L.cg_lbm_observe_slab.argtypes = [p, i, i, i, i, i, C.POINTER(Observables)]
    L.cg_lbm_get_field.argtypes = [p, i, p, i]
    L.cg_lbm_info.argtypes = [p, C.POINTER(Info)]
    L.cg_lbm_snapshot_bytes.argtypes = [p]
    L.cg_lbm_snapshot_bytes.restype = i64
    L.cg_lbm_save.argtypes = [p, p]
    L.cg_lbm_load.argtypes = [p, p]
    L.cg_lbm_set_timing.argtypes = [p, i]
    L.cg_lbm_set_graph.argtypes = [p, i]
    L.cg_lbm_graph_captures.argtypes = [p]
    L.cg_lbm_graph_captures.restype = C.c_int64
    L.cg_lbm_kernel_times.argtypes = [p, p, p, p, C.POINTER(C.c_int)]
    L.cg_lbm_reset_timing.argtypes = [p]
    L.cg_lbm_tune.argtypes = [p, i, C.c_char_p, C.c_size_t]
    L.cg_lbm_set_wetting.argtypes = [p, d, p]
    L.cg_lbm_set_body_force.argtypes = [p, C.POINTER(C.c_double)]
    L.cg_lbm_adjoint.argtypes = [p, C.POINTER(AdjointSpec), C.POINTER(Gradients)]
    L.cg_lbm_set_pressure.argtypes = [p, d, d]
    L.cg_lbm_switch_inlet.argtypes = [p, d]
    L.cg_lbm_line_crossings.argtypes = [p, C.POINTER(Line), p, i, C.POINTER(i)]
    L.cg_lbm_drop_shape.argtypes = [p, i, i, i, d, i, C.POINTER(Drop)]
    L.cg_batch_graph_captures.argtypes = [p]
    L.cg_batch_graph_captures.restype = i64
    L.cg_stream_probe.argtypes = [i, p, p, C.c_size_t, i, i, i, p, i, C.POINTER(C.c_float)]
    L.cg_batch_create.argtypes = [p, i, C.POINTER(p)]
    L.cg_batch_destroy.argtypes = [p]
    L.cg_batch_destroy.restype = None
    L.cg_batch_step.argtypes = [p, i64]
    L.cg_batch_sync.argtypes = [p]
    L.cg_batch_observe.argtypes = [p, i, i, i, C.POINTER(Observables)]
    L.cg_batch_set_graph.argtypes = [p, i]
    L.cg_batch_tune.argtypes = [p, i, C.c_char_p, C.c_size_t]
    L.cg_batch_info.argtypes = [p, C.POINTER(i64), p, p]
    _LIB = L
    return L


def check(rc):
    if rc != CG_OK:
        raise CgError(rc, load().cg_last_error().decode())
    return rc
