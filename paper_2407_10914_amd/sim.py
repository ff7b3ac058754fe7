"""Python front end of one run: a thin wrapper over the C ABI (lib.py)."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lib as L


def _torch():
    import torch

    return torch


class TorchAllocator:
    """Device memory from PyTorch's caching allocator on the current stream."""

    def __init__(self, device=0):
        torch = _torch()
        self.device = device
        self.stream = torch.cuda.current_stream(device)
        self._live = {}

        def _alloc(nbytes, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:  # out of memory: the library reports CG_ENOMEM
                return None

        def _free(ptr, ctx):
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:
                pass

        self.alloc_fn = L.ALLOC_FN(_alloc)
        self.free_fn = L.FREE_FN(_free)


class Sim:
    """One colour-gradient LBM run on the GPU.

    Arrays are (nz, ny, nx) numpy arrays (x fastest); populations (Q, nz, ny, nx).
    """

    def __init__(self, solid, *, dim, periodic, tau_r=1.0, tau_b=1.0, sigma=0.0, beta=0.7, scheme=0,
                 theta_deg=90.0, theta_field=None, s1_line=0, bc=0, rho_in=1.0, rho_out=1.0, zeta_r=0.0,
                 g=(0.0, 0.0, 0.0), precision="f32", collision=None, rho0=1.0, eps_c=None, eps_f=None,
                 eps_v=None, device=0, torch_alloc=True, block=0, pull_table=0):
        lib = L.load()
        solid = np.ascontiguousarray(solid, dtype=np.uint8)
        if solid.ndim == 2:
            solid = solid[None]
        self.shape = solid.shape
        nz, ny, nx = self.shape
        self._solid = solid
        geo = L.Geometry(dim, nx, ny, nz, solid.ctypes.data_as(C.c_void_p), (C.c_uint8 * 3)(*periodic))
        self._tf = None
        if theta_field is not None:
            self._tf = np.ascontiguousarray(theta_field, dtype=np.float64).reshape(-1)
        wet = L.Wetting(int(scheme), float(theta_deg),
                        None if self._tf is None else self._tf.ctypes.data_as(C.c_void_p), int(s1_line))
        bcs = L.BC(int(bc), float(rho_in), float(rho_out), float(zeta_r), (C.c_double * 3)(*[float(x) for x in g]))
        prec = L.CG_FP64 if precision in ("f64", "fp64", "double", L.CG_FP64) else L.CG_FP32
        opt = L.Options()
        lib.cg_options_default(C.byref(opt), prec)
        if collision is None:
            opt.collision = L.CG_MRT if dim == 3 else L.CG_BGK
        else:
            opt.collision = L.CG_MRT if collision in ("mrt", L.CG_MRT) else L.CG_BGK
        opt.rho0 = rho0
        for k, v in (("eps_c", eps_c), ("eps_f", eps_f), ("eps_v", eps_v)):
            if v is not None:
                setattr(opt, k, v)
        opt.device = device
        opt.block = int(block)
        opt.pull_table = int(pull_table)
        self._alloc = None
        if torch_alloc:
            self._alloc = TorchAllocator(device)
            opt.stream = self._alloc.stream.cuda_stream
            opt.alloc = self._alloc.alloc_fn
            opt.free = self._alloc.free_fn
        self.precision = "f64" if prec == L.CG_FP64 else "f32"
        self.dim = dim
        h = C.c_void_p()
        L.check(lib.cg_lbm_create(C.byref(geo), tau_r, tau_b, sigma, beta, C.byref(wet), C.byref(bcs),
                                  C.byref(opt), C.byref(h)))
        self._h = h
        inf = self.info()
        self.q = inf["q"]

    # ------------------------------------------------------------------ admin
    def close(self):
        h = getattr(self, "_h", None)
        if h:
            L.load().cg_lbm_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        i = L.Info()
        L.check(L.load().cg_lbm_info(self._h, C.byref(i)))
        return i.as_dict()

    @property
    def time(self):
        return L.load().cg_lbm_time(self._h)

    # ------------------------------------------------------------------ state
    def set_phase(self, phi0):
        a = np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1)
        assert a.size == self._solid.size
        L.check(L.load().cg_lbm_set_phase(self._h, a.ctypes.data_as(C.c_void_p)))

    def set_state(self, fr, fb):
        """Canonical pre-collision populations (Q, nz, ny, nx): numpy (host) or
        torch float64 CUDA tensors."""
        if hasattr(fr, "data_ptr"):
            assert fr.is_cuda and fb.is_cuda and fr.dtype == fb.dtype
            fr, fb = fr.contiguous(), fb.contiguous()
            L.check(L.load().cg_lbm_set_state(self._h, fr.data_ptr(), fb.data_ptr(), 1))
            return
        a = np.ascontiguousarray(fr, dtype=np.float64)
        b = np.ascontiguousarray(fb, dtype=np.float64)
        L.check(L.load().cg_lbm_set_state(self._h, a.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p), 0))

    def step(self, n=1):
        L.check(L.load().cg_lbm_step(self._h, int(n)))

    def sync(self):
        L.check(L.load().cg_lbm_sync(self._h))

    def observe(self, axis=-1, plane=0, check=True, slab=None):
        """Observables; slab = (axis, lo, hi) restricts them (not the plane
        flux) to the fluid nodes with lo <= coordinate < hi."""
        o = L.Observables()
        if slab is None:
            rc = L.load().cg_lbm_observe(self._h, axis, plane, C.byref(o))
        else:
            rc = L.load().cg_lbm_observe_slab(self._h, int(slab[0]), int(slab[1]), int(slab[2]), axis, plane,
                                              C.byref(o))
        if check:
            L.check(rc)
        return o.as_dict()

    def field(self, name, device=False):
        """A field of the current state: numpy (host) or a torch CUDA tensor."""
        which, comps = L.FIELDS[name]
        comps = self.q if comps == "q" else comps
        shape = (comps,) + self.shape if comps > 1 else self.shape
        if device:
            torch = _torch()
            out = torch.empty(shape, dtype=torch.float64, device="cuda")
            L.check(L.load().cg_lbm_get_field(self._h, which, out.data_ptr(), 1))
            return out
        out = np.empty(shape, dtype=np.float64)
        L.check(L.load().cg_lbm_get_field(self._h, which, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def populations(self, device=False):
        return self.field("f_r", device), self.field("f_b", device)

    # ------------------------------------------------------------ snapshots
    def save(self):
        n = L.load().cg_lbm_snapshot_bytes(self._h)
        buf = np.empty(n, dtype=np.uint8)
        L.check(L.load().cg_lbm_save(self._h, buf.ctypes.data_as(C.c_void_p)))
        return buf

    def load(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        L.check(L.load().cg_lbm_load(self._h, buf.ctypes.data_as(C.c_void_p)))

    # ------------------------------------------------------------ parameters
    def set_wetting(self, theta_deg=None, theta_field=None):
        """New contact angle: global (degrees) or a per-voxel field (nz, ny, nx)."""
        lib = L.load()
        if theta_field is not None:
            tf = np.ascontiguousarray(theta_field, dtype=np.float64).reshape(-1)
            assert tf.size == self._solid.size
            self._tf = tf
            L.check(lib.cg_lbm_set_wetting(self._h, 0.0, tf.ctypes.data_as(C.c_void_p)))
        else:
            L.check(lib.cg_lbm_set_wetting(self._h, float(theta_deg), None))

    def set_body_force(self, g):
        L.check(L.load().cg_lbm_set_body_force(self._h, (C.c_double * 3)(*[float(x) for x in g])))

    def set_pressure(self, rho_in, rho_out):
        """New Zou-He inlet/outlet densities for the following steps."""
        L.check(L.load().cg_lbm_set_pressure(self._h, float(rho_in), float(rho_out)))

    def switch_inlet(self, zeta_r):
        """Inject the other fluid from now on (Eqs. 37-38): 1.0 = red, 0.0 = blue."""
        L.check(L.load().cg_lbm_switch_inlet(self._h, float(zeta_r)))

    # ------------------------------------------------------- interface points
    def line_crossings(self, axis, at=(0, 0, 0), lo=0, hi=None, blend=0.0, blend_axis=0, max_points=256):
        """phi = 0 crossings along one grid line (device side): the line along
        `axis` through the voxel coordinates `at` (x, y, z; the entry on
        `axis` is ignored), blended with the next line along `blend_axis`."""
        n = (self.shape[2], self.shape[1], self.shape[0])
        ln = L.Line(int(axis), (C.c_int * 3)(*[int(v) for v in at]), int(lo), int(n[axis] if hi is None else hi),
                    int(blend_axis), float(blend))
        pts = (C.c_double * max(1, max_points))()
        cnt = C.c_int()
        L.check(L.load().cg_lbm_line_crossings(self._h, C.byref(ln), pts, int(max_points), C.byref(cnt)))
        return [pts[k] for k in range(min(cnt.value, max_points))]

    def drop_shape(self, base_axis=0, wall_axis=1, slice=0, wall=0.5, row=1):
        """Base, height, cap radius and angle (through the drop) of a sessile
        drop, Eqs. 45-46, from the device phase field."""
        d = L.Drop()
        L.check(L.load().cg_lbm_drop_shape(self._h, int(base_axis), int(wall_axis), int(slice), float(wall), int(row),
                                           C.byref(d)))
        return d.as_dict()

    def front(self, axis=2, at=None):
        """First interface point from the low end along `axis` on one grid line
        (default: the middle of the other axes), or nan."""
        if at is None:
            at = (self.shape[2] // 2, self.shape[1] // 2, self.shape[0] // 2)
        xs = self.line_crossings(axis, at, max_points=1)
        return xs[0] if xs else float("nan")

    # --------------------------------------------------------------- adjoint
    def adjoint(self, objective="saturation", *, n_steps, checkpoint_every=None, axis=2, lo=0, hi=1 << 30,
                delta=0.0, field_grad=False):
        """Objective J of the state n_steps ahead and its exact discrete
        gradient with respect to the contact angle (global, per degree; and,
        with field_grad, per voxel as a float64 CUDA tensor (nz, ny, nx)), the
        body-force acceleration and, with Zou-He faces, the inlet and outlet
        densities.  The run's state is left unchanged."""
        torch = _torch()
        sp = L.AdjointSpec()
        sp.objective = L.OBJECTIVES[objective] if isinstance(objective, str) else int(objective)
        sp.axis, sp.lo, sp.hi = int(axis), int(lo), int(hi)
        sp.n_steps = int(n_steps)
        sp.checkpoint_every = int(checkpoint_every or n_steps)
        sp.delta = float(delta)
        gr = L.Gradients()
        field = None
        if field_grad:
            field = torch.empty(self.shape, dtype=torch.float64, device="cuda")
            gr.dJ_dtheta_field = field.data_ptr()
        L.check(L.load().cg_lbm_adjoint(self._h, C.byref(sp), C.byref(gr)))
        return {"J": gr.J, "dJ_dtheta": gr.dJ_dtheta, "dJ_dg": np.array(gr.dJ_dg[:]),
                "dJ_drho_in": gr.dJ_drho_in, "dJ_drho_out": gr.dJ_drho_out,
                "dJ_dtheta_field": field, "ms_forward": gr.ms_forward, "ms_reverse": gr.ms_reverse,
                "work_bytes": gr.work_bytes}

    # ---------------------------------------------------------------- timing
    KERNELS = ("k_phase", "k_sb_phi", "k_normal", "k_sb_n", "k_curv", "k_main", "k_face")

    def set_graph(self, on=True):
        """Replay steps from captured HIP graphs (same results, less launch
        overhead for small runs)."""
        L.check(L.load().cg_lbm_set_graph(self._h, 1 if on else 0))

    @property
    def graph_captures(self):
        return L.load().cg_lbm_graph_captures(self._h)

    def set_timing(self, kernels="all"):
        """Bracket launches of the named kernels with HIP events ("all", None,
        or an iterable of names)."""
        if kernels == "all":
            mask = -1
        elif not kernels:
            mask = 0
        else:
            mask = 0
            for k in kernels:
                mask |= 1 << self.KERNELS.index(k)
        L.check(L.load().cg_lbm_set_timing(self._h, mask))

    def reset_timing(self):
        L.check(L.load().cg_lbm_reset_timing(self._h))

    def tune(self, reps=5):
        """Pick the block size of every step kernel (advances the run by 3*reps steps)."""
        buf = C.create_string_buffer(1024)
        L.check(L.load().cg_lbm_tune(self._h, int(reps), buf, 1024))
        return buf.value.decode()

    def kernel_times(self):
        names = (C.c_char * 32 * 16)()
        counts = (C.c_int64 * 16)()
        ms = (C.c_double * 16)()
        n = C.c_int(16)
        L.check(L.load().cg_lbm_kernel_times(self._h, names, counts, ms, C.byref(n)))
        return {bytes(names[k]).split(b"\0", 1)[0].decode(): (counts[k], ms[k]) for k in range(n.value)}


class Batch:
    """Runs of one precision and lattice advanced together by persistent
    launches (one per stage for all runs) replayed from a hipGraph.  The runs
    (Sim objects) must outlive the batch; each can still be observed or read
    through its own Sim after sync()."""

    def __init__(self, sims):
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*[s._h.value for s in self.sims])
        h = C.c_void_p()
        L.check(L.load().cg_batch_create(arr, len(self.sims), C.byref(h)))
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            L.load().cg_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        L.check(L.load().cg_batch_step(self._h, int(n)))

    def sync(self):
        L.check(L.load().cg_batch_sync(self._h))

    def set_graph(self, on=True):
        L.check(L.load().cg_batch_set_graph(self._h, 1 if on else 0))

    def observe(self, i, axis=-1, plane=0):
        """Observables of run i after the queued steps (cg_batch_observe)."""
        o = L.Observables()
        L.check(L.load().cg_batch_observe(self._h, int(i), axis, plane, C.byref(o)))
        return o.as_dict()

    def tune(self, reps=5):
        buf = C.create_string_buffer(4096)
        L.check(L.load().cg_batch_tune(self._h, int(reps), buf, 4096))
        return buf.value.decode()

    @property
    def graph_captures(self):
        return L.load().cg_batch_graph_captures(self._h)

    def info(self):
        n = C.c_int64()
        bs = (C.c_int * 6)()
        gr = (C.c_int * 6)()
        L.check(L.load().cg_batch_info(self._h, C.byref(n), bs, gr))
        return {"total_nodes": n.value, "block": list(bs), "grid": list(gr)}
