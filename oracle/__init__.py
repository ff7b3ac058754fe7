"""Python access to the plain FP64 CPU oracle (``liboracle.so``).

Test infrastructure only: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are its only callers.  The GPU product path never imports
this package.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("periodic", C.c_int * 3),
        ("collision", C.c_int), ("scheme", C.c_int), ("s1_line", C.c_int), ("bc", C.c_int),
        ("tau_r", C.c_double), ("tau_b", C.c_double), ("sigma", C.c_double), ("beta", C.c_double),
        ("rho0", C.c_double), ("theta_deg", C.c_double),
        ("rho_in", C.c_double), ("rho_out", C.c_double), ("zeta_r", C.c_double),
        ("g", C.c_double * 3),
        ("eps_c", C.c_double), ("eps_f", C.c_double), ("eps_v", C.c_double),
    ]


class Obs(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "mass_r", "mass_b", "n_fluid", "sat_w", "sat_nw_mass", "flux_t", "flux_r", "flux_b",
        "vol_r", "vol_b", "p_in", "p_out", "n_in", "n_out", "u_max", "nan_count")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class TangentSpec(C.Structure):
    _fields_ = [("objective", C.c_int), ("axis", C.c_int), ("lo", C.c_int), ("hi", C.c_int), ("n_steps", C.c_int),
                ("seed", C.c_int), ("theta_dir", C.c_void_p)]


OBJECTIVES = {"sat_nw": 0, "red_volume": 1, "flux": 2}
SEEDS = {"theta": 0, "gx": 1, "gy": 2, "gz": 3, "theta_field": 4, "rho_in": 5, "rho_out": 6}


def lib():
    """Load liboracle.so, building it first if it is not there."""
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b

            _b.build()
        _LIB = C.CDLL(path)
        d, i, p = C.c_double, C.c_int, C.c_void_p
        L = _LIB
        L.orc_last_error.restype = C.c_char_p
        L.orc_create.restype = p
        L.orc_create.argtypes = [C.POINTER(Params), p, p]
        L.orc_destroy.argtypes = [p]
        L.orc_q.argtypes = [p]
        for name in ("orc_set_phase",):
            getattr(L, name).argtypes = [p, p]
        L.orc_set_state.argtypes = [p, p, p]
        L.orc_get_state.argtypes = [p, p, p]
        L.orc_step.argtypes = [p, i]
        L.orc_macro.argtypes = [p, p, p, p, p]
        L.orc_stages.argtypes = [p, p, p, p, p, p]
        L.orc_observe.argtypes = [p, i, i, C.POINTER(Obs)]
        L.orc_observe_slab.argtypes = [p, i, i, i, i, i, C.POINTER(Obs)]
        L.orc_setup_info.argtypes = [p, p, p, p, p, p]
        L.orc_lattice.argtypes = [i, p, p, p]
        L.orc_mrt_matrix.argtypes = [p, p]
        L.orc_meq.argtypes = [d, d, p, p]
        L.orc_forcing_moments.argtypes = [p, p, p, p]
        L.orc_rates.argtypes = [d, d, d, p, p]
        L.orc_collide_node.argtypes = [i, i, p, d, d, p, p, d, d, p, p]
        L.orc_recolor.argtypes = [i, p, d, d, d, p, p, p]
        L.orc_scheme1.argtypes = [i, p, p, d, i, d, d, p]
        L.orc_scheme2.argtypes = [i, p, p, d, d, p]
        L.orc_zouhe_inlet.argtypes = [p, p, d, d]
        L.orc_zouhe_outlet.argtypes = [p, p, d, d]
        L.orc_tangent.argtypes = [C.POINTER(Params), p, p, p, C.POINTER(TangentSpec), p, p]
        L.orc_objective.argtypes = [p, i, i, i, i, p]
        L.orc_switch_inlet.argtypes = [p, d]
        L.orc_set_threads.argtypes = [i]
        L.orc_set_pressure.argtypes = [p, d, d]
        L.orc_set_body_force.argtypes = [p, p]
        L.orc_set_visit_order.argtypes = [p, p]
    return _LIB


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.size == n
    return a


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle: " + lib().orc_last_error().decode())


# ---------------------------------------------------------------- node pieces
def lattice(dim):
    e = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    q = lib().orc_lattice(dim, _ptr(e), _ptr(w), _ptr(opp))
    return e[:q].copy(), w[:q].copy(), opp[:q].copy()


def mrt_matrix():
    M = np.zeros((19, 19))
    n2 = np.zeros(19)
    lib().orc_mrt_matrix(_ptr(M), _ptr(n2))
    return M, n2


def meq(rho, rho0, u):
    out = np.zeros(19)
    lib().orc_meq(rho, rho0, _ptr(_f64(u, 3)), _ptr(out))
    return out


def forcing_moments(u, F, S):
    out = np.zeros(19)
    lib().orc_forcing_moments(_ptr(_f64(u, 3)), _ptr(_f64(F, 3)), _ptr(_f64(S, 19)), _ptr(out))
    return out


def rates(phi, tau_r, tau_b):
    a, b = C.c_double(), C.c_double()
    lib().orc_rates(phi, tau_r, tau_b, C.byref(a), C.byref(b))
    return a.value, b.value


def collide_node(dim, collision, ft, rho, rho0, u, F, s_nu, s_q, S=None):
    ft = _f64(ft)
    out = np.zeros_like(ft)
    _check(lib().orc_collide_node(dim, collision, _ptr(ft), rho, rho0, _ptr(_f64(u, 3)), _ptr(_f64(F, 3)),
                                  s_nu, s_q, _ptr(None if S is None else _f64(S, 19)), _ptr(out)))
    return out


def recolor(dim, fpp, rho_r, rho_b, beta, n):
    fpp = _f64(fpp)
    a, b = np.zeros_like(fpp), np.zeros_like(fpp)
    lib().orc_recolor(dim, _ptr(fpp), rho_r, rho_b, beta, _ptr(_f64(n, 3)), _ptr(a), _ptr(b))
    return a, b


def scheme1(dim, nc, nw, theta_deg, line=0, eps_f=1e-12, eps_v=1e-12):
    out = np.zeros(3)
    lib().orc_scheme1(dim, _ptr(_f64(nc, 3)), _ptr(_f64(nw, 3)), theta_deg, line, eps_f, eps_v, _ptr(out))
    return out


def scheme2(dim, nc, nw, theta_deg, eps_v=1e-12):
    out = np.zeros(3)
    lib().orc_scheme2(dim, _ptr(_f64(nc, 3)), _ptr(_f64(nw, 3)), theta_deg, eps_v, _ptr(out))
    return out


def zouhe_inlet(fr, fb, rho_in, zeta_r):
    fr, fb = _f64(fr, 19).copy(), _f64(fb, 19).copy()
    lib().orc_zouhe_inlet(_ptr(fr), _ptr(fb), rho_in, zeta_r)
    return fr, fb


def zouhe_outlet(fr, fb, rho_out, phi_up):
    fr, fb = _f64(fr, 19).copy(), _f64(fb, 19).copy()
    lib().orc_zouhe_outlet(_ptr(fr), _ptr(fb), rho_out, phi_up)
    return fr, fb


def set_threads(n):
    """OpenMP threads of the oracle's node loops; returns the count in use."""
    return lib().orc_set_threads(int(n))


# ----------------------------------------------------------------- simulation
DEFAULT_EPS = {"f64": dict(eps_c=1e-6, eps_f=1e-12, eps_v=1e-12),
               "f32": dict(eps_c=1e-6, eps_f=1e-6, eps_v=1e-6)}


class OracleSim:
    """A whole run of the oracle on a dense voxel box (arrays (nz, ny, nx))."""

    def __init__(self, solid, *, dim, periodic, tau_r=1.0, tau_b=1.0, sigma=0.0, beta=0.7, rho0=1.0,
                 collision=None, scheme=0, theta_deg=90.0, s1_line=0, bc=0, rho_in=1.0, rho_out=1.0,
                 zeta_r=0.0, g=(0.0, 0.0, 0.0), theta_field=None, eps="f64", eps_c=None, eps_f=None,
                 eps_v=None):
        solid = np.ascontiguousarray(solid, dtype=np.uint8)
        if solid.ndim == 2:
            solid = solid[None]
        self.shape = solid.shape
        nz, ny, nx = self.shape
        P = Params()
        P.dim, P.nx, P.ny, P.nz = dim, nx, ny, nz
        for a in range(3):
            P.periodic[a] = int(periodic[a])
            P.g[a] = float(g[a])
        P.collision = (1 if dim == 3 else 0) if collision is None else int(collision)
        P.scheme, P.s1_line, P.bc = int(scheme), int(s1_line), int(bc)
        P.tau_r, P.tau_b, P.sigma, P.beta, P.rho0 = tau_r, tau_b, sigma, beta, rho0
        P.theta_deg, P.rho_in, P.rho_out, P.zeta_r = theta_deg, rho_in, rho_out, zeta_r
        e = dict(DEFAULT_EPS[eps])
        for k, v in (("eps_c", eps_c), ("eps_f", eps_f), ("eps_v", eps_v)):
            if v is not None:
                e[k] = v
        P.eps_c, P.eps_f, P.eps_v = e["eps_c"], e["eps_f"], e["eps_v"]
        self.params = P
        self.dim = dim
        self._solid = solid
        tf = None if theta_field is None else _f64(theta_field, solid.size)
        self._theta_field = tf
        self._h = lib().orc_create(C.byref(P), _ptr(solid), _ptr(tf))
        if not self._h:
            raise ValueError("oracle: " + lib().orc_last_error().decode())
        self.q = lib().orc_q(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    @property
    def fluid(self):
        return self._solid == 0

    def set_phase(self, phi0):
        _check(lib().orc_set_phase(self._h, _ptr(_f64(phi0, self._solid.size))))

    def set_state(self, fr, fb):
        n = self.q * self._solid.size
        _check(lib().orc_set_state(self._h, _ptr(_f64(fr, n)), _ptr(_f64(fb, n))))

    def get_state(self):
        fr = np.zeros((self.q,) + self.shape)
        fb = np.zeros_like(fr)
        _check(lib().orc_get_state(self._h, _ptr(fr), _ptr(fb)))
        return fr, fb

    def step(self, n=1):
        _check(lib().orc_step(self._h, int(n)))

    def macro(self):
        rr, rb, ph = (np.zeros(self.shape) for _ in range(3))
        u = np.zeros((3,) + self.shape)
        _check(lib().orc_macro(self._h, _ptr(rr), _ptr(rb), _ptr(ph), _ptr(u)))
        return dict(rho_r=rr, rho_b=rb, phi=ph, u=u)

    def stages(self):
        ph, k = np.zeros(self.shape), np.zeros(self.shape)
        n3, c3, f3 = (np.zeros((3,) + self.shape) for _ in range(3))
        _check(lib().orc_stages(self._h, _ptr(ph), _ptr(n3), _ptr(c3), _ptr(k), _ptr(f3)))
        return dict(phi=ph, n=n3, C=c3, kappa=k, F=f3)

    def objective(self, which, axis=2, lo=0, hi=1 << 30):
        """Objective of the current state (same definitions as ``tangent``)."""
        J = C.c_double()
        _check(lib().orc_objective(self._h, OBJECTIVES.get(which, which), axis, lo, hi, C.byref(J)))
        return J.value

    def tangent(self, phi0, *, objective, n_steps, seed, theta_dir=None, axis=2, lo=0, hi=1 << 30):
        """(J, dJ) after n_steps from the rest state of phi0, dJ the exact
        discrete directional derivative (forward mode, dual numbers) along the
        seeded parameter: "theta" (global angle, per degree), "gx"/"gy"/"gz"
        (body-force acceleration), "rho_in"/"rho_out" (Zou-He densities) or
        "theta_field" along theta_dir (dense voxel array, degrees)."""
        sp = TangentSpec()
        sp.objective = OBJECTIVES.get(objective, objective)
        sp.axis, sp.lo, sp.hi, sp.n_steps = axis, lo, hi, int(n_steps)
        sp.seed = SEEDS.get(seed, seed)
        td = None if theta_dir is None else _f64(theta_dir, self._solid.size)
        sp.theta_dir = _ptr(td)
        J, dJ = C.c_double(), C.c_double()
        _check(lib().orc_tangent(C.byref(self.params), _ptr(self._solid), _ptr(self._theta_field),
                                 _ptr(_f64(phi0, self._solid.size)), C.byref(sp), C.byref(J), C.byref(dJ)))
        return J.value, dJ.value

    def switch_inlet(self, zeta_r):
        """Replace the injected fluid (Eqs. 37-38): 1.0 = red, 0.0 = blue."""
        _check(lib().orc_switch_inlet(self._h, float(zeta_r)))

    def set_visit_order(self, perm):
        """Visit the voxels in the order `perm` (a permutation of the flat
        voxel indices) in every per-voxel loop of the step."""
        perm = np.ascontiguousarray(perm, dtype=np.int64).ravel()
        if perm.size != self._solid.size:
            raise ValueError("perm must list every voxel once")
        _check(lib().orc_set_visit_order(self._h, _ptr(perm)))

    def set_pressure(self, rho_in, rho_out):
        _check(lib().orc_set_pressure(self._h, float(rho_in), float(rho_out)))

    def set_body_force(self, g):
        _check(lib().orc_set_body_force(self._h, _ptr(_f64(g, 3))))

    def observe(self, axis=2, plane=0, slab=None):
        """Observables; slab = (axis, lo, hi) restricts them (not the plane flux)
        to the fluid nodes with lo <= coordinate < hi."""
        o = Obs()
        if slab is None:
            _check(lib().orc_observe(self._h, axis, plane, C.byref(o)))
        else:
            _check(lib().orc_observe_slab(self._h, int(slab[0]), int(slab[1]), int(slab[2]), axis, plane,
                                          C.byref(o)))
        return o.as_dict()

    def setup_info(self):
        cls = np.zeros(self.shape, np.uint8)
        g3 = np.zeros(self.shape)
        nw = np.zeros((3,) + self.shape)
        ct, st = np.zeros(self.shape), np.zeros(self.shape)
        _check(lib().orc_setup_info(self._h, _ptr(cls), _ptr(g3), _ptr(nw), _ptr(ct), _ptr(st)))
        return dict(cls=cls, g3=g3, nw=nw, cos_t=ct, sin_t=st)
