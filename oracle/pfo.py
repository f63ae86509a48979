"""ctypes wrapper of the FP64 oracle library (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import this module.  It builds ``libpfo.so`` from ``pfo.c`` on
first use if the library is missing or older than its source.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

NFIELDS = 36
FIELD_NAMES = (["C1", "C2", "C3", "rho"]
               + [f"gradC{k}_{d}" for k in (1, 2, 3) for d in "xy"]
               + ["lapC1", "lapC2", "lapC3", "mu1", "mu2", "mu3"]
               + [f"gradmu{k}_{d}" for k in (1, 2, 3) for d in "xy"]
               + ["lapmu1", "lapmu2", "lapmu3", "dif1", "dif2", "Fs_x", "Fs_y", "u_x", "u_y", "p",
                  "gradp_x", "gradp_y", "gradrho_x", "gradrho_y"])
assert len(FIELD_NAMES) == NFIELDS


class Params(ct.Structure):
    _fields_ = [
        ("nx", ct.c_int32), ("ny", ct.c_int32), ("n_h", ct.c_int32),
        ("rho", ct.c_double * 3), ("nu", ct.c_double * 3),
        ("powerlaw_comp", ct.c_int32),
        ("K", ct.c_double), ("n", ct.c_double), ("nu_min", ct.c_double), ("nu_max", ct.c_double),
        ("sigma12", ct.c_double), ("sigma13", ct.c_double), ("sigma23", ct.c_double), ("Lambda", ct.c_double),
        ("xi", ct.c_double), ("D0", ct.c_double),
        ("variable_mobility", ct.c_int32),
        ("tau_h", ct.c_double),
        ("g", ct.c_double), ("fx", ct.c_double),
        ("strain_literal", ct.c_int32), ("mobility_flux", ct.c_int32),
        ("hforce_mode", ct.c_int32), ("gforce_cd", ct.c_int32),
        ("force_potential", ct.c_int32), ("mix_linear", ct.c_int32),
        ("tau_iterations", ct.c_int32),
        ("open_x", ct.c_int32), ("u_in", ct.c_double),
    ]


def make_params(d: dict) -> Params:
    """Parameter block from a case's dict.  The case dicts carry the HIP
    library's name `hforce_cd` (1: central differences for grad C_i in the
    hbar forcing), which is this oracle's hforce_mode = 1 unless hforce_mode
    is given."""
    p = Params()
    for name, typ in Params._fields_:
        if name in ("rho", "nu"):
            arr = (ct.c_double * 3)(*[float(v) for v in d[name]])
            setattr(p, name, arr)
        elif name in d:
            setattr(p, name, d[name])
    if d.get("hforce_cd") and "hforce_mode" not in d:
        p.hforce_mode = 1
    return p


def lib():
    global _lib
    if _lib is None:
        so = os.environ.get("PFO_LIBRARY")   # another build of pfo.c (the pins' mutation check)
        if not so:
            so = os.path.join(_HERE, "libpfo.so")
            src = os.path.join(_HERE, "pfo.c")
            stamp = max(os.path.getmtime(src), os.path.getmtime(os.path.join(_HERE, "build.py")))
            if not os.path.exists(so) or os.path.getmtime(so) < stamp:
                _build.build()
        L = ct.CDLL(so)
        P = ct.POINTER
        dp = P(ct.c_double)
        L.pfo_create.argtypes = [P(Params), P(ct.c_void_p)]
        L.pfo_destroy.argtypes = [ct.c_void_p]
        L.pfo_destroy.restype = None
        L.pfo_init_fields.argtypes = [ct.c_void_p, dp, dp, dp]
        L.pfo_step.argtypes = [ct.c_void_p, ct.c_int64]
        L.pfo_macroscopic.argtypes = [ct.c_void_p, dp, dp, dp, dp]
        L.pfo_fields.argtypes = [ct.c_void_p, dp]
        L.pfo_bubble_centroid_velocity.argtypes = [ct.c_void_p, ct.c_int, dp]
        L.pfo_state_doubles.argtypes = [ct.c_void_p]
        L.pfo_state_doubles.restype = ct.c_size_t
        L.pfo_get_state.argtypes = [ct.c_void_p, dp]
        L.pfo_set_state.argtypes = [ct.c_void_p, dp]
        L.pfo_lattice.argtypes = [P(ct.c_int), P(ct.c_int), dp, P(ct.c_int)]
        L.pfo_lattice.restype = None
        L.pfo_stencil.argtypes = [dp, ct.c_int, ct.c_int, ct.c_int, ct.c_int, dp]
        L.pfo_bulk_energy.argtypes = [P(Params), ct.c_double, ct.c_double, ct.c_double]
        L.pfo_bulk_energy.restype = ct.c_double
        L.pfo_chem_potential.argtypes = [P(Params), dp, dp, dp]
        L.pfo_chem_potential.restype = None
        L.pfo_mixture_tau.argtypes = [P(Params), dp, ct.c_double]
        L.pfo_mixture_tau.restype = ct.c_double
        L.pfo_set_threads.argtypes = [ct.c_int]
        L.pfo_set_threads.restype = None
        L.pfo_get_threads.argtypes = []
        L.pfo_get_threads.restype = ct.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's per-node loops (results do not depend on it)."""
    lib().pfo_set_threads(int(n))


def get_threads() -> int:
    return int(lib().pfo_get_threads())


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """One FP64 domain. Arrays are float64 of shape (planes, ny, nx)."""

    def __init__(self, params: dict):
        self.params = dict(params)
        self._p = make_params(self.params)
        self.nx, self.ny, self.n_h = int(params["nx"]), int(params["ny"]), int(params["n_h"])
        h = ct.c_void_p()
        rc = lib().pfo_create(ct.byref(self._p), ct.byref(h))
        if rc != 0:
            raise ValueError(f"pfo_create failed ({rc})")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().pfo_destroy(h)
            self._h = None

    def init_fields(self, C, u=None, p=None):
        C, u, p = _f64(C), _f64(u), _f64(p)
        assert C.size == self.n_h * self.nx * self.ny
        rc = lib().pfo_init_fields(self._h, _ptr(C), _ptr(u), _ptr(p))
        if rc != 0:
            raise ValueError(f"pfo_init_fields failed ({rc})")

    def step(self, n: int = 1):
        rc = lib().pfo_step(self._h, int(n))
        if rc != 0:
            raise ValueError(f"pfo_step failed ({rc})")

    def macroscopic(self):
        ny, nx = self.ny, self.nx
        rho = np.empty((ny, nx)); u = np.empty((2, ny, nx)); p = np.empty((ny, nx))
        phi = np.empty((self.n_h, ny, nx))
        lib().pfo_macroscopic(self._h, _ptr(rho), _ptr(u), _ptr(p), _ptr(phi))
        return dict(rho=rho, u=u, p=p, phi=phi)

    def fields(self):
        out = np.empty((NFIELDS, self.ny, self.nx))
        lib().pfo_fields(self._h, _ptr(out))
        return {k: out[i] for i, k in enumerate(FIELD_NAMES)}

    def centroid(self, comp: int = 0):
        out = np.empty(6)
        rc = lib().pfo_bubble_centroid_velocity(self._h, int(comp), _ptr(out))
        if rc != 0:
            raise ValueError("pfo_bubble_centroid_velocity failed")
        return out

    def get_state(self):
        n = lib().pfo_state_doubles(self._h)
        out = np.empty(n)
        lib().pfo_get_state(self._h, _ptr(out))
        return out

    def set_state(self, s):
        s = _f64(s)
        assert s.size == lib().pfo_state_doubles(self._h)
        lib().pfo_set_state(self._h, _ptr(s))

    def populations(self):
        """(gbar[9], hbar[n_h][9], tau) views of a copy of the state."""
        s = self.get_state()
        n = self.nx * self.ny
        g = s[:9 * n].reshape(9, self.ny, self.nx)
        h = s[9 * n:9 * n + 9 * n * self.n_h].reshape(self.n_h, 9, self.ny, self.nx)
        tau = s[9 * n + 9 * n * self.n_h:].reshape(self.ny, self.nx)
        return g, h, tau


def lattice():
    ex = (ct.c_int * 9)(); ey = (ct.c_int * 9)(); w = (ct.c_double * 9)(); opp = (ct.c_int * 9)()
    lib().pfo_lattice(ex, ey, w, opp)
    return np.array(ex[:]), np.array(ey[:]), np.array(w[:]), np.array(opp[:])


STENCIL_KIND = dict(grad_cd=0, lap_cd=1, dir_md=2, grad_md=3, dir_cd=4)


def stencil(f, kind: str, a: int = 0):
    f = _f64(f)
    ny, nx = f.shape
    planes = 2 if kind in ("grad_cd", "grad_md") else 1
    out = np.empty((planes, ny, nx))
    rc = lib().pfo_stencil(_ptr(f), nx, ny, STENCIL_KIND[kind], int(a), _ptr(out))
    assert rc == 0
    return out if planes == 2 else out[0]


def bulk_energy(params: dict, c1, c2, c3):
    p = make_params(params)
    return lib().pfo_bulk_energy(ct.byref(p), float(c1), float(c2), float(c3))


def chem_potential(params: dict, c, lap):
    p = make_params(params)
    c = np.ascontiguousarray(c, dtype=np.float64); lap = np.ascontiguousarray(lap, dtype=np.float64)
    mu = np.empty(3)
    lib().pfo_chem_potential(ct.byref(p), _ptr(c), _ptr(lap), _ptr(mu))
    return mu


def mixture_tau(params: dict, c, gdot: float):
    p = make_params(params)
    c = np.ascontiguousarray(c, dtype=np.float64)
    return lib().pfo_mixture_tau(ct.byref(p), _ptr(c), float(gdot))


def run_case(case: dict, steps: int, **switches):
    """Initialise an oracle domain from a generated case and advance it."""
    prm = dict(case["params"]); prm.update(switches)
    o = Oracle(prm)
    o.init_fields(case["C"], case.get("u"), case.get("p"))
    if steps:
        o.step(steps)
    return o
