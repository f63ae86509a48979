"""Python binding of the HIP library (argument marshalling only).

Every function forwards to the C ABI of include/pflbm.h in the in-tree
libpflbm.so; PyTorch supplies the device workspace, the output tensors and
the stream.  There is no fallback: without the built library (or without a
GPU) every call raises.
"""
from __future__ import annotations

import ctypes as ct
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpflbm.so")

STATUS = {0: "ok", -1: "invalid argument", -2: "workspace", -3: "device", -4: "non-finite",
          -5: "state", -6: "unsupported"}

# every symbol declared in include/pflbm.h
EXPORTS = ("pflbm_workspace_bytes", "pflbm_create", "pflbm_init_fields", "pflbm_step", "pflbm_macroscopic",
           "pflbm_bubble_centroid_velocity", "pflbm_state_bytes", "pflbm_get_state", "pflbm_set_state",
           "pflbm_export_populations", "pflbm_num_variants", "pflbm_variant_name", "pflbm_set_variant",
           "pflbm_autotune", "pflbm_set_graph", "pflbm_stream", "pflbm_bytes_per_update", "pflbm_destroy",
           "pflbm_status_string", "pflbm_check_state", "pflbm_case_nonfinite",
           "pflbm_bubble_centroid_velocity_noalloc")


class PflbmError(RuntimeError):
    def __init__(self, where: str, status: int):
        super().__init__(f"{where}: {STATUS.get(status, status)} ({status})")
        self.status = status


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
        ("storage", ct.c_int32), ("store_h", ct.c_int32),
        ("tau_iterations", ct.c_int32), ("hforce_cd", ct.c_int32),
        ("open_x", ct.c_int32), ("u_in", ct.c_double), ("mobility_flux", ct.c_int32),
    ]


def make_params(d: dict) -> Params:
    p = Params()
    for name, _ in Params._fields_:
        if name in ("rho", "nu"):
            setattr(p, name, (ct.c_double * 3)(*[float(v) for v in d[name]]))
        elif name in d:
            setattr(p, name, d[name])
    return p


_lib = None


def lib():
    """The loaded libpflbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2207_09431_amd.build.build()")
        L = ct.CDLL(LIB_PATH)
        P, vp, i32, dp, fp = ct.POINTER, ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_double), ct.c_void_p
        L.pflbm_workspace_bytes.argtypes = [P(Params), i32]
        L.pflbm_workspace_bytes.restype = ct.c_size_t
        L.pflbm_create.argtypes = [P(Params), i32, vp, ct.c_size_t, vp, P(vp)]
        L.pflbm_create.restype = i32
        L.pflbm_init_fields.argtypes = [vp, i32, dp, dp, dp]
        L.pflbm_init_fields.restype = i32
        L.pflbm_step.argtypes = [vp, ct.c_int64]
        L.pflbm_step.restype = i32
        L.pflbm_macroscopic.argtypes = [vp, i32, fp, fp, fp, fp]
        L.pflbm_macroscopic.restype = i32
        L.pflbm_bubble_centroid_velocity.argtypes = [vp, i32, i32, dp]
        L.pflbm_bubble_centroid_velocity.restype = i32
        L.pflbm_state_bytes.argtypes = [vp]
        L.pflbm_state_bytes.restype = ct.c_size_t
        L.pflbm_get_state.argtypes = [vp, vp, ct.c_size_t]
        L.pflbm_get_state.restype = i32
        L.pflbm_set_state.argtypes = [vp, vp, ct.c_size_t]
        L.pflbm_set_state.restype = i32
        L.pflbm_export_populations.argtypes = [vp, i32, fp]
        L.pflbm_export_populations.restype = i32
        L.pflbm_num_variants.argtypes = [vp]
        L.pflbm_num_variants.restype = i32
        L.pflbm_variant_name.argtypes = [vp, i32]
        L.pflbm_variant_name.restype = ct.c_char_p
        L.pflbm_set_variant.argtypes = [vp, i32]
        L.pflbm_set_variant.restype = i32
        L.pflbm_autotune.argtypes = [vp, i32, P(i32), P(ct.c_float)]
        L.pflbm_autotune.restype = i32
        L.pflbm_set_graph.argtypes = [vp, i32]
        L.pflbm_set_graph.restype = i32
        L.pflbm_stream.argtypes = [vp]
        L.pflbm_stream.restype = vp
        L.pflbm_bytes_per_update.argtypes = [vp]
        L.pflbm_bytes_per_update.restype = ct.c_double
        L.pflbm_destroy.argtypes = [vp]
        L.pflbm_destroy.restype = i32
        L.pflbm_status_string.argtypes = [i32]
        L.pflbm_status_string.restype = ct.c_char_p
        L.pflbm_bubble_centroid_velocity_noalloc.argtypes = [vp, i32, i32, dp]
        L.pflbm_bubble_centroid_velocity_noalloc.restype = i32
        L.pflbm_check_state.argtypes = [vp]
        L.pflbm_check_state.restype = i32
        L.pflbm_case_nonfinite.argtypes = [vp, i32]
        L.pflbm_case_nonfinite.restype = i32
        _lib = L
    return _lib


def _check(where, st):
    if st != 0:
        raise PflbmError(where, st)


def workspace_bytes(cases) -> int:
    arr = (Params * len(cases))(*[make_params(c) for c in cases])
    return int(lib().pflbm_workspace_bytes(arr, len(cases)))


def _dp(a):
    return None if a is None else a.ctypes.data_as(ct.POINTER(ct.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _read_json(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


class Solver:
    """A set of domains advanced together on one GPU (one case = plain path)."""

    def __init__(self, cases, device="cuda:0", stream=None):
        import torch
        if isinstance(cases, dict):
            cases = [cases]
        self.params = [dict(c) for c in cases]
        self.torch = torch
        self.device = torch.device(device)
        L = lib()
        arr = (Params * len(cases))(*[make_params(c) for c in cases])
        nbytes = int(L.pflbm_workspace_bytes(arr, len(cases)))
        if nbytes == 0:
            raise PflbmError("pflbm_workspace_bytes", -1)
        with torch.cuda.device(self.device):
            # zeroed so that the row padding (never written by the kernels) is
            # deterministic in checkpoints taken with get_state
            self.workspace = torch.zeros(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ct.c_void_p()
        _check("pflbm_create", L.pflbm_create(arr, len(cases), ct.c_void_p(self.workspace.data_ptr()), nbytes,
                                              ct.c_void_p(self.stream.cuda_stream), ct.byref(h)))
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _check("pflbm_destroy", lib().pflbm_destroy(h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_fields(self, case_id, C, u=None, p=None):
        prm = self._case_params(case_id, "pflbm_init_fields")
        ny, nx, nh = prm["ny"], prm["nx"], prm["n_h"]
        C, u, p = _f64(C), _f64(u), _f64(p)
        # the ABI reads exactly n_h, 2 and 1 planes of (ny, nx): reject other shapes here
        for name, a, shape in (("C", C, (nh, ny, nx)), ("u", u, (2, ny, nx)), ("p", p, (ny, nx))):
            if a is not None and a.shape != shape and not (name == "C" and nh == 1 and a.shape == (ny, nx)):
                raise PflbmError(f"pflbm_init_fields: {name} has shape {a.shape}, expected {shape}", -1)
        _check("pflbm_init_fields", lib().pflbm_init_fields(self._h, int(case_id), _dp(C), _dp(u), _dp(p)))

    def check_state(self):
        """Scans every case's state; raises PflbmError(-4) if any is non-finite."""
        _check("pflbm_check_state", lib().pflbm_check_state(self._h))

    def case_nonfinite(self, case_id=0):
        """True if the case was flagged non-finite by a synchronising call."""
        r = lib().pflbm_case_nonfinite(self._h, int(case_id))
        if r < 0:
            raise PflbmError("pflbm_case_nonfinite", r)
        return bool(r)

    def step(self, n=1):
        _check("pflbm_step", lib().pflbm_step(self._h, int(n)))

    def _empty(self, *shape):
        return self.torch.empty(*shape, dtype=self.torch.float32, device=self.device)

    def _case_params(self, case_id, where):
        # output shapes come from the case; an unknown case is the ABI's INVALID_ARG
        if not 0 <= int(case_id) < len(self.params):
            raise PflbmError(where, -1)
        return self.params[int(case_id)]

    def macroscopic(self, case_id=0):
        prm = self._case_params(case_id, "pflbm_macroscopic")
        ny, nx = prm["ny"], prm["nx"]
        out = dict(rho=self._empty(ny, nx), u=self._empty(2, ny, nx), p=self._empty(ny, nx),
                   phi=self._empty(prm["n_h"], ny, nx))
        ptr = lambda t: ct.c_void_p(t.data_ptr())
        _check("pflbm_macroscopic", lib().pflbm_macroscopic(self._h, int(case_id), ptr(out["rho"]), ptr(out["u"]),
                                                            ptr(out["p"]), ptr(out["phi"])))
        return out

    def bubble_centroid_velocity(self, case_id=0, comp=0):
        out = np.empty(6)
        _check("pflbm_bubble_centroid_velocity",
               lib().pflbm_bubble_centroid_velocity(self._h, int(case_id), int(comp), _dp(out)))
        return out

    def bubble_centroid_velocity_noalloc(self, case_id=0, comp=0):
        """bubble_centroid_velocity with the reduction's scratch in the
        library's static device array (no workspace, no allocation)."""
        out = np.empty(6)
        _check("pflbm_bubble_centroid_velocity_noalloc",
               lib().pflbm_bubble_centroid_velocity_noalloc(self._h, int(case_id), int(comp), _dp(out)))
        return out

    def state_bytes(self):
        return int(lib().pflbm_state_bytes(self._h))

    def get_state(self):
        n = self.state_bytes()
        buf = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        _check("pflbm_get_state", lib().pflbm_get_state(self._h, ct.c_void_p(buf.data_ptr()), n))
        return buf

    def set_state(self, buf):
        # the ABI copies device to device: take only a contiguous byte tensor on this solver's GPU
        if (buf.device != self.device and not (buf.is_cuda and self.device.index is None)) or \
                buf.dtype != self.torch.uint8 or not buf.is_contiguous():
            raise PflbmError("pflbm_set_state: expected a contiguous uint8 tensor on " + str(self.device), -1)
        _check("pflbm_set_state", lib().pflbm_set_state(self._h, ct.c_void_p(buf.data_ptr()), buf.numel()))

    def export_populations(self, case_id=0):
        prm = self._case_params(case_id, "pflbm_export_populations")
        out = self._empty(9 + prm["n_h"] + 1, prm["ny"], prm["nx"])
        _check("pflbm_export_populations",
               lib().pflbm_export_populations(self._h, int(case_id), ct.c_void_p(out.data_ptr())))
        return out

    def variants(self):
        n = lib().pflbm_num_variants(self._h)
        names = []
        for i in range(n):
            s = lib().pflbm_variant_name(self._h, i)
            names.append(None if s is None else s.decode())
        return names

    def set_variant(self, index):
        _check("pflbm_set_variant", lib().pflbm_set_variant(self._h, int(index)))

    def autotune(self, steps=10, cache=None):
        """Pick the fastest tile variant for these cases on this GPU.  With a
        `cache` path (JSON), a previous choice for the same case shapes is
        reused instead of timing again.  Returns the chosen variant name."""
        key = None
        names = self.variants()
        if cache is not None:
            import torch
            dev = torch.cuda.get_device_properties(self.device).name
            key = json.dumps([dev, [(p["nx"], p["ny"], p["n_h"], p.get("store_h", 0), p.get("storage", 0))
                                    for p in self.params]])
            table = _read_json(cache)
            if key in table and table[key] in names:
                self.set_variant(names.index(table[key]))
                return table[key]
        n = len(names)
        ms = (ct.c_float * n)()
        best = ct.c_int32(-1)
        _check("pflbm_autotune", lib().pflbm_autotune(self._h, int(steps), ct.byref(best), ms))
        self.tuning = {names[i]: float(ms[i]) for i in range(n) if ms[i] >= 0}
        name = names[best.value]
        if cache is not None:
            table = _read_json(cache)
            table[key] = name
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        return name

    def set_graph(self, steps_per_graph):
        _check("pflbm_set_graph", lib().pflbm_set_graph(self._h, int(steps_per_graph)))

    def bytes_per_update(self):
        return float(lib().pflbm_bytes_per_update(self._h))

    def synchronize(self):
        self.stream.synchronize()
