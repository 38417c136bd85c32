"""Thin ctypes binding of the C ABI in ``include/cmlb.h``.

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libcmlb.so``.  The functions keep the C names (``cmlb_create``,
``cmlb_step``, ...); :class:`Context` wraps them for numpy users.  If the
library has not been built, :func:`load` raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcmlb.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ERANGE, ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSTABLE",
                -5: "ERANGE", -6: "ESTATE"}
FP64, FP32, FP16 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16": FP16}
BC = {"periodic": 0, "walls": 1, "moving_walls": 1}
FLOW = {"none": 0, "prescribed": 1, "coupled": 2}


class SimParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc_y", ctypes.c_int32), ("flow", ctypes.c_int32),
        ("W", ctypes.c_double), ("phi_a", ctypes.c_double), ("phi_b", ctypes.c_double),
        ("M_phi", ctypes.c_double), ("D_s", ctypes.c_double),
        ("rho_a", ctypes.c_double), ("rho_b", ctypes.c_double), ("nu_a", ctypes.c_double),
        ("nu_b", ctypes.c_double), ("omega_zeta", ctypes.c_double),
        ("sigma0", ctypes.c_double), ("beta", ctypes.c_double), ("c_max", ctypes.c_double),
        ("u_wall", ctypes.c_double), ("F_ext_x", ctypes.c_double), ("F_ext_y", ctypes.c_double),
        ("vel_period_T", ctypes.c_double),
    ]


EXPORTS = (
    "cmlb_create", "cmlb_init_fields", "cmlb_step", "cmlb_read_fields", "cmlb_inventory",
    "cmlb_inventories", "cmlb_inventories_noalloc", "cmlb_get_populations", "cmlb_set_populations", "cmlb_set_step_count", "cmlb_fault_flags",
    "cmlb_synchronize", "cmlb_set_tile_rows", "cmlb_set_tile_shape", "cmlb_launch_options",
    "cmlb_set_use_graph",
    "cmlb_set_xcd_remap", "cmlb_set_tile_order", "cmlb_set_store_policy", "cmlb_autotune",
    "cmlb_copy", "cmlb_copy_planes", "cmlb_launch_costs", "cmlb_step_count", "cmlb_num_sims",
    "cmlb_last_error", "cmlb_destroy",
)

EXPORTS3 = (
    "cmlb3_create", "cmlb3_init_fields", "cmlb3_step", "cmlb3_read_fields", "cmlb3_inventory",
    "cmlb3_get_populations", "cmlb3_set_populations", "cmlb3_fault_flags", "cmlb3_synchronize",
    "cmlb3_set_use_graph", "cmlb3_set_tile_shape", "cmlb3_launch_options",
    "cmlb3_set_store_policy", "cmlb3_autotune", "cmlb3_step_count",
    "cmlb3_last_error", "cmlb3_destroy",
)


class SimParams3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc_y", ctypes.c_int32), ("flow", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("W", ctypes.c_double), ("phi_a", ctypes.c_double), ("phi_b", ctypes.c_double),
        ("M_phi", ctypes.c_double), ("D_s", ctypes.c_double),
        ("rho_a", ctypes.c_double), ("rho_b", ctypes.c_double), ("nu_a", ctypes.c_double),
        ("nu_b", ctypes.c_double), ("omega_zeta", ctypes.c_double),
        ("sigma0", ctypes.c_double), ("beta", ctypes.c_double), ("c_max", ctypes.c_double),
        ("u_wall", ctypes.c_double), ("F_ext_x", ctypes.c_double), ("F_ext_y", ctypes.c_double),
        ("F_ext_z", ctypes.c_double), ("vel_period_T", ctypes.c_double),
    ]


_lib = None


class CmlbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libcmlb.so and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_2504_09024_amd.build` "
            "(no CPU fallback exists)")
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.cmlb_create.argtypes = [ctypes.POINTER(SimParams), ctypes.c_int32, ctypes.c_int32, vp,
                              ctypes.POINTER(vp)]
    L.cmlb_init_fields.argtypes = [vp, ctypes.c_int32, dp, dp, dp, dp, dp]
    L.cmlb_step.argtypes = [vp, ctypes.c_int32]
    L.cmlb_read_fields.argtypes = [vp, ctypes.c_int32, dp, dp, dp, dp, dp]
    L.cmlb_inventory.argtypes = [vp, ctypes.c_int32, dp, dp]
    L.cmlb_inventories.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, dp]
    L.cmlb_inventories_noalloc.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp]
    L.cmlb_get_populations.argtypes = [vp, ctypes.c_int32, dp, dp, dp]
    L.cmlb_set_populations.argtypes = [vp, ctypes.c_int32, dp, dp, dp]
    L.cmlb_set_step_count.argtypes = [vp, ctypes.c_int64]
    L.cmlb_fault_flags.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.cmlb_synchronize.argtypes = [vp]
    L.cmlb_set_tile_rows.argtypes = [vp, ctypes.c_int32]
    L.cmlb_set_tile_shape.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.cmlb_launch_options.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
    L.cmlb_set_use_graph.argtypes = [vp, ctypes.c_int32]
    L.cmlb_set_xcd_remap.argtypes = [vp, ctypes.c_int32]
    L.cmlb_set_tile_order.argtypes = [vp, ctypes.c_int32]
    L.cmlb_set_store_policy.argtypes = [vp, ctypes.c_int32]
    ip = ctypes.POINTER(ctypes.c_int32)
    L.cmlb_autotune.argtypes = [vp, ctypes.c_int32, ip, ip, ip]
    L.cmlb_copy.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, vp]
    L.cmlb_copy_planes.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, vp]
    L.cmlb_launch_costs.argtypes = [ctypes.c_int32, ctypes.c_int32, dp, dp]
    L.cmlb_step_count.argtypes = [vp]
    L.cmlb_step_count.restype = ctypes.c_int64
    L.cmlb_num_sims.argtypes = [vp]
    L.cmlb_num_sims.restype = ctypes.c_int32
    L.cmlb_last_error.argtypes = [vp]
    L.cmlb_last_error.restype = ctypes.c_char_p
    L.cmlb_destroy.argtypes = [vp]
    L.cmlb_destroy.restype = None
    for name in EXPORTS:
        if name not in ("cmlb_step_count", "cmlb_num_sims", "cmlb_last_error", "cmlb_destroy"):
            getattr(L, name).restype = ctypes.c_int
    p3 = ctypes.POINTER(SimParams3)
    L.cmlb3_create.argtypes = [p3, ctypes.c_int32, ctypes.c_int32, vp, ctypes.POINTER(vp)]
    L.cmlb3_init_fields.argtypes = [vp, ctypes.c_int32] + [dp] * 6
    L.cmlb3_step.argtypes = [vp, ctypes.c_int32]
    L.cmlb3_read_fields.argtypes = [vp, ctypes.c_int32] + [dp] * 6
    L.cmlb3_inventory.argtypes = [vp, ctypes.c_int32, dp, dp]
    L.cmlb3_get_populations.argtypes = [vp, ctypes.c_int32, dp, dp, dp]
    L.cmlb3_set_populations.argtypes = [vp, ctypes.c_int32, dp, dp, dp]
    L.cmlb3_fault_flags.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.cmlb3_synchronize.argtypes = [vp]
    L.cmlb3_set_use_graph.argtypes = [vp, ctypes.c_int32]
    L.cmlb3_set_tile_shape.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.cmlb3_set_store_policy.argtypes = [vp, ctypes.c_int32]
    L.cmlb3_launch_options.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
    L.cmlb3_autotune.argtypes = [vp, ctypes.c_int32] + [ctypes.POINTER(ctypes.c_int32)] * 3
    L.cmlb3_step_count.argtypes = [vp]
    L.cmlb3_step_count.restype = ctypes.c_int64
    L.cmlb3_last_error.argtypes = [vp]
    L.cmlb3_last_error.restype = ctypes.c_char_p
    L.cmlb3_destroy.argtypes = [vp]
    L.cmlb3_destroy.restype = None
    for name in EXPORTS3:
        if name not in ("cmlb3_step_count", "cmlb3_last_error", "cmlb3_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def device_copy(src_ptr: int, dst_ptr: int, nbytes: int, nontemporal: bool = False,
                stream=None) -> None:
    """cmlb_copy: asynchronous device-to-device copy on `stream` (a HIP
    stream handle; None = the default stream).  A measurement aid for the
    plain-copy bandwidth ceiling, not part of the method."""
    L = load()
    rc = L.cmlb_copy(ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr), int(nbytes),
                     1 if nontemporal else 0, ctypes.c_void_p(stream) if stream else None)
    if rc != 0:
        raise CmlbError(rc, "cmlb_copy")


def device_copy_planes(src_ptr: int, dst_ptr: int, plane_bytes: int, planes: int,
                       nontemporal: bool = False, stream=None) -> None:
    """cmlb_copy_planes: the same copy over `planes` (9 or 27) contiguous
    planes of plane_bytes, with one read and one write stream per plane open
    at once.  A measurement aid, not part of the method."""
    L = load()
    rc = L.cmlb_copy_planes(ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr), int(plane_bytes),
                            int(planes), 1 if nontemporal else 0,
                            ctypes.c_void_p(stream) if stream else None)
    if rc != 0:
        raise CmlbError(rc, "cmlb_copy_planes")


def launch_costs(blocks: int = 64, iters: int = 2048):
    """cmlb_launch_costs: (microseconds per grid-wide barrier in one
    cooperative launch, microseconds per kernel of a replayed graph), both
    with `blocks` workgroups of 256 threads.  A measurement aid, not part of
    the method."""
    L = load()
    a, b = ctypes.c_double(), ctypes.c_double()
    rc = L.cmlb_launch_costs(int(blocks), int(iters), ctypes.byref(a), ctypes.byref(b))
    if rc != 0:
        raise CmlbError(rc, "cmlb_launch_costs")
    return a.value, b.value


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape):
    """An FP64 C-ordered copy of `a`, which must have exactly `shape` or be
    flat with that many elements (a transposed or otherwise reshaped array
    would scramble the nodes, so any other shape raises ValueError)."""
    if a is None:
        return None
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if arr.shape != tuple(shape):
        if arr.ndim == 1 and arr.size == int(np.prod(shape)):
            arr = arr.reshape(shape)
        else:
            raise ValueError(f"array of shape {arr.shape} where {tuple(shape)} (or flat) is "
                             "expected")
    return arr


def make_params(d: dict) -> SimParams:
    p = SimParams()
    for name, _ in SimParams._fields_:
        if name not in d:
            continue
        v = d[name]
        if name == "bc_y" and isinstance(v, str):
            v = BC[v]
        if name == "flow" and isinstance(v, str):
            v = FLOW[v]
        setattr(p, name, v)
    return p


class Context:
    """A set of simulations advanced together by the HIP library.

    ``params``: list of dicts keyed by ``cmlb_sim_params`` names (strings
    accepted for ``bc_y`` and ``flow``).  ``stream``: a hipStream_t handle
    as an int (e.g. ``torch.cuda.current_stream().cuda_stream``) or None.
    """

    def __init__(self, params, precision="fp64", stream=None):
        if isinstance(params, dict):
            params = [params]
        self.L = load()
        self.params = [dict(p) for p in params]
        arr = (SimParams * len(params))(*[make_params(p) for p in params])
        self._arr = arr
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.precision = prec
        h = ctypes.c_void_p()
        rc = self.L.cmlb_create(arr, len(params), prec, ctypes.c_void_p(stream or 0),
                                ctypes.byref(h))
        if rc != OK:
            raise CmlbError(rc, "cmlb_create failed")
        self.h = h
        self.shapes = [(int(p["ny"]), int(p["nx"])) for p in self.params]
        fl = self.params[0].get("flow", 0)
        self.coupled = (FLOW[fl] if isinstance(fl, str) else fl) == 2

    def _check(self, rc, what):
        if rc != OK:
            msg = self.L.cmlb_last_error(self.h)
            raise CmlbError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "h", None):
            self.L.cmlb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def init_fields(self, sim, phi, c, ux=None, uy=None, P=None):
        sh = self.shapes[sim]
        arrs = [_f64(v, sh) for v in (phi, c, ux, uy, P)]
        self._check(self.L.cmlb_init_fields(self.h, sim, *[_dptr(a) for a in arrs]),
                    "cmlb_init_fields")

    def step(self, n=1):
        self._check(self.L.cmlb_step(self.h, int(n)), "cmlb_step")

    def read_fields(self, sim=0):
        sh = self.shapes[sim]
        out = {k: np.zeros(sh) for k in ("phi", "c", "ux", "uy", "P")}
        self._check(self.L.cmlb_read_fields(self.h, sim, _dptr(out["phi"]), _dptr(out["c"]),
                                            _dptr(out["ux"]), _dptr(out["uy"]),
                                            _dptr(out["P"])), "cmlb_read_fields")
        return out

    def inventory(self, sim=0):
        a, b = ctypes.c_double(), ctypes.c_double()
        self._check(self.L.cmlb_inventory(self.h, sim, ctypes.byref(a), ctypes.byref(b)),
                    "cmlb_inventory")
        return a.value, b.value

    def inventories(self, first=0, n=None):
        """cmlb_inventories: (total phi, total c) of simulations first ..
        first + n - 1 (all from `first` when n is None), as an (n, 2) array."""
        n = len(self.shapes) - first if n is None else int(n)
        out = np.zeros((max(n, 0), 2))
        self._check(self.L.cmlb_inventories(self.h, int(first), n, _dptr(out)),
                    "cmlb_inventories")
        return out

    def inventories_noalloc(self, d_sums, first=0, n=None):
        """cmlb_inventories_noalloc: enqueue the totals of simulations first ..
        first + n - 1 into device memory at address `d_sums` (2 n doubles,
        caller-owned); asynchronous, allocates nothing."""
        n = len(self.shapes) - first if n is None else int(n)
        self._check(self.L.cmlb_inventories_noalloc(self.h, int(first), n,
                                                     ctypes.c_void_p(int(d_sums))),
                    "cmlb_inventories_noalloc")

    def get_populations(self, sim=0):
        ny, nx = self.shapes[sim]
        f = np.zeros((9, ny, nx))
        h = np.zeros((9, ny, nx))
        g = np.zeros((9, ny, nx)) if self.coupled else None
        self._check(self.L.cmlb_get_populations(self.h, sim, _dptr(f), _dptr(h), _dptr(g)),
                    "cmlb_get_populations")
        return f, h, g

    def set_populations(self, sim, f, h, g=None):
        ny, nx = self.shapes[sim]
        f = _f64(f, (9, ny, nx))
        h = _f64(h, (9, ny, nx))
        g = _f64(g, (9, ny, nx)) if g is not None else None
        self._check(self.L.cmlb_set_populations(self.h, sim, _dptr(f), _dptr(h), _dptr(g)),
                    "cmlb_set_populations")

    def set_step_count(self, n):
        self._check(self.L.cmlb_set_step_count(self.h, int(n)), "cmlb_set_step_count")

    def fault_flags(self, sim=0):
        v = ctypes.c_int32()
        self._check(self.L.cmlb_fault_flags(self.h, sim, ctypes.byref(v)), "cmlb_fault_flags")
        return v.value

    def synchronize(self):
        self._check(self.L.cmlb_synchronize(self.h), "cmlb_synchronize")

    def set_tile_rows(self, rows):
        self._check(self.L.cmlb_set_tile_rows(self.h, int(rows)), "cmlb_set_tile_rows")

    def set_tile_shape(self, width, rows):
        self._check(self.L.cmlb_set_tile_shape(self.h, int(width), int(rows)),
                    "cmlb_set_tile_shape")

    def launch_options(self):
        """Accepted (width, rows) tile shapes."""
        buf = (ctypes.c_int32 * 64)()
        n = self.L.cmlb_launch_options(self.h, buf, 64)
        return [(buf[2 * i], buf[2 * i + 1]) for i in range(max(n, 0))]

    def set_use_graph(self, on):
        self._check(self.L.cmlb_set_use_graph(self.h, 1 if on else 0), "cmlb_set_use_graph")

    def set_store_policy(self, policy):
        """0 auto, 1 default stores, 2 non-temporal stores (or "auto",
        "default", "nt")."""
        if isinstance(policy, str):
            policy = {"auto": 0, "default": 1, "nt": 2}[policy]
        self._check(self.L.cmlb_set_store_policy(self.h, int(policy)), "cmlb_set_store_policy")

    def autotune(self, steps=20):
        """Time every launch option on these simulations (state restored);
        keeps and returns the fastest as (width, rows, store policy)."""
        w, r, p = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.L.cmlb_autotune(self.h, int(steps), ctypes.byref(w), ctypes.byref(r),
                                         ctypes.byref(p)), "cmlb_autotune")
        return w.value, r.value, {1: "default", 2: "nt"}[p.value]

    def set_tile_order(self, group):
        self._check(self.L.cmlb_set_tile_order(self.h, int(group)), "cmlb_set_tile_order")

    def set_xcd_remap(self, on):
        self._check(self.L.cmlb_set_xcd_remap(self.h, 1 if on else 0), "cmlb_set_xcd_remap")

    @property
    def step_count(self):
        return self.L.cmlb_step_count(self.h)


def make_params3(d: dict) -> SimParams3:
    p = SimParams3()
    for name, _ in SimParams3._fields_:
        if name not in d:
            continue
        v = d[name]
        if name == "bc_y" and isinstance(v, str):
            v = BC[v]
        if name == "flow" and isinstance(v, str):
            v = FLOW[v]
        setattr(p, name, v)
    return p


class Context3:
    """A set of 3D (D3Q27) simulations advanced together by the HIP library.
    ``params``: dicts keyed by ``cmlb3_sim_params`` names.  Fields are numpy
    arrays [nz][ny][nx]; populations [27][nz][ny][nx]."""

    def __init__(self, params, precision="fp64", stream=None):
        if isinstance(params, dict):
            params = [params]
        self.L = load()
        self.params = [dict(p) for p in params]
        arr = (SimParams3 * len(params))(*[make_params3(p) for p in params])
        self._arr = arr
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        h = ctypes.c_void_p()
        rc = self.L.cmlb3_create(arr, len(params), prec, ctypes.c_void_p(stream or 0),
                                 ctypes.byref(h))
        if rc != OK:
            raise CmlbError(rc, "cmlb3_create failed")
        self.h = h
        self.shapes = [(int(p["nz"]), int(p["ny"]), int(p["nx"])) for p in self.params]
        fl = self.params[0].get("flow", 0)
        self.coupled = (FLOW[fl] if isinstance(fl, str) else fl) == 2

    def _check(self, rc, what):
        if rc != OK:
            msg = self.L.cmlb3_last_error(self.h)
            raise CmlbError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "h", None):
            self.L.cmlb3_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_fields(self, sim, phi, c, ux=None, uy=None, uz=None, P=None):
        sh = self.shapes[sim]
        arrs = [_f64(v, sh) for v in (phi, c, ux, uy, uz, P)]
        self._check(self.L.cmlb3_init_fields(self.h, sim, *[_dptr(a) for a in arrs]),
                    "cmlb3_init_fields")

    def step(self, n=1):
        self._check(self.L.cmlb3_step(self.h, int(n)), "cmlb3_step")

    def read_fields(self, sim=0):
        sh = self.shapes[sim]
        out = {k: np.zeros(sh) for k in ("phi", "c", "ux", "uy", "uz", "P")}
        self._check(self.L.cmlb3_read_fields(self.h, sim, *[_dptr(out[k]) for k in (
            "phi", "c", "ux", "uy", "uz", "P")]), "cmlb3_read_fields")
        return out

    def inventory(self, sim=0):
        a, b = ctypes.c_double(), ctypes.c_double()
        self._check(self.L.cmlb3_inventory(self.h, sim, ctypes.byref(a), ctypes.byref(b)),
                    "cmlb3_inventory")
        return a.value, b.value

    def get_populations(self, sim=0):
        sh = (27,) + self.shapes[sim]
        f, h = np.zeros(sh), np.zeros(sh)
        g = np.zeros(sh) if self.coupled else None
        self._check(self.L.cmlb3_get_populations(self.h, sim, _dptr(f), _dptr(h), _dptr(g)),
                    "cmlb3_get_populations")
        return f, h, g

    def set_populations(self, sim, f, h, g=None):
        sh = (27,) + self.shapes[sim]
        f, h = _f64(f, sh), _f64(h, sh)
        g = _f64(g, sh) if g is not None else None
        self._check(self.L.cmlb3_set_populations(self.h, sim, _dptr(f), _dptr(h), _dptr(g)),
                    "cmlb3_set_populations")

    def fault_flags(self, sim=0):
        v = ctypes.c_int32()
        self._check(self.L.cmlb3_fault_flags(self.h, sim, ctypes.byref(v)), "cmlb3_fault_flags")
        return v.value

    def synchronize(self):
        self._check(self.L.cmlb3_synchronize(self.h), "cmlb3_synchronize")

    def set_use_graph(self, on):
        self._check(self.L.cmlb3_set_use_graph(self.h, 1 if on else 0), "cmlb3_set_use_graph")

    def set_store_policy(self, policy):
        """0 auto, 1 default stores, 2 non-temporal stores (or "auto",
        "default", "nt")."""
        if isinstance(policy, str):
            policy = {"auto": 0, "default": 1, "nt": 2}[policy]
        self._check(self.L.cmlb3_set_store_policy(self.h, int(policy)), "cmlb3_set_store_policy")

    def set_tile_shape(self, ty, zs):
        """Collision columns of 64 x ty nodes marching through zs planes."""
        self._check(self.L.cmlb3_set_tile_shape(self.h, int(ty), int(zs)), "cmlb3_set_tile_shape")

    def launch_options(self):
        buf = (ctypes.c_int32 * 32)()
        n = self.L.cmlb3_launch_options(self.h, buf, 32)
        return [(buf[2 * i], buf[2 * i + 1]) for i in range(max(n, 0))]

    def autotune(self, steps=20):
        """cmlb3_autotune: time every collision shape under both store
        policies on these simulations (state restored); keeps and returns
        the fastest as (ty, zs, store policy)."""
        ty, zs, p = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.L.cmlb3_autotune(self.h, int(steps), ctypes.byref(ty), ctypes.byref(zs),
                                          ctypes.byref(p)), "cmlb3_autotune")
        return ty.value, zs.value, {1: "default", 2: "nt"}[p.value]

    @property
    def step_count(self):
        return self.L.cmlb3_step_count(self.h)
