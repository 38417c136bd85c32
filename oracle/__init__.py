"""Plain FP64 CPU oracle of the coupled central-moment LB step (arXiv 2504.09024).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline
leg of the benchmark may load it; the GPU library never does.  It shares no code
with the GPU library.  The arithmetic lives in ``cmlb_oracle.c`` (plain C, FP64,
central moments by their definition sum, back-transform by a 9x9 linear solve);
this module only marshals numpy arrays through ctypes.

Parity status of each function is recorded in the test files that pin it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names a build of the same sources with a planted mistake
# (-DORACLE_PLANT=k); only the test of the pins themselves sets it.
PLANTED_LIB = os.environ.get("ORACLE_LIB")
LIB_PATH = PLANTED_LIB or os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "cmlb_oracle.c")
SRC3 = os.path.join(HERE, "cmlb3_oracle.c")
SOURCES = (SRC, SRC3, os.path.join(HERE, "cmlb_oracle.h"), os.path.join(HERE, "cmlb3_oracle.h"))

FLOW_NONE, FLOW_PRESCRIBED, FLOW_COUPLED = 0, 1, 2
DIAG_NAMES = (
    "phi", "c", "P_hat", "rho", "nu", "gphix", "gphiy", "nx", "ny", "theta", "theta_c",
    "curv", "gcx", "gcy", "gpsix", "gpsiy", "sigma", "fsx", "fsy", "ux", "uy", "P",
)


def build(verbose: bool = False, plant: int = 0, out: str | None = None) -> str:
    """Compile the oracle with gcc (OpenMP over rows; results do not depend on
    the thread count because no value is reduced across threads).  ``plant``
    builds a copy with planted mistake ``plant`` into ``out`` instead."""
    path = out or os.path.join(HERE, "liboracle.so")
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-D_GNU_SOURCE",
           "-Wall", f"-DORACLE_PLANT={int(plant)}", SRC, SRC3, "-o", path + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(path + ".tmp", path)
    return path


class OParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("walls", ctypes.c_int32),
        ("flow", ctypes.c_int32), ("force_abs_grad", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("W", ctypes.c_double), ("phi_a", ctypes.c_double), ("phi_b", ctypes.c_double),
        ("M_phi", ctypes.c_double), ("D_s", ctypes.c_double),
        ("rho_a", ctypes.c_double), ("rho_b", ctypes.c_double), ("nu_a", ctypes.c_double),
        ("nu_b", ctypes.c_double), ("omega_zeta", ctypes.c_double),
        ("sigma0", ctypes.c_double), ("beta", ctypes.c_double), ("c_max", ctypes.c_double),
        ("u_wall", ctypes.c_double), ("F_ext_x", ctypes.c_double), ("F_ext_y", ctypes.c_double),
        ("vel_period_T", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not PLANTED_LIB and (not os.path.exists(LIB_PATH) or any(
                os.path.getmtime(LIB_PATH) < os.path.getmtime(f) for f in SOURCES)):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(OParams)
        L.o_num_threads.restype = ctypes.c_int
        L.o_central_moments.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.o_populations_from_central.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.o_weights.argtypes = [dp]
        L.o_directions.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.o_langmuir.argtypes = [ctypes.c_double] * 4
        L.o_langmuir.restype = ctypes.c_double
        L.o_omega_from_transport.argtypes = [ctypes.c_double]
        L.o_omega_from_transport.restype = ctypes.c_double
        L.o_collide_scalar.argtypes = [dp] + [ctypes.c_double] * 6 + [dp]
        L.o_collide_flow.argtypes = [dp] + [ctypes.c_double] * 10 + [dp]
        L.o_check_params.argtypes = [pp]
        L.o_init.argtypes = [pp] + [dp] * 8
        L.o_step.argtypes = [pp, ctypes.c_int64, dp, dp, dp, dp, dp, dp, dp, dp]
        L.o_run.argtypes = [pp, ctypes.c_int64, ctypes.c_int64, dp, dp, dp, dp, dp]
        L.o_fields.argtypes = [pp, ctypes.c_int64, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.o_node_diag.argtypes = [pp, ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_int,
                                  ctypes.c_int, dp]
        _declare3(L)
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


# ---- single-node functions -------------------------------------------------

def num_threads() -> int:
    return int(lib().o_num_threads())


def central_moments(q, ux, uy):
    q = _vec(q)
    out = np.zeros(9)
    lib().o_central_moments(_ptr(q), ux, uy, _ptr(out))
    return out


def populations_from_central(kappa, ux, uy):
    k = _vec(kappa)
    out = np.zeros(9)
    rc = lib().o_populations_from_central(_ptr(k), ux, uy, _ptr(out))
    if rc != 0:
        raise ValueError("singular moment system")
    return out


def weights():
    out = np.zeros(9)
    lib().o_weights(_ptr(out))
    return out


def directions():
    ex = (ctypes.c_int * 9)()
    ey = (ctypes.c_int * 9)()
    lib().o_directions(ex, ey)
    return np.array(list(ex)), np.array(list(ey))


def langmuir(sigma0, beta, c_max, c):
    return lib().o_langmuir(sigma0, beta, c_max, c)


def omega_from_transport(coeff):
    return lib().o_omega_from_transport(coeff)


def collide_scalar(q, ux, uy, s, jx, jy, omega1):
    q = _vec(q)
    out = np.zeros(9)
    lib().o_collide_scalar(_ptr(q), ux, uy, s, jx, jy, omega1, _ptr(out))
    return out


def collide_flow(g, ux, uy, P, rho, fpx, fpy, ftx, fty, omega_zeta, omega_nu):
    g = _vec(g)
    out = np.zeros(9)
    lib().o_collide_flow(_ptr(g), ux, uy, P, rho, fpx, fpy, ftx, fty, omega_zeta, omega_nu,
                         _ptr(out))
    return out


# ---- whole-grid simulation ------------------------------------------------

PARAM_KEYS = [f[0] for f in OParams._fields_ if f[0] not in ("pad_",)]


def make_params(**kw) -> OParams:
    """Build the oracle's parameter block.  Keys follow the library's
    parameter names; ``bc_y`` ("periodic"/"walls") and ``flow``
    ("none"/"prescribed"/"coupled") may be given as strings."""
    p = OParams()
    d = dict(kw)
    bc = d.pop("bc_y", None)
    if bc is not None:
        d["walls"] = 1 if bc in ("walls", "moving_walls", 1) else 0
    fl = d.pop("flow", None)
    if fl is not None:
        d["flow"] = {"none": 0, "prescribed": 1, "coupled": 2}.get(fl, fl)
    for k, v in d.items():
        if k not in PARAM_KEYS:
            continue
        setattr(p, k, v)
    return p


class OracleSim:
    """One simulation held as FP64 numpy population arrays [9][ny][nx]."""

    def __init__(self, params: OParams, phi, c, ux=None, uy=None, P=None):
        self.p = params
        rc = lib().o_check_params(ctypes.byref(params))
        if rc != 0:
            raise ValueError(f"invalid oracle parameters (code {rc})")
        nx, ny = params.nx, params.ny
        shape = (9, ny, nx)
        self.f = np.zeros(shape)
        self.h = np.zeros(shape)
        self.coupled = params.flow == FLOW_COUPLED
        self.g = np.zeros(shape) if self.coupled else None
        phi = _vec(phi).reshape(ny, nx)
        c = _vec(c).reshape(ny, nx)
        ux = None if ux is None else _vec(ux).reshape(ny, nx)
        uy = None if uy is None else _vec(uy).reshape(ny, nx)
        P = None if P is None else _vec(P).reshape(ny, nx)
        if params.flow == FLOW_PRESCRIBED:
            self.ux_shape = ux if ux is not None else np.zeros((ny, nx))
            self.uy_shape = uy if uy is not None else np.zeros((ny, nx))
        else:
            self.ux_shape = self.uy_shape = None
        rc = lib().o_init(ctypes.byref(params), _ptr(phi), _ptr(c), _ptr(ux), _ptr(uy), _ptr(P),
                          _ptr(self.f), _ptr(self.h), _ptr(self.g))
        if rc != 0:
            raise RuntimeError(f"oracle init failed ({rc})")
        self.t = 0

    @classmethod
    def from_populations(cls, params, f, h, g=None, t=0, ux_shape=None, uy_shape=None):
        self = cls.__new__(cls)
        self.p = params
        self.f = np.ascontiguousarray(f, dtype=np.float64).copy()
        self.h = np.ascontiguousarray(h, dtype=np.float64).copy()
        self.coupled = params.flow == FLOW_COUPLED
        self.g = None if g is None else np.ascontiguousarray(g, dtype=np.float64).copy()
        self.ux_shape = None if ux_shape is None else _vec(ux_shape)
        self.uy_shape = None if uy_shape is None else _vec(uy_shape)
        self.t = t
        return self

    def run(self, nsteps: int) -> int:
        fault = lib().o_run(ctypes.byref(self.p), self.t, nsteps, _ptr(self.ux_shape),
                            _ptr(self.uy_shape), _ptr(self.f), _ptr(self.h), _ptr(self.g))
        self.t += nsteps
        return fault

    def fields(self):
        ny, nx = self.p.ny, self.p.nx
        out = {k: np.zeros((ny, nx)) for k in ("phi", "c", "ux", "uy", "P")}
        fault = lib().o_fields(ctypes.byref(self.p), self.t, _ptr(self.ux_shape),
                               _ptr(self.uy_shape), _ptr(self.f), _ptr(self.h), _ptr(self.g),
                               _ptr(out["phi"]), _ptr(out["c"]), _ptr(out["ux"]),
                               _ptr(out["uy"]), _ptr(out["P"]))
        out["fault"] = fault
        return out

    def inventory(self):
        """Correctly rounded FP64 totals of phi and c (math.fsum)."""
        import math
        return math.fsum(self.f.ravel()), math.fsum(self.h.ravel())

    def diag(self, x, y):
        out = np.zeros(len(DIAG_NAMES))
        lib().o_node_diag(ctypes.byref(self.p), self.t, _ptr(self.ux_shape),
                          _ptr(self.uy_shape), _ptr(self.f), _ptr(self.h), _ptr(self.g), x, y,
                          _ptr(out))
        return dict(zip(DIAG_NAMES, out))


# ---- three-dimensional (D3Q27) form ----------------------------------------

class OParams3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("walls", ctypes.c_int32), ("flow", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("W", ctypes.c_double), ("phi_a", ctypes.c_double), ("phi_b", ctypes.c_double),
        ("M_phi", ctypes.c_double), ("D_s", ctypes.c_double),
        ("rho_a", ctypes.c_double), ("rho_b", ctypes.c_double), ("nu_a", ctypes.c_double),
        ("nu_b", ctypes.c_double), ("omega_zeta", ctypes.c_double),
        ("sigma0", ctypes.c_double), ("beta", ctypes.c_double), ("c_max", ctypes.c_double),
        ("u_wall", ctypes.c_double), ("F_ext_x", ctypes.c_double), ("F_ext_y", ctypes.c_double),
        ("F_ext_z", ctypes.c_double), ("vel_period_T", ctypes.c_double),
    ]


def _declare3(L):
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    pp = ctypes.POINTER(OParams3)
    L.o3_directions.argtypes = [ip, ip, ip]
    L.o3_weights.argtypes = [dp]
    L.o3_central_moments.argtypes = [dp, dp, dp]
    L.o3_populations_from_central.argtypes = [dp, dp, dp]
    L.o3_populations_from_central_solve.argtypes = [dp, dp, dp]
    L.o3_collide_scalar.argtypes = [dp, dp, ctypes.c_double, dp, ctypes.c_double, dp]
    L.o3_collide_flow.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, dp, dp,
                                  ctypes.c_double, ctypes.c_double, dp]
    L.o3_check_params.argtypes = [pp]
    L.o3_init.argtypes = [pp] + [dp] * 9
    L.o3_step.argtypes = [pp, ctypes.c_int64] + [dp] * 7
    L.o3_run.argtypes = [pp, ctypes.c_int64, ctypes.c_int64] + [dp] * 4
    L.o3_fields.argtypes = [pp, ctypes.c_int64] + [dp] * 10


PARAM_KEYS3 = [f[0] for f in OParams3._fields_ if f[0] != "pad_"]


def make_params3(**kw) -> OParams3:
    """Parameter block of the 3D oracle (keys as the library's; ``bc_y`` and
    ``flow`` may be strings)."""
    p = OParams3()
    d = dict(kw)
    bc = d.pop("bc_y", None)
    if bc is not None:
        d["walls"] = 1 if bc in ("walls", "moving_walls", 1) else 0
    fl = d.pop("flow", None)
    if fl is not None:
        d["flow"] = {"none": 0, "prescribed": 1, "coupled": 2}.get(fl, fl)
    for k, v in d.items():
        if k in PARAM_KEYS3:
            setattr(p, k, v)
    return p


def directions3():
    ex, ey, ez = ((ctypes.c_int * 27)() for _ in range(3))
    lib().o3_directions(ex, ey, ez)
    return np.array(list(ex)), np.array(list(ey)), np.array(list(ez))


def weights3():
    out = np.zeros(27)
    lib().o3_weights(_ptr(out))
    return out


def central_moments3(q, u):
    q, u = _vec(q), _vec(u)
    out = np.zeros(27)
    lib().o3_central_moments(_ptr(q), _ptr(u), _ptr(out))
    return out


def populations_from_central3(kappa, u, solve=False):
    k, u = _vec(kappa), _vec(u)
    out = np.zeros(27)
    if solve:
        if lib().o3_populations_from_central_solve(_ptr(k), _ptr(u), _ptr(out)) != 0:
            raise ValueError("singular moment system")
    else:
        lib().o3_populations_from_central(_ptr(k), _ptr(u), _ptr(out))
    return out


def collide_scalar3(q, u, s, j, omega1):
    q, u, j = _vec(q), _vec(u), _vec(j)
    out = np.zeros(27)
    lib().o3_collide_scalar(_ptr(q), _ptr(u), s, _ptr(j), omega1, _ptr(out))
    return out


def collide_flow3(g, u, P, rho, fp, ft, omega_zeta, omega_nu):
    g, u, fp, ft = _vec(g), _vec(u), _vec(fp), _vec(ft)
    out = np.zeros(27)
    lib().o3_collide_flow(_ptr(g), _ptr(u), P, rho, _ptr(fp), _ptr(ft), omega_zeta, omega_nu,
                          _ptr(out))
    return out


class OracleSim3:
    """One 3D simulation as FP64 numpy population arrays [27][nz][ny][nx]."""

    def __init__(self, params: OParams3, phi, c, ux=None, uy=None, uz=None, P=None):
        self.p = params
        rc = lib().o3_check_params(ctypes.byref(params))
        if rc != 0:
            raise ValueError(f"invalid oracle parameters (code {rc})")
        sh = (params.nz, params.ny, params.nx)
        self.f = np.zeros((27,) + sh)
        self.h = np.zeros((27,) + sh)
        self.coupled = params.flow == FLOW_COUPLED
        self.g = np.zeros((27,) + sh) if self.coupled else None
        arrs = [None if a is None else _vec(a).reshape(sh) for a in (phi, c, ux, uy, uz, P)]
        if params.flow == FLOW_PRESCRIBED:
            self.ushape = np.ascontiguousarray(np.stack(
                [a if a is not None else np.zeros(sh) for a in arrs[2:5]]))
        else:
            self.ushape = None
        rc = lib().o3_init(ctypes.byref(params), *[_ptr(a) for a in arrs], _ptr(self.f),
                           _ptr(self.h), _ptr(self.g))
        if rc != 0:
            raise RuntimeError(f"oracle init failed ({rc})")
        self.t = 0

    @classmethod
    def from_populations(cls, params, f, h, g=None, t=0, ushape=None):
        self = cls.__new__(cls)
        self.p = params
        self.f = np.ascontiguousarray(f, dtype=np.float64).copy()
        self.h = np.ascontiguousarray(h, dtype=np.float64).copy()
        self.coupled = params.flow == FLOW_COUPLED
        self.g = None if g is None else np.ascontiguousarray(g, dtype=np.float64).copy()
        self.ushape = None if ushape is None else _vec(ushape)
        self.t = t
        return self

    def run(self, nsteps: int) -> int:
        fault = lib().o3_run(ctypes.byref(self.p), self.t, nsteps, _ptr(self.ushape),
                             _ptr(self.f), _ptr(self.h), _ptr(self.g))
        self.t += nsteps
        return fault

    def fields(self):
        sh = (self.p.nz, self.p.ny, self.p.nx)
        out = {k: np.zeros(sh) for k in ("phi", "c", "ux", "uy", "uz", "P")}
        fault = lib().o3_fields(ctypes.byref(self.p), self.t, _ptr(self.ushape), _ptr(self.f),
                                _ptr(self.h), _ptr(self.g), _ptr(out["phi"]), _ptr(out["c"]),
                                _ptr(out["ux"]), _ptr(out["uy"]), _ptr(out["uz"]),
                                _ptr(out["P"]))
        out["fault"] = fault
        return out

    def inventory(self):
        import math
        return math.fsum(self.f.ravel()), math.fsum(self.h.ravel())
