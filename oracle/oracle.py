"""Python binding of the FP64 CPU oracle (rlb_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rlb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

Q = 19
BC_PERIODIC, BC_FIXED, BC_OUTFLOW = 0, 1, 2
TAU_UNIFORM, TAU_ETA_OVER_S = 0, 1
DENSW_PAPER, DENSW_ISOTROPIC = 0, 1
FLUX_MINMOD, FLUX_RUSANOV = 0, 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle into oracle/liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("nu", ctypes.c_double), ("dt", ctypes.c_double),
        ("euler", ctypes.c_int), ("tau_mode", ctypes.c_int),
        ("tau", ctypes.c_double), ("eta_over_s", ctypes.c_double),
        ("alpha", ctypes.c_double), ("with_h", ctypes.c_int),
        ("bc", ctypes.c_int * 6), ("face", (ctypes.c_double * 5) * 6),
        ("guard_umax", ctypes.c_double), ("guard_efloor", ctypes.c_double),
        ("basic", ctypes.c_int), ("dens_w", ctypes.c_int), ("flux", ctypes.c_int),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    L = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_lattice.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                              dp, dp, dp]
    L.orc_feq.argtypes = [ctypes.c_double, ctypes.c_int] + [ctypes.c_double] * 4 + [dp]
    L.orc_heq.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 4 + [dp]
    L.orc_moments.argtypes = [ctypes.c_double, ctypes.c_int, dp, dp, dp, dp]
    L.orc_recover.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int, dp]
    L.orc_recover.restype = ctypes.c_int
    L.orc_create.argtypes = [ctypes.POINTER(_Cfg)]
    L.orc_create.restype = ctypes.c_void_p
    L.orc_destroy.argtypes = [ctypes.c_void_p]
    L.orc_init.argtypes = [ctypes.c_void_p, dp, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_uint8)]
    L.orc_init.restype = ctypes.c_int
    L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    L.orc_step.restype = ctypes.c_int64
    L.orc_fields.argtypes = [ctypes.c_void_p, dp, dp, dp, dp, dp]
    L.orc_get_pops.argtypes = [ctypes.c_void_p, dp, dp]
    L.orc_set_pops.argtypes = [ctypes.c_void_p, dp, dp, dp]
    L.orc_get_hist.argtypes = [ctypes.c_void_p, dp]
    L.orc_guard_events.argtypes = [ctypes.c_void_p]
    L.orc_guard_events.restype = ctypes.c_int64
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_set_num_threads.argtypes = [ctypes.c_int]
    L.orc_set_num_threads.restype = None
    _lib = L
    return L


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def lattice(nu: float, basic: bool = False, density_weights: int = 0):
    """(e[19,3] int, xi[19,4], w[19], w'[19]) in the oracle's own order; the
    extended set (Sec. II.A) or, with basic=True, the basic set (Sec. II);
    density_weights: DENSW_PAPER (Eqs. (59)-(60)) or DENSW_ISOTROPIC."""
    L = _load()
    e = np.zeros((Q, 3), dtype=np.int32)
    xi = np.zeros((Q, 4))
    w = np.zeros(Q)
    wp = np.zeros(Q)
    L.orc_lattice(nu, int(basic), int(density_weights), e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                  _p(xi), _p(w), _p(wp))
    return e.astype(np.int64), xi, w, wp


def feq(nu, eps, ux, uy, uz, basic: bool = False) -> np.ndarray:
    out = np.zeros(Q)
    _load().orc_feq(nu, int(basic), eps, ux, uy, uz, _p(out))
    return out


def heq(nu, n, ux, uy, uz, basic: bool = False, density_weights: int = 0) -> np.ndarray:
    out = np.zeros(Q)
    _load().orc_heq(nu, int(basic), int(density_weights), n, ux, uy, uz, _p(out))
    return out


def moments(nu, f, h=None, basic: bool = False):
    f = _f64(f)
    h = None if h is None else _f64(h)
    T0 = np.zeros(4)
    N0 = np.zeros(1)
    _load().orc_moments(nu, int(basic), _p(f), _p(h), _p(T0), _p(N0))
    return T0, float(N0[0])


def recover(T0, N0, with_h=True):
    out = np.zeros(5)
    rc = _load().orc_recover(float(T0[0]), float(T0[1]), float(T0[2]), float(T0[3]),
                             float(N0), int(with_h), _p(out))
    return rc, out


@dataclass
class Config:
    nx: int
    ny: int = 1
    nz: int = 1
    nu: float = 27.0 ** 0.25
    dt: float = 0.25
    euler: bool = False
    tau_mode: int = TAU_UNIFORM
    tau: float = 1.0
    eta_over_s: float = 0.0
    alpha: float = 0.0
    with_h: bool = False
    bc: Sequence[int] = (BC_PERIODIC,) * 6
    face: Sequence[Sequence[float]] = field(default_factory=lambda: [[3.0, 0, 0, 0, 1.0]] * 6)
    guard_umax: float = 0.0
    guard_efloor: float = 1e-10
    basic: bool = False  # the basic model of Sec. II (dt, euler, alpha, guard unused/off)
    density_weights: int = 0  # DENSW_PAPER | DENSW_ISOTROPIC (extended set)
    flux: int = 0  # FLUX_MINMOD (Eqs. (47)-(53)) | FLUX_RUSANOV (extended set)

    def _c(self) -> _Cfg:
        c = _Cfg()
        c.nx, c.ny, c.nz = self.nx, self.ny, self.nz
        c.nu, c.dt = self.nu, self.dt
        c.euler = int(self.euler)
        c.tau_mode = int(self.tau_mode)
        c.tau, c.eta_over_s, c.alpha = self.tau, self.eta_over_s, self.alpha
        c.with_h = int(self.with_h)
        for k in range(6):
            c.bc[k] = int(self.bc[k])
            for j in range(5):
                c.face[k][j] = float(self.face[k][j])
        c.guard_umax, c.guard_efloor = self.guard_umax, self.guard_efloor
        c.basic = int(self.basic)
        c.dens_w = int(self.density_weights)
        c.flux = int(self.flux)
        return c


class OracleError(RuntimeError):
    pass


class Oracle:
    """Whole-domain FP64 stepper.  Arrays are C-order [z][y][x]."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        self._L = _load()
        self._cc = cfg._c()
        h = self._L.orc_create(ctypes.byref(self._cc))
        if not h:
            raise OracleError("invalid oracle configuration")
        self._h = ctypes.c_void_p(h)
        self.shape = (cfg.nz, cfg.ny, cfg.nx)
        self.ncell = cfg.nx * cfg.ny * cfg.nz

    def close(self):
        if self._h:
            self._L.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, eps, ux, uy, uz, n=None, obstacle=None):
        a = [_f64(v).reshape(-1) for v in (eps, ux, uy, uz)]
        nn = None if n is None else _f64(n).reshape(-1)
        ob = None
        if obstacle is not None:
            ob = np.ascontiguousarray(np.asarray(obstacle, dtype=np.uint8).reshape(-1))
        rc = self._L.orc_init(self._h, _p(a[0]), _p(a[1]), _p(a[2]), _p(a[3]), _p(nn),
                              None if ob is None else ob.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        if rc != 0:
            raise OracleError("inadmissible initial fields")

    def step(self, nsteps: int) -> int:
        """Returns 0, or 1 + index of the first step that met an inadmissible state."""
        return int(self._L.orc_step(self._h, int(nsteps)))

    def fields(self):
        out = [np.zeros(self.ncell) for _ in range(5)]
        self._L.orc_fields(self._h, *[_p(o) for o in out])
        return [o.reshape(self.shape) for o in out]

    def pops(self):
        f = np.zeros((Q, self.ncell))
        h = np.zeros((Q, self.ncell)) if self.cfg.with_h else None
        self._L.orc_get_pops(self._h, _p(f), _p(h))
        return f, h

    def set_pops(self, f, h=None, hist=None):
        f = _f64(f).reshape(Q, self.ncell)
        h = None if h is None else _f64(h).reshape(Q, self.ncell)
        hist = None if hist is None else _f64(hist).reshape(5, self.ncell)
        self._L.orc_set_pops(self._h, _p(f), _p(h), _p(hist))

    def hist(self):
        out = np.zeros((5, self.ncell))
        self._L.orc_get_hist(self._h, _p(out))
        return out

    @property
    def guard_events(self) -> int:
        return int(self._L.orc_guard_events(self._h))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's later parallel regions (timing only)."""
    _load().orc_set_num_threads(int(n))
