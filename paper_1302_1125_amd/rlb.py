"""Python binding of librlb.so (include/rlb.h): argument marshalling only.

Every step of the update runs in the HIP kernels of the library.  There is no
CPU fallback: importing works anywhere, but creating a context needs the
built library and a gfx950 device, and fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librlb.so")

RLB_OK = 0
RLB_E_INVALID_ARG = -1
RLB_E_OUT_OF_MEMORY = -2
RLB_E_DEVICE = -3
RLB_E_INADMISSIBLE = -4
RLB_E_STATE = -5

RLB_FP64, RLB_MIXED = 0, 1
RLB_COLL_IMPLICIT, RLB_COLL_EULER = 0, 1
RLB_TAU_UNIFORM, RLB_TAU_ETA_OVER_S = 0, 1
RLB_BC_PERIODIC, RLB_BC_FIXED, RLB_BC_OUTFLOW = 0, 1, 2
RLB_LATTICE_EXTENDED, RLB_LATTICE_BASIC = 0, 1
RLB_DENSW_PAPER, RLB_DENSW_ISOTROPIC = 0, 1
RLB_FLUX_MINMOD, RLB_FLUX_RUSANOV = 0, 1

EXPORTED = [
    "rlb_config_default", "rlb_create", "rlb_init_fields", "rlb_step", "rlb_step_async",
    "rlb_sync", "rlb_moments", "rlb_stats_get", "rlb_destroy", "rlb_status_str",
    "rlb_last_error", "rlb_footprint_bytes", "rlb_steps_per_launch", "rlb_moments_noalloc",
]


class rlb_config(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("collision", ctypes.c_int32),
        ("tau_mode", ctypes.c_int32), ("with_density", ctypes.c_int32),
        ("nu", ctypes.c_double), ("dt_over_dx", ctypes.c_double), ("tau", ctypes.c_double),
        ("eta_over_s", ctypes.c_double), ("alpha", ctypes.c_double),
        ("bc", ctypes.c_int32 * 6), ("face_states", (ctypes.c_double * 5) * 6),
        ("guard_umax", ctypes.c_double), ("guard_efloor", ctypes.c_double),
        ("lattice", ctypes.c_int32), ("density_weights", ctypes.c_int32), ("flux", ctypes.c_int32),
    ]


class rlb_stats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64), ("guard_events", ctypes.c_int64),
        ("first_bad_step", ctypes.c_int64),
        ("sum_T00", ctypes.c_double), ("sum_T0x", ctypes.c_double),
        ("sum_T0y", ctypes.c_double), ("sum_T0z", ctypes.c_double), ("sum_N0", ctypes.c_double),
    ]


class RLBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librlb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RLBError(RLB_E_DEVICE, f"HIP library not built: {path} (run __graft_entry__.build())")
    try:
        # Load torch's HIP runtime first (same soname), so that the process
        # holds a single runtime and torch streams can be handed to the library.
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    L.rlb_config_default.argtypes = [ctypes.POINTER(rlb_config)]
    L.rlb_create.argtypes = [ctypes.POINTER(rlb_config), vp, ctypes.POINTER(vp)]
    L.rlb_init_fields.argtypes = [vp, dp, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_uint8)]
    L.rlb_step.argtypes = [vp, ctypes.c_int64]
    L.rlb_step_async.argtypes = [vp, ctypes.c_int64]
    L.rlb_sync.argtypes = [vp]
    L.rlb_moments.argtypes = [vp, dp, dp, dp, dp, dp]
    L.rlb_moments_noalloc.argtypes = [vp, dp, dp, dp, dp, dp]
    L.rlb_stats_get.argtypes = [vp, ctypes.POINTER(rlb_stats)]
    L.rlb_destroy.argtypes = [vp]
    L.rlb_destroy.restype = None
    L.rlb_status_str.argtypes = [ctypes.c_int]
    L.rlb_status_str.restype = ctypes.c_char_p
    L.rlb_last_error.argtypes = []
    L.rlb_last_error.restype = ctypes.c_char_p
    L.rlb_footprint_bytes.argtypes = [ctypes.POINTER(rlb_config)]
    L.rlb_footprint_bytes.restype = ctypes.c_uint64
    L.rlb_steps_per_launch.argtypes = [vp]
    L.rlb_steps_per_launch.restype = ctypes.c_int32
    for name in ("rlb_config_default", "rlb_create", "rlb_init_fields", "rlb_step",
                 "rlb_step_async", "rlb_sync", "rlb_moments", "rlb_moments_noalloc",
                 "rlb_stats_get"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != RLB_OK:
        L = load()
        raise RLBError(status, f"{L.rlb_status_str(status).decode()}: {L.rlb_last_error().decode()}")


def _dp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64)).reshape(-1)


def rlb_config_default() -> rlb_config:
    c = rlb_config()
    _check(load().rlb_config_default(ctypes.byref(c)))
    return c


def config_from(nx, ny=1, nz=1, precision=RLB_FP64, collision=RLB_COLL_IMPLICIT,
                tau_mode=RLB_TAU_UNIFORM, with_density=False, nu=27.0 ** 0.25, dt_over_dx=0.25,
                tau=1.0, eta_over_s=0.0, alpha=0.0, bc: Sequence[int] = (0,) * 6,
                face_states=None, guard_umax=0.0, guard_efloor=1e-10,
                lattice=RLB_LATTICE_EXTENDED, density_weights=RLB_DENSW_PAPER,
                flux=RLB_FLUX_MINMOD) -> rlb_config:
    c = rlb_config_default()
    c.nx, c.ny, c.nz = int(nx), int(ny), int(nz)
    c.precision, c.collision, c.tau_mode = int(precision), int(collision), int(tau_mode)
    c.with_density = int(bool(with_density))
    c.nu, c.dt_over_dx, c.tau = float(nu), float(dt_over_dx), float(tau)
    c.eta_over_s, c.alpha = float(eta_over_s), float(alpha)
    for k in range(6):
        c.bc[k] = int(bc[k])
        if face_states is not None:
            for j in range(5):
                c.face_states[k][j] = float(face_states[k][j])
    c.guard_umax, c.guard_efloor = float(guard_umax), float(guard_efloor)
    c.lattice = int(lattice)
    c.density_weights = int(density_weights)
    c.flux = int(flux)
    return c


def config_for_workload(w, precision=None) -> rlb_config:
    """rlb_config of a paper_1302_1125_amd.workloads.Workload."""
    return config_from(w.nx, w.ny, w.nz, precision=w.precision if precision is None else precision,
                       collision=w.collision, tau_mode=w.tau_mode, with_density=w.with_density,
                       nu=w.nu, dt_over_dx=w.dt, tau=w.tau, eta_over_s=w.eta_over_s, alpha=w.alpha,
                       bc=w.bc, face_states=w.face_states, guard_umax=w.guard_umax,
                       guard_efloor=w.guard_efloor, lattice=w.lattice,
                       density_weights=w.density_weights, flux=w.flux)


def rlb_footprint_bytes(cfg: rlb_config) -> int:
    return int(load().rlb_footprint_bytes(ctypes.byref(cfg)))


class Context:
    """Owner of one rlb_ctx.  Methods map 1:1 onto the C calls."""

    def __init__(self, cfg: rlb_config, stream: Optional[int] = None):
        self._L = load()
        self.cfg = cfg
        h = ctypes.c_void_p()
        _check(self._L.rlb_create(ctypes.byref(cfg), ctypes.c_void_p(stream) if stream else None,
                                  ctypes.byref(h)))
        self._h = h
        self.shape = (cfg.nz, cfg.ny, cfg.nx)
        self.ncell = cfg.nx * cfg.ny * cfg.nz

    def close(self):
        if getattr(self, "_h", None):
            self._L.rlb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def rlb_init_fields(self, eps, ux, uy, uz, n=None, obstacle=None):
        a = [_f64(v) for v in (eps, ux, uy, uz)]
        for v in a:
            if v.size != self.ncell:
                raise ValueError("field size does not match the grid")
        nn = None if n is None else _f64(n)
        ob = None
        if obstacle is not None:
            ob = np.ascontiguousarray(np.asarray(obstacle, dtype=np.uint8)).reshape(-1)
            if ob.size != self.ncell:
                raise ValueError("obstacle size does not match the grid")
        _check(self._L.rlb_init_fields(
            self._h, _dp(a[0]), _dp(a[1]), _dp(a[2]), _dp(a[3]), _dp(nn),
            None if ob is None else ob.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))

    def rlb_step(self, nsteps: int):
        _check(self._L.rlb_step(self._h, int(nsteps)))

    def rlb_step_async(self, nsteps: int):
        _check(self._L.rlb_step_async(self._h, int(nsteps)))

    def rlb_sync(self):
        _check(self._L.rlb_sync(self._h))

    def rlb_steps_per_launch(self) -> int:
        return int(self._L.rlb_steps_per_launch(self._h))

    def rlb_moments(self):
        """(eps, ux, uy, uz, n) as float64 arrays of shape [nz, ny, nx]."""
        out = [np.empty(self.ncell) for _ in range(5)]
        _check(self._L.rlb_moments(self._h, *[_dp(o) for o in out]))
        return [o.reshape(self.shape) for o in out]

    def rlb_moments_noalloc(self, out=None):
        """rlb_moments through the library's fixed device read-back array (no
        device allocation; grids of at most 2^20 cells).  `out`: optional five
        float64 host arrays of ncell elements to fill (else new ones)."""
        if out is None:
            out = [np.empty(self.ncell) for _ in range(5)]
        for o in out:
            if o.dtype != np.float64 or o.size != self.ncell or not o.flags.c_contiguous:
                raise ValueError("outputs: five contiguous float64 arrays of ncell elements")
        _check(self._L.rlb_moments_noalloc(self._h, *[_dp(o) for o in out]))
        return [o.reshape(self.shape) for o in out]

    def status_of_moments_noalloc(self) -> int:
        """rlb_moments_noalloc returning the raw status (outputs discarded)."""
        out = [np.empty(self.ncell) for _ in range(5)]
        return int(self._L.rlb_moments_noalloc(self._h, *[_dp(o) for o in out]))

    def rlb_stats_get(self) -> rlb_stats:
        s = rlb_stats()
        _check(self._L.rlb_stats_get(self._h, ctypes.byref(s)))
        return s

    def status_of_step(self, nsteps: int) -> int:
        """rlb_step returning the raw status instead of raising."""
        return int(self._L.rlb_step(self._h, int(nsteps)))


def context_for_workload(w, precision=None, stream=None, init=True) -> Context:
    ctx = Context(config_for_workload(w, precision), stream)
    if init:
        ctx.rlb_init_fields(w.eps, w.ux, w.uy, w.uz, w.n if w.with_density else None, w.obstacle)
    return ctx


# ---------------------------------------------------------------------------
# Batched serving (rlb_server_*)
# ---------------------------------------------------------------------------

EXPORTED += ["rlb_server_create", "rlb_server_submit", "rlb_server_poll", "rlb_server_result",
             "rlb_server_drain", "rlb_server_stats_get", "rlb_server_destroy",
             "rlb_request_footprint_bytes"]


class rlb_request(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("n", ctypes.c_int32), ("steps", ctypes.c_int64),
        ("eps", ctypes.POINTER(ctypes.c_double)), ("ux", ctypes.POINTER(ctypes.c_double)),
        ("uy", ctypes.POINTER(ctypes.c_double)), ("uz", ctypes.POINTER(ctypes.c_double)),
        ("dens", ctypes.POINTER(ctypes.c_double)),
        ("eta_over_s", ctypes.c_double), ("tau", ctypes.c_double), ("alpha", ctypes.c_double),
        ("bc_lo", ctypes.c_int32), ("bc_hi", ctypes.c_int32),
        ("face_lo", ctypes.c_double * 5), ("face_hi", ctypes.c_double * 5),
    ]


class rlb_server_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
        ("failed", ctypes.c_uint64), ("rejected", ctypes.c_uint64), ("capacity_cells", ctypes.c_uint64),
        ("resident_cells_peak", ctypes.c_uint64), ("resident_requests_peak", ctypes.c_uint64),
        ("chunks", ctypes.c_uint64), ("global_steps", ctypes.c_uint64),
        ("cell_updates", ctypes.c_double), ("busy_seconds", ctypes.c_double),
        ("wall_seconds", ctypes.c_double), ("latency_p50", ctypes.c_double),
        ("latency_p99", ctypes.c_double), ("latency_max", ctypes.c_double),
    ]


def _load_server(L):
    if getattr(L, "_server_ready", False):
        return
    dp = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    L.rlb_server_create.argtypes = [ctypes.POINTER(rlb_config), ctypes.c_uint64, ctypes.c_int32,
                                    ctypes.POINTER(vp)]
    L.rlb_server_submit.argtypes = [vp, ctypes.POINTER(rlb_request), ctypes.POINTER(ctypes.c_uint64)]
    L.rlb_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]
    L.rlb_server_result.argtypes = [vp, ctypes.c_uint64, dp, dp, dp, dp, dp, dp,
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.rlb_server_drain.argtypes = [vp]
    L.rlb_server_stats_get.argtypes = [vp, ctypes.POINTER(rlb_server_stats)]
    L.rlb_server_destroy.argtypes = [vp]
    L.rlb_server_destroy.restype = None
    L.rlb_request_footprint_bytes.argtypes = [ctypes.POINTER(rlb_config), ctypes.c_int32]
    L.rlb_request_footprint_bytes.restype = ctypes.c_uint64
    for name in ("rlb_server_create", "rlb_server_submit", "rlb_server_poll", "rlb_server_result",
                 "rlb_server_drain", "rlb_server_stats_get"):
        getattr(L, name).restype = ctypes.c_int
    L._server_ready = True


def rlb_request_footprint_bytes(common: rlb_config, n: int) -> int:
    L = load()
    _load_server(L)
    return int(L.rlb_request_footprint_bytes(ctypes.byref(common), int(n)))


class Server:
    """Owner of one rlb_server (continuous batching of 1D requests)."""

    def __init__(self, common: rlb_config, budget_bytes: int, chunk_steps: int = 64):
        self._L = load()
        _load_server(self._L)
        self.common = common
        h = ctypes.c_void_p()
        _check(self._L.rlb_server_create(ctypes.byref(common), int(budget_bytes), int(chunk_steps),
                                         ctypes.byref(h)))
        self._h = h
        self._sizes = {}

    def close(self):
        if getattr(self, "_h", None):
            self._L.rlb_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def rlb_server_submit(self, eps, ux, uy, uz, dens=None, steps=0, eta_over_s=0.0, tau=1.0,
                          alpha=0.0, bc_lo=RLB_BC_FIXED, bc_hi=RLB_BC_FIXED, face_lo=None,
                          face_hi=None) -> int:
        a = [_f64(v) for v in (eps, ux, uy, uz)]
        d = None if dens is None else _f64(dens)
        r = rlb_request()
        r.struct_size = ctypes.sizeof(rlb_request)
        r.n = a[0].size
        r.steps = int(steps)
        r.eps, r.ux, r.uy, r.uz = (_dp(v) for v in a)
        r.dens = _dp(d)
        r.eta_over_s, r.tau, r.alpha = float(eta_over_s), float(tau), float(alpha)
        r.bc_lo, r.bc_hi = int(bc_lo), int(bc_hi)
        for k in range(5):
            r.face_lo[k] = float(face_lo[k]) if face_lo is not None else (3.0 if k == 0 else (1.0 if k == 4 else 0.0))
            r.face_hi[k] = float(face_hi[k]) if face_hi is not None else (3.0 if k == 0 else (1.0 if k == 4 else 0.0))
        rid = ctypes.c_uint64()
        _check(self._L.rlb_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        self._sizes[rid.value] = r.n
        return rid.value

    def submit_request(self, q) -> int:
        """Submit a workloads.ServingRequest."""
        return self.rlb_server_submit(q.eps, q.ux, q.uy, q.uz, q.dens, q.steps, q.eta_over_s, q.tau,
                                      q.alpha, q.bc_lo, q.bc_hi, q.face_lo, q.face_hi)

    def rlb_server_poll(self, rid: int) -> bool:
        d = ctypes.c_int32()
        _check(self._L.rlb_server_poll(self._h, ctypes.c_uint64(rid), ctypes.byref(d)))
        return bool(d.value)

    def rlb_server_result(self, rid: int, raise_inadmissible: bool = True):
        """(fields [eps, ux, uy, uz, n], latency_s, first_bad, guard_events, status)."""
        n = self._sizes[rid]
        out = [np.empty(n) for _ in range(5)]
        lat = ctypes.c_double()
        bad = ctypes.c_int64()
        gev = ctypes.c_int64()
        st = int(self._L.rlb_server_result(self._h, ctypes.c_uint64(rid), *[_dp(o) for o in out],
                                           ctypes.byref(lat), ctypes.byref(bad), ctypes.byref(gev)))
        if st != RLB_OK and (st != RLB_E_INADMISSIBLE or raise_inadmissible):
            _check(st)
        del self._sizes[rid]
        return out, lat.value, bad.value, gev.value, st

    def rlb_server_drain(self):
        _check(self._L.rlb_server_drain(self._h))

    def rlb_server_stats_get(self) -> rlb_server_stats:
        s = rlb_server_stats()
        _check(self._L.rlb_server_stats_get(self._h, ctypes.byref(s)))
        return s
