"""Test-side helpers: build the oracle for a workload and compare fields."""
import math

import numpy as np

from oracle import oracle as O


def oracle_for(w, **over):
    cfg = O.Config(nx=w.nx, ny=w.ny, nz=w.nz, nu=w.nu, dt=w.dt, euler=(w.collision == 1),
                   tau_mode=w.tau_mode, tau=w.tau, eta_over_s=w.eta_over_s, alpha=w.alpha,
                   with_h=bool(w.with_density), bc=list(w.bc), face=[list(s) for s in w.face_states],
                   guard_umax=w.guard_umax, guard_efloor=w.guard_efloor)
    for k, v in over.items():
        setattr(cfg, k, v)
    o = O.Oracle(cfg)
    o.init(w.eps, w.ux, w.uy, w.uz, w.n if w.with_density else None, w.obstacle)
    return o


def derived(fields):
    """(eps, p, n, gamma u^x, gamma u^y, gamma u^z) from (eps, ux, uy, uz, n)."""
    eps, ux, uy, uz, n = [np.asarray(a, dtype=np.float64) for a in fields]
    g = 1.0 / np.sqrt(1.0 - (ux * ux + uy * uy + uz * uz))
    return {"eps": eps, "p": eps / 3.0, "n": n, "gux": g * ux, "guy": g * uy, "guz": g * uz}


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    den = np.linalg.norm(b)
    if den == 0.0:
        return float(np.linalg.norm(a - b))
    return float(np.linalg.norm(a - b) / den)


def field_errors(test_fields, ref_fields, keys=("eps", "p", "n", "gux", "guy", "guz")):
    """Rel. L2 error per field.  Components of gamma u are normalised by the
    L2 norm of the whole gamma u vector field (a component that is zero in
    the reference, e.g. u^y of a symmetric flow, has no scale of its own)."""
    A, B = derived(test_fields), derived(ref_fields)
    vnorm = math.sqrt(sum(float(np.linalg.norm(B[k])) ** 2 for k in ("gux", "guy", "guz")))
    out = {}
    for k in keys:
        den = vnorm if k in ("gux", "guy", "guz") else float(np.linalg.norm(B[k]))
        num = float(np.linalg.norm(A[k] - B[k]))
        out[k] = num / den if den > 0 else num
    return out
