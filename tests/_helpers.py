"""Test-side helpers: build the oracle for a workload and compare fields."""
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
    A, B = derived(test_fields), derived(ref_fields)
    out = {}
    for k in keys:
        if np.linalg.norm(B[k]) == 0.0 and np.linalg.norm(A[k]) == 0.0:
            out[k] = 0.0
        elif np.linalg.norm(B[k]) == 0.0:
            out[k] = float(np.abs(A[k]).max())
        else:
            out[k] = rel_l2(A[k], B[k])
    return out
