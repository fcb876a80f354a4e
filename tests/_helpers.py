"""Test-side helpers: build the oracle for a workload and compare fields."""
import math

import numpy as np

from oracle import oracle as O


def oracle_for(w, **over):
    cfg = O.Config(nx=w.nx, ny=w.ny, nz=w.nz, nu=w.nu, dt=w.dt, euler=(w.collision == 1),
                   tau_mode=w.tau_mode, tau=w.tau, eta_over_s=w.eta_over_s, alpha=w.alpha,
                   with_h=bool(w.with_density), bc=list(w.bc), face=[list(s) for s in w.face_states],
                   guard_umax=w.guard_umax, guard_efloor=w.guard_efloor,
                   basic=(w.lattice == 1), density_weights=w.density_weights, flux=w.flux)
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


def crop_workload(w, center, radius):
    """Workload restricted to the window of `radius` cells around `center`
    (z, y, x).  Axes whose window reaches the domain edge keep that face's
    boundary condition; other crop faces are outflow (the dependency cone of
    the centre cell never reaches them within radius // 2 - 1 steps).
    Periodic axes wrap.  Returns (cropped workload, index of the centre)."""
    import numpy as np
    n = (w.nz, w.ny, w.nx)
    axis_of = {0: 2, 1: 1, 2: 0}  # array axis -> lattice axis (x = 0)
    idx = []
    bc = list(w.bc)
    cpos = []
    for ax in range(3):
        a = axis_of[ax]
        N = n[ax]
        c = center[ax]
        lo_f, hi_f = 2 * a, 2 * a + 1
        if N == 1:
            idx.append(np.array([0]))
            cpos.append(0)
            continue
        periodic = w.bc[lo_f] == 0
        if 2 * radius + 1 >= N:
            idx.append(np.arange(N))
            cpos.append(c)
            continue
        if periodic:
            idx.append(np.arange(c - radius, c + radius + 1) % N)
            cpos.append(radius)
            bc[lo_f] = bc[hi_f] = 2
            continue
        lo = max(0, c - radius)
        hi = min(N, c + radius + 1)
        idx.append(np.arange(lo, hi))
        cpos.append(c - lo)
        if lo > 0:
            bc[lo_f] = 2
        if hi < N:
            bc[hi_f] = 2
    sel = np.ix_(idx[0], idx[1], idx[2])
    cw = w.copy_with(nz=len(idx[0]), ny=len(idx[1]), nx=len(idx[2]), bc=bc)
    cw.eps, cw.ux, cw.uy, cw.uz, cw.n = (None if a is None else a[sel].copy()
                                         for a in (w.eps, w.ux, w.uy, w.uz, w.n))
    if w.obstacle is not None:
        cw.obstacle = w.obstacle[sel].copy()
    # size-1 axes of the crop must be periodic
    for ax, a in ((0, 2), (1, 1), (2, 0)):
        if len(idx[ax]) == 1:
            cw.bc[2 * a] = cw.bc[2 * a + 1] = 0
    return cw, tuple(cpos)


def sampled_oracle_fields(w, cells, steps):
    """Oracle fields after `steps` steps at each sampled cell, each from the
    cropped dependency cone (radius 2 steps + 2)."""
    import numpy as np
    out = []
    for cell in cells:
        cw, cp = crop_workload(w, cell, 2 * steps + 2)
        o = oracle_for(cw)
        assert o.step(steps) == 0
        fl = o.fields()
        out.append([float(a[cp]) for a in fl])
    return np.array(out)
