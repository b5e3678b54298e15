"""Helpers shared by the parity tests: tolerances, order-free particle
comparisons and a bridge that drives the oracle with the GPU's state.

Particles carry no identity, and the GPU stores them tile by tile in an order
of its own, so particle sets are compared through quantities that do not
depend on order and are continuous in the particle state: sorted momentum
components and area-weighted (bilinear) moment densities on the nodes.
"""
from __future__ import annotations

import numpy as np

from oracle import OracleSim, Species

# FP32 path vs FP64 oracle, one step from the same state (rel. L2 per field)
TOL_STEP_FP32 = 1e-5
# FP64 path vs FP64 oracle
TOL_STEP_FP64 = 1e-11


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt((b ** 2).sum())
    num = np.sqrt(((a - b) ** 2).sum())
    if den == 0:
        return float(num)
    return float(num / den)


def round_to_f32(p):
    q = dict(p)
    for k in ("x", "y", "ux", "uy", "uz"):
        v = np.asarray(p[k], dtype=np.float32).astype(np.float64)
        if k in ("x", "y"):
            v = np.minimum(v, np.nextafter(np.float32(1), np.float32(0)))
        q[k] = v
    return q


def moments(p, nx, ny, window=False):
    """Bilinear moment densities on the nodes: sum w, w*ux, w*uy, w*uz, w*|u|^2."""
    X = p["ix"] + p["x"]
    Y = p["iy"] + p["y"]
    i0 = np.floor(X).astype(np.int64)
    j0 = np.floor(Y).astype(np.int64)
    wx = X - i0
    wy = Y - j0
    u2 = p["ux"] ** 2 + p["uy"] ** 2 + p["uz"] ** 2
    vals = [np.ones_like(X), p["ux"], p["uy"], p["uz"], u2]
    out = np.zeros((len(vals), ny, nx))
    for a in (0, 1):
        for b in (0, 1):
            w = (wx if a else 1 - wx) * (wy if b else 1 - wy)
            ii = i0 + a
            jj = (j0 + b) % ny
            if window:
                ok = (ii >= 0) & (ii < nx)
            else:
                ii = ii % nx
                ok = np.ones_like(ii, dtype=bool)
            idx = (jj * nx + ii)[ok]
            for k, v in enumerate(vals):
                out[k] += np.bincount(idx, (w * v)[ok], minlength=nx * ny).reshape(ny, nx)
    return out


def compare_particles(pg, po, nx, ny, window=False, tol=TOL_STEP_FP32):
    """Max over the order-free comparisons; counts must agree exactly."""
    assert len(pg["ix"]) == len(po["ix"]), (len(pg["ix"]), len(po["ix"]))
    if len(po["ix"]) == 0:
        return 0.0
    errs = [rel_l2(moments(pg, nx, ny, window), moments(po, nx, ny, window))]
    for k in ("ux", "uy", "uz"):
        a, b = np.sort(pg[k]), np.sort(po[k])
        scale = max(np.abs(b).max(), 1e-30)
        errs.append(float(np.abs(a - b).max() / scale))
    return max(errs)


def oracle_from_workload(w):
    o = OracleSim(w.nx, w.ny, w.lx, w.ly, w.dt, window=w.moving_window,
                  filter_passes=w.filter_passes, filter_compensate=w.filter_compensate,
                  seed=w.seed)
    return o


def add_species(o, w, load):
    for s in w.species:
        o.add_species(Species(s.qm, s.density, s.x_lo, s.x_hi, s.ppc, s.uth, s.ufl), load=load)
    if w.laser is not None and load:
        L = w.laser
        o.add_laser(L.a0, L.omega0, L.W0, L.fwhm, L.x_center, L.focus, L.axis, L.pol)


def oracle_mirror(sim, w):
    """An oracle holding exactly the GPU's current state (fields, particles,
    step counter, window shifts), cast to FP64."""
    o = oracle_from_workload(w)
    add_species(o, w, load=False)
    for k in range(len(w.species)):
        o.set_particles(k, sim.get_particles(k))
    o.set_fields(sim.get_fields())
    e = sim.energy()
    o.set_iter(e["step"], e["nshift"])
    return o
