"""Helpers shared by the parity tests: tolerances, element-wise comparisons
of field planes and of particles, and a bridge that drives the oracle with
the GPU's state.

Field planes are compared one component at a time, by relative L2 and by the
largest element-wise difference relative to the component's largest value
(the paper's own validation yardstick is the maximum relative error of a
field map, Sec. 4.2).

Particles carry no identity, and the GPU stores them tile by tile in an order
of its own.  After one step from the same state every particle of one side
lies within rounding of exactly one particle of the other in phase space
(cell + offset, momentum), so the two sets are paired by nearest neighbour
in that space; the pairing must be one to one, and every component of every
pair is then compared element by element.
"""
from __future__ import annotations

import numpy as np

from oracle import OracleSim, Species

# FP32 path vs FP64 oracle, one step from the same state (rel. L2 per field)
TOL_STEP_FP32 = 1e-5
# FP64 path vs FP64 oracle
TOL_STEP_FP64 = 1e-11
# Element-wise bound per component: max |gpu - oracle| <= TOL_MAX * max |oracle|
# of that component.  FP32: every output element of one step is a short sum of
# terms rounded at 2^-24 relative to the largest input term, so 1e-5 leaves
# two decades of margin while a single wrong cell at 1e-4 of the component's
# scale fails.  FP64: the fixed-point current resolution (~1e-15 of the
# current scale) dominates.
TOL_MAX_FP32 = 1e-5
TOL_MAX_FP64 = 1e-11
# Floor of both bounds, relative to the scale of the whole group (all current
# components, or all six field components): a component that is zero in exact
# arithmetic (Jy under a laser polarised along z, B before a filament forms)
# is computed from inputs on the group's scale, each rounded at 2^-24 in FP32,
# so it carries a few ulps of that scale; 1e-6 is about 16 ulps.  FP64: the
# fixed-point current resolution summed over ~1e3 terms.
FLOOR_FP32 = 1e-6
FLOOR_FP64 = 1e-12
# Particles after one step: position (cells) and momentum (relative to the
# largest |u| of the set).  FP32 offsets carry 2^-24 ulps; the displacement,
# under one cell, is computed from u with a few ulps of relative error.
TOL_POS_FP32 = 2e-6
TOL_POS_FP64 = 1e-12
TOL_U_FP32 = 1e-5
TOL_U_FP64 = 1e-11


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt((b ** 2).sum())
    num = np.sqrt(((a - b) ** 2).sum())
    if den == 0:
        return float(num)
    return float(num / den)


def plane_errors(a, b):
    """Per component k of (K, ny, nx) arrays a (tested) and b (reference):
    (relative L2, max |a - b|, max |b|)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = []
    for k in range(a.shape[0]):
        d = np.abs(a[k] - b[k])
        out.append((rel_l2(a[k], b[k]), float(d.max()) if d.size else 0.0,
                    float(np.abs(b[k]).max()) if d.size else 0.0))
    return out


def check_planes(a, b, names, tol_l2, tol_max, what="", floor=0.0):
    """Assert the per-component bounds, each with a floor relative to the
    group's scale:
        rms(a_k - b_k) <= tol_l2 * rms(b_k) + floor * rms(b over the group),
        max|a_k - b_k| <= tol_max * max|b_k| + floor * max|b over the group|.
    Returns {name: (rel_l2, max_rel)} (relative to the component itself).
    If the whole group is zero in the reference, so must be a."""
    bg = np.asarray(b, dtype=np.float64)
    g_rms = float(np.sqrt((bg ** 2).mean())) if bg.size else 0.0
    g_max = float(np.abs(bg).max()) if bg.size else 0.0
    res, bad = {}, {}
    for k, (name, (l2, dmax, bmax)) in enumerate(zip(names, plane_errors(a, b))):
        mrel = dmax / bmax if bmax > 0 else dmax
        res[name] = (l2, mrel)
        if g_max == 0.0:
            ok = dmax == 0.0
        else:
            bk = bg[k]
            rms_b = float(np.sqrt((bk ** 2).mean()))
            rms_d = float(np.sqrt(((np.asarray(a[k], dtype=np.float64) - bk) ** 2).mean()))
            ok = (rms_d <= tol_l2 * rms_b + floor * g_rms and
                  dmax <= tol_max * bmax + floor * g_max)
        if not ok:
            bad[name] = (l2, dmax, bmax, g_max)
    assert not bad, (what, bad)
    return res


def match_particles(pg, po, nx, ny, window=False, x_range=None):
    """Pair every oracle particle (po) with its nearest GPU particle (pg) in
    (global x, global y, ux, uy, uz), x and y in cells, periodic unless the
    window is on.  Returns (index into pg per po particle, wrapped position
    differences dX, dY).  With x_range = (a, b) only oracle particles with
    a <= X < b are paired, against the GPU particles with a - 1 <= X < b + 1
    (a sample of a set too large to pair whole)."""
    from scipy.spatial import cKDTree
    Xg = pg["ix"] + pg["x"]
    Yg = pg["iy"] + pg["y"]
    Xo = po["ix"] + po["x"]
    Yo = po["iy"] + po["y"]
    sel_o = np.arange(len(Xo))
    sel_g = np.arange(len(Xg))
    if x_range is not None:
        a, b = x_range
        sel_o = np.nonzero((Xo >= a) & (Xo < b))[0]
        sel_g = np.nonzero((Xg >= a - 1) & (Xg < b + 1))[0]
    U = [np.concatenate([pg[k][sel_g], po[k][sel_o]]) for k in ("ux", "uy", "uz")]
    lo = [u.min() - 1.0 for u in U]
    span = [u.max() - u.min() + 2.0 for u in U]
    big = 1e6 * (1 + max(span))
    xbox = big if window else float(nx)

    def pts(X, Y, p, sel):
        c = [np.mod(X[sel], nx) if not window else X[sel] + 2.0, np.mod(Y[sel], ny)]
        c += [p[k][sel] - lo[i] for i, k in enumerate(("ux", "uy", "uz"))]
        return np.stack(c, axis=1)

    tree = cKDTree(pts(Xg, Yg, pg, sel_g), boxsize=[xbox, float(ny), big, big, big],
                   balanced_tree=False, compact_nodes=False)
    _, idx = tree.query(pts(Xo, Yo, po, sel_o), workers=-1)
    gi = sel_g[idx]
    dX = Xg[gi] - Xo[sel_o]
    dY = Yg[gi] - Yo[sel_o]
    if not window:
        dX -= nx * np.round(dX / nx)
    dY -= ny * np.round(dY / ny)
    return sel_o, gi, dX, dY


def check_particles(pg, po, nx, ny, window=False, fp64=False, x_range=None, what=""):
    """Pair the two sets one to one and bound every component of every pair:
    |dX|, |dY| <= TOL_POS cells; |du| <= TOL_U * max |u| of the set.
    Returns the largest errors."""
    if x_range is None:
        assert len(pg["ix"]) == len(po["ix"]), (what, len(pg["ix"]), len(po["ix"]))
    if len(po["ix"]) == 0:
        return dict(pos=0.0, u=0.0)
    so, gi, dX, dY = match_particles(pg, po, nx, ny, window, x_range)
    assert len(so) > 0, what
    assert len(np.unique(gi)) == len(gi), (what, "pairing is not one to one",
                                           len(gi) - len(np.unique(gi)))
    tp = TOL_POS_FP64 if fp64 else TOL_POS_FP32
    tu = TOL_U_FP64 if fp64 else TOL_U_FP32
    pos = float(max(np.abs(dX).max(), np.abs(dY).max()))
    umax = max(float(np.abs(po[k]).max()) for k in ("ux", "uy", "uz"))
    du = max(float(np.abs(pg[k][gi] - po[k][so]).max()) for k in ("ux", "uy", "uz"))
    urel = du / umax if umax > 0 else du
    assert pos <= tp and urel <= tu, (what, dict(pos=pos, u=urel, umax=umax))
    return dict(pos=pos, u=urel)


def round_to_f32(p):
    q = dict(p)
    for k in ("x", "y", "ux", "uy", "uz"):
        v = np.asarray(p[k], dtype=np.float32).astype(np.float64)
        if k in ("x", "y"):
            v = np.minimum(v, np.nextafter(np.float32(1), np.float32(0)))
        q[k] = v
    return q


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


J_NAMES = ("Jx", "Jy", "Jz")
F_NAMES = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")
# particle sets larger than this are paired on a strip of 32 columns
PAIR_WHOLE_MAX = 40_000_000


def compare_state(sim, o, w, fp64=False, what=""):
    """Per-component and element-wise comparison of J, filtered J, E, B and
    every particle after a step from the same state.  Returns the errors,
    with J, Jf and F the largest relative L2 of their components."""
    t = TOL_STEP_FP64 if fp64 else TOL_STEP_FP32
    tm = TOL_MAX_FP64 if fp64 else TOL_MAX_FP32
    fl = FLOOR_FP64 if fp64 else FLOOR_FP32
    errs = {}
    for key, a, b, names in (
            ("J", sim.get_current(False), o.get_current(False), J_NAMES),
            ("Jf", sim.get_current(True), o.get_current(True), J_NAMES),
            ("F", sim.get_fields(), o.get_fields(), F_NAMES)):
        r = check_planes(a, b, names, t, tm, "%s %s" % (what, key), floor=fl)
        errs[key] = max(v[0] for v in r.values())
        errs.update({"%s.%s" % (key, n): v for n, v in r.items()})
    for k in range(len(w.species)):
        pg, po = sim.get_particles(k), o.get_particles(k)
        assert len(pg["ix"]) == len(po["ix"]), (what, k, len(pg["ix"]), len(po["ix"]))
        xr = None
        if len(po["ix"]) > PAIR_WHOLE_MAX:
            xr = (w.nx // 2 - 16 + 0.5, w.nx // 2 + 16 + 0.5)
        errs["p%d" % k] = check_particles(pg, po, w.nx, w.ny, window=w.moving_window,
                                          fp64=fp64, x_range=xr, what="%s species %d" % (what, k))
    print("parity", what, {k: v for k, v in errs.items() if k in ("J", "Jf", "F")
                           or k.startswith("p")}, flush=True)
    return errs
