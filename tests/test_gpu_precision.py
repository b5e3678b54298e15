"""Precision study: the FP32 and FP64 GPU paths against the FP64 oracle on
the 8000 x 512 laser-wakefield geometry.

The geometry keeps the 2000 x 256 run's cell size (0.02 x 0.2) and step
(dt = 0.014), fills the whole 160 x 102.4 box with cold plasma at 4 x 4
particles per cell (65,536,000 particles), and drives it with the same laser
under a moving window (paper Sec. 4.1).  All three runs start from their own
loader and laser (identical up to the FP32 rounding of the initial state)
and then run free: no state is copied between them.

Over a 64-step prefix (PIC_PRECISION_PREFIX overrides), every step compares
E, B and the filtered current J of each GPU path with the oracle's, as
relative L2 errors.  The GPU paths then run on to 200 steps, where FP64
diagnostics at every step give the energy history and the Gauss and
continuity residuals of each path (window interior, see pic_energy).  PIC_PRECISION_REPORT names a
JSON file that receives every number measured.

Tolerances (eps = 2^-24, the FP32 rounding unit):
  - FP32 vs oracle, every step of the prefix: E, B and J within 1e-5 relative
    L2; the cold plasma's motion is driven by the laser and is not chaotic
    over the prefix, so the rounding of each step adds up slowly.
  - FP64 vs oracle: within 1e-9 (the FP64 current sums are fixed point with a
    resolution of 2^-e of the scale; everything else rounds at 1e-16).
  - Total energy: FP64 vs oracle within 1e-9, FP32 vs oracle within 1e-5 at
    the end of the prefix; FP32 vs FP64 within 1e-5 at every step to 200
    (twice the fields' relative error, with margin).
  - Gauss residual of the FP32 path at step n: E is stored in FP32, so each
    step adds a rounding of eps |E| to every component, and the divergence of
    those roundings walks randomly: at most 2 eps (E0 / dmin) sqrt(n) +
    eps rho_max, with E0 = a0 omega0 the laser amplitude and dmin the smaller
    cell size.
  - Continuity residual of the FP32 path: rho^n and rho^{n-1} are stored in
    FP32 (eps rho_max / dt), J is rounded at the tile flush and again when the
    tiles are folded (2 eps |J| per value, with |J| <= rho_max since |v| < 1,
    entering div J over dmin); a factor 2 covers the rounding of the
    per-particle deposit terms: 4 eps rho_max (1/dt + 2/dmin).
  - FP64 residuals: below 1e-10 rho_max (Gauss) and 1e-10 rho_max / dt.
"""
import json
import os
import time

import numpy as np
import pytest

from inputs import lwfa8000

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2106_12485_amd import Simulation  # noqa: E402
from parity_util import add_species, oracle_from_workload  # noqa: E402

PREFIX = int(os.environ.get("PIC_PRECISION_PREFIX", "64"))
STEPS = 200
TOL32 = 1e-5
TOL64 = 1e-9


def rel(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / max((b ** 2).sum(), 1e-300)))


def diag_row(e):
    return dict(step=int(e["step"]), e_energy=e["e_energy"], b_energy=e["b_energy"],
                ke=float(np.sum(e["ke"])), total=e["total"], gauss=e["gauss_res_max"],
                cont=e["cont_res_max"], rho_max=e["rho_max"],
                particles=int(np.sum(e["n_particles"])), nshift=int(e["nshift"]))


@pytest.mark.timeout(900)
def test_precision_study_lwfa_8000x512():
    w = lwfa8000()
    t0 = time.time()
    g32 = Simulation(w)
    g64 = Simulation(w, fp64=True)
    o = oracle_from_workload(w)
    add_species(o, w, load=True)
    o.set_threads(min(16, os.cpu_count() or 1))
    print("loaded %d particles in %.1f s" % (o.count(0), time.time() - t0), flush=True)
    assert g32.count(0) == g64.count(0) == o.count(0) == 65536000

    prefix = []
    for n in range(1, PREFIX + 1):
        g32.step(1)
        g64.step(1)
        o.step(1)
        fo, jo = o.get_fields(), o.get_current(True)
        row = dict(step=n, nshift=o.nshift)
        for name, g in (("fp32", g32), ("fp64", g64)):
            f, j = g.get_fields(), g.get_current(True)
            row[name] = dict(E=rel(f[:3], fo[:3]), B=rel(f[3:], fo[3:]), J=rel(j, jo))
        prefix.append(row)
        print("step %3d shift %3d  fp32 E %.2e B %.2e J %.2e   fp64 E %.2e B %.2e J %.2e"
              % (n, o.nshift, row["fp32"]["E"], row["fp32"]["B"], row["fp32"]["J"],
                 row["fp64"]["E"], row["fp64"]["B"], row["fp64"]["J"]), flush=True)
    eo = o.energy()
    at_prefix = dict(oracle=dict(total=eo["total"], e_energy=eo["e_energy"],
                                 b_energy=eo["b_energy"], ke=float(eo["ke"].sum())),
                     fp32=diag_row(g32.energy()), fp64=diag_row(g64.energy()))
    o.close()

    history = {"fp32": [], "fp64": []}
    for n in range(PREFIX + 1, STEPS + 1):
        g32.step(1)
        g64.step(1)
        for name, g in (("fp32", g32), ("fp64", g64)):
            history[name].append(diag_row(g.energy()))
    f32, f64 = g32.get_fields(), g64.get_fields()
    emax = float(np.abs(f64[:3]).max())
    final = dict(E=rel(f32[:3], f64[:3]), B=rel(f32[3:], f64[3:]),
                 J=rel(g32.get_current(True), g64.get_current(True)))
    print("step %d fp32 vs fp64: E %.2e B %.2e J %.2e" % (STEPS, final["E"], final["B"],
                                                          final["J"]), flush=True)
    for name in ("fp32", "fp64"):
        h = history[name][1:]
        print("%s: max gauss %.3e max cont %.3e (rho_max %.3f, |E|max %.2f)" % (
            name, max(r["gauss"] for r in h), max(r["cont"] for r in h),
            max(r["rho_max"] for r in h), emax), flush=True)
    report = dict(workload=w.name, prefix=prefix, at_prefix=at_prefix, history=history,
                  fp32_vs_fp64_at_end=final, e_max_at_end=emax,
                  tolerances=dict(fp32=TOL32, fp64=TOL64))
    path = os.environ.get("PIC_PRECISION_REPORT")
    if path:
        with open(path, "w") as fh:
            json.dump(report, fh, indent=1)

    for row in prefix:
        for q in ("E", "B", "J"):
            assert row["fp32"][q] <= TOL32, (row["step"], q, row["fp32"][q])
            assert row["fp64"][q] <= TOL64, (row["step"], q, row["fp64"][q])
    ot = at_prefix["oracle"]["total"]
    assert abs(at_prefix["fp64"]["total"] / ot - 1) < 1e-9
    assert abs(at_prefix["fp32"]["total"] / ot - 1) < 1e-5
    eps = 2.0 ** -24
    dmin = min(w.lx / w.nx, w.ly / w.ny)
    e0 = w.laser.a0 * w.laser.omega0
    for h32, h64 in zip(history["fp32"], history["fp64"]):
        assert h32["step"] == h64["step"] and h32["nshift"] == h64["nshift"]
        assert abs(h32["total"] / h64["total"] - 1) < 1e-5, (h32["step"], h32, h64)
        assert abs(h32["particles"] - h64["particles"]) <= 1e-6 * h64["particles"]
    # the continuity residual needs the previous step's charge: skip the first
    for h32, h64 in zip(history["fp32"][1:], history["fp64"][1:]):
        n, rho = h32["step"], h32["rho_max"]
        assert 0 <= h32["gauss"] <= 2 * eps * (e0 / dmin) * np.sqrt(n) + eps * rho, h32
        assert 0 <= h32["cont"] <= 4 * eps * rho * (1 / w.dt + 2 / dmin), h32
        rho = h64["rho_max"]
        assert 0 <= h64["gauss"] <= 1e-10 * rho and 0 <= h64["cont"] <= 1e-10 * rho / w.dt, h64
    assert g32.status() == 0 and g64.status() == 0
