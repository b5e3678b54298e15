"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Each one-step test drives both sides from the same state (FP32-representable
particles and fields) and compares, after one step, every component of the
current before and after the filter (Jx, Jy, Jz) and of the fields (Ex .. Bz)
by relative L2 and element by element, and every particle paired one to one
with its oracle counterpart, component by component.  Tolerances (FP32 path;
FP64 path in brackets): relative L2 <= 1e-5 [1e-11] per component;
max |gpu - oracle| <= 1e-5 [1e-11] * max |oracle| per component; positions
within 2e-6 [1e-12] cells and momenta within 1e-5 [1e-11] of the largest |u|.
"""
import math
import os
import zlib

import numpy as np
import pytest

from inputs import (LaserSpec, SpeciesSpec, Workload, clouds1024, lwfa, lwfa2000x512,
                    random_particles, thermal64, weibel512)
from parity_util import (TOL_STEP_FP32, add_species, compare_state,
                         oracle_from_workload, oracle_mirror, round_to_f32)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - the GPU suite needs an MI355X
    pytest.skip("no GPU", allow_module_level=True)

from paper_2106_12485_amd import PIC_E_CAPACITY, PicError, Simulation  # noqa: E402


def step_both(sim, o, direct=False):
    if direct:
        sim.deposit()
        sim.field_advance()
    else:
        sim.step(1)
    o.step(1)


def random_state(w, rng, uth=0.4, famp=0.2, n_per_species=None):
    parts = []
    for k, s in enumerate(w.species):
        n = n_per_species or w.nx * w.ny * s.ppc[0] * s.ppc[1]
        xr = (1, w.nx - 1) if w.moving_window else None
        parts.append(round_to_f32(random_particles(rng, w.nx, w.ny, n, uth=uth, ufl=s.ufl,
                                                   x_range=xr)))
    f = (famp * rng.standard_normal((6, w.ny, w.nx))).astype(np.float32).astype(np.float64)
    return parts, f


def setup_pair(w, parts, f, fp64=False, it=0, nshift=0, capacity_factor=0.0,
               deposit="reduction"):
    sim = Simulation(w, fp64=fp64, load=False, capacity_factor=capacity_factor,
                     deposit=deposit)
    o = oracle_from_workload(w)
    add_species(o, w, load=False)
    for k, p in enumerate(parts):
        sim.set_particles(k, p)
        o.set_particles(k, p)
    sim.set_fields(f)
    o.set_fields(f)
    if it or nshift:
        sim.set_time(it, nshift)
        o.set_iter(it, nshift)
    return sim, o


def two_species(nx, ny, lx, ly, dt=0.07, **kw):
    sp = [SpeciesSpec(-1.0, 1.0, ppc=(2, 2), uth=(0.3,) * 3),
          SpeciesSpec(0.5, 0.5, ppc=(2, 1), uth=(0.2,) * 3, ufl=(0.3, -0.2, 0.1))]
    return Workload("t", nx, ny, lx, ly, dt, 1, sp, **kw)


CASES = {
    # name: (workload, fp64, direct launches)
    "ragged_40x36_comp": (two_species(40, 36, 4.0, 3.6, filter_passes=1, filter_compensate=True),
                          False, False),
    "ragged_40x36_fp64": (two_species(40, 36, 4.0, 3.6, filter_passes=1, filter_compensate=True),
                          True, False),
    "no_filter_direct": (two_species(34, 18, 3.4, 1.8, filter_passes=0), False, True),
    "three_passes": (two_species(48, 32, 4.8, 3.2, filter_passes=3, filter_compensate=True),
                     False, False),
    # three strips of columns (the last one ragged) and five of rows; halo 3
    "two_passes_comp_130x40": (two_species(130, 40, 13.0, 4.0, filter_passes=2,
                                           filter_compensate=True), False, False),
    # odd sizes against the streaming strips (61/59/57/55 columns by 6 rows for
    # filter + Yee, 4-tile rows for the fold): ragged strips on both axes
    "odd_67x9": (two_species(67, 9, 6.7, 0.9, filter_passes=1), False, False),
    "odd_66x66_three": (two_species(66, 66, 6.6, 6.6, filter_passes=3), False, False),
    "odd_62x31_four": (two_species(62, 31, 6.2, 3.1, filter_passes=4), False, False),
    "narrow_3x70": (two_species(3, 70, 0.3, 7.0, filter_passes=1), False, False),
    # the FP64 instances of the streaming kernels, filter halos 1, 3 and 4
    "odd_67x9_fp64": (two_species(67, 9, 6.7, 0.9, filter_passes=1), True, False),
    "two_passes_comp_130x40_fp64": (two_species(130, 40, 13.0, 4.0, filter_passes=2,
                                                filter_compensate=True), True, False),
    "odd_62x31_four_fp64": (two_species(62, 31, 6.2, 3.1, filter_passes=4), True, False),
    "window_121x23": (two_species(121, 23, 2.42, 4.6, dt=0.014, moving_window=True,
                                  filter_passes=2, filter_compensate=True), False, False),
    "single_tile_4x4": (two_species(4, 4, 0.4, 0.4, filter_passes=1), False, False),
    "single_tile_2x2": (two_species(2, 2, 0.2, 0.2, filter_passes=2), False, True),
    "two_tiles_wrap_18x20": (two_species(18, 20, 1.8, 2.0, filter_passes=1), False, False),
    "anisotropic_cells": (two_species(64, 20, 1.28, 4.0, dt=0.0185, filter_passes=1), False, False),
    "window_60x20": (two_species(60, 20, 1.2, 4.0, dt=0.014, moving_window=True,
                                 filter_passes=1, filter_compensate=True), False, False),
    "window_60x20_fp64": (two_species(60, 20, 1.2, 4.0, dt=0.014, moving_window=True,
                                      filter_passes=1, filter_compensate=True), True, True),
    # 2 x 256 particles per cell: tiles loaded past 65,536 take 1024-thread push blocks
    "big_tiles_36x34": (Workload("big", 36, 34, 3.6, 3.4, 0.07, 1,
                                 [SpeciesSpec(-1.0, 1.0, ppc=(16, 16), uth=(0.3,) * 3),
                                  SpeciesSpec(1.0, 1.0, ppc=(16, 16), uth=(0.3,) * 3,
                                              ufl=(0.0, 0.0, 0.5))],
                                 filter_passes=1), False, False),
    "big_tiles_36x34_fp64": (Workload("big", 36, 34, 3.6, 3.4, 0.07, 1,
                                      [SpeciesSpec(-1.0, 1.0, ppc=(16, 16), uth=(0.3,) * 3),
                                       SpeciesSpec(1.0, 1.0, ppc=(16, 16), uth=(0.3,) * 3,
                                                   ufl=(0.0, 0.0, 0.5))],
                                      filter_passes=1), True, False),
    # a window narrower than a tile: the shift takes its separate launches
    "window_12x20": (two_species(12, 20, 0.24, 4.0, dt=0.014, moving_window=True,
                                 filter_passes=1, filter_compensate=True), False, False),
    # one-cell last tiles (n % 16 == 1): the fold searches two tiles each way;
    # along x (fold inside the Yee launch), along y with the compensator (the
    # separate fold launch), both with two tiles per axis (wrap), FP64, the
    # window, and tiles with one push block per species (64-bit slices)
    "thin_x_33x20": (two_species(33, 20, 3.3, 2.0, filter_passes=1), False, False),
    "thin_y_20x33_comp": (two_species(20, 33, 2.0, 3.3, filter_passes=1,
                                      filter_compensate=True), False, False),
    "thin_both_17x17": (two_species(17, 17, 1.7, 1.7, filter_passes=1), False, True),
    "thin_49x33_fp64": (two_species(49, 33, 4.9, 3.3, filter_passes=1), True, False),
    "thin_window_60x17": (two_species(60, 17, 1.2, 3.4, dt=0.014, moving_window=True,
                                      filter_passes=1, filter_compensate=True), False, False),
    "thin_big_tiles_33x17": (Workload("big", 33, 17, 3.3, 1.7, 0.07, 1,
                                      [SpeciesSpec(-1.0, 1.0, ppc=(16, 16), uth=(0.3,) * 3),
                                       SpeciesSpec(1.0, 1.0, ppc=(16, 16), uth=(0.3,) * 3,
                                                   ufl=(0.0, 0.0, 0.5))],
                                      filter_passes=1), False, False),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_one_step_matches_oracle(name):
    w, fp64, direct = CASES[name]
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    parts, f = random_state(w, rng)
    # with the window, start one step before a shift so that it is exercised
    it = 0
    if w.moving_window:
        it = int(math.ceil(3 * w.dx / w.dt)) - 1
    nsh = int(it * w.dt / w.dx + 1e-12) if w.moving_window else 0
    sim, o = setup_pair(w, parts, f, fp64=fp64, it=it, nshift=nsh)
    step_both(sim, o, direct)
    if w.moving_window:
        assert o.nshift == nsh + 1
    compare_state(sim, o, w, fp64, name)
    assert sim.status() == 0


# empty and sparse particle sets: (workload, particles per species, fp64)
SPARSE = {
    "vacuum_40x36": (two_species(40, 36, 4.0, 3.6, filter_passes=1, filter_compensate=True),
                     (0, 0), False),
    "vacuum_window_60x20_fp64": (two_species(60, 20, 1.2, 4.0, dt=0.014, moving_window=True,
                                             filter_passes=1), (0, 0), True),
    "one_species_empty_40x36": (two_species(40, 36, 4.0, 3.6, filter_passes=2), (0, 2880), False),
    "seven_particles_40x36": (two_species(40, 36, 4.0, 3.6, filter_passes=1), (4, 3), False),
    "three_particles_window_60x20": (two_species(60, 20, 1.2, 4.0, dt=0.014, moving_window=True,
                                                 filter_passes=1, filter_compensate=True),
                                     (2, 1), False),
    # the largest grid extents (65535 cells: cell indices use 16 bits each,
    # unsigned; ragged last tile of 15 cells), a few hundred particles; the
    # window's storage adds an 18-cell gap, so its largest nx is 65518
    "max_nx_65535x18": (two_species(65535, 18, 6553.5, 1.8, filter_passes=1), (300, 200), False),
    "max_ny_18x65535": (two_species(18, 65535, 1.8, 6553.5, filter_passes=1,
                                    filter_compensate=True), (300, 200), False),
    "max_nx_window_65518x18": (two_species(65518, 18, 1310.36, 3.6, dt=0.014, moving_window=True,
                                           filter_passes=1), (300, 200), False),
    # one-cell last tiles along both axes, then 5 more steps of hand-offs
    "thin_17x33": (two_species(17, 33, 1.7, 3.3, filter_passes=1), (400, 300), False),
}


@pytest.mark.parametrize("name", sorted(SPARSE))
def test_empty_and_sparse_particle_sets_match_oracle(name):
    """One step with no particles at all (the field solver alone), with one
    species empty, with a handful of particles leaving almost every tile
    empty, and on the largest grid extents; the window cases start one step
    before a shift."""
    w, counts, fp64 = SPARSE[name]
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    parts = []
    for s, n in zip(w.species, counts):
        xr = (1, w.nx - 1) if w.moving_window else None
        parts.append(round_to_f32(random_particles(rng, w.nx, w.ny, n, uth=0.4, ufl=s.ufl,
                                                   x_range=xr)))
    f = (0.2 * rng.standard_normal((6, w.ny, w.nx))).astype(np.float32).astype(np.float64)
    it = int(math.ceil(3 * w.dx / w.dt)) - 1 if w.moving_window else 0
    nsh = int(it * w.dt / w.dx + 1e-12) if w.moving_window else 0
    sim, o = setup_pair(w, parts, f, fp64=fp64, it=it, nshift=nsh)
    for k, n in enumerate(counts):
        assert sim.count(k) == o.count(k) == n
    step_both(sim, o, False)
    if w.moving_window:
        assert o.nshift == nsh + 1
    compare_state(sim, o, w, fp64, name)
    if sum(counts) == 0:
        assert not sim.get_current(False).any()
    # a few more steps on the GPU alone: the counts hold and nothing overflows
    sim.step(5)
    e = sim.energy()
    assert e["status"] == 0 and sim.status() == 0
    if not w.moving_window:
        assert list(e["n_particles"]) == list(counts)


@pytest.mark.parametrize("fp64", [False, True])
def test_loader_matches_oracle(fp64):
    w = Workload("load", 40, 34, 4.0, 3.4, 0.07, 1,
                 [SpeciesSpec(-1.0, 1.0, 0.0, 2.0, (4, 2), (0.05, 0.1, 0.2), (0.6, 0.0, -0.1)),
                  SpeciesSpec(-0.5, 0.7, 2.05, 4.0, (3, 3), (0.02,) * 3, (-0.6, 0.1, 0.0))],
                 seed=0x5EED1234ABCD)
    sim = Simulation(w, fp64=fp64)
    o = oracle_from_workload(w)
    add_species(o, w, load=True)
    for k, s in enumerate(w.species):
        pg, po = sim.get_particles(k), o.get_particles(k)
        assert len(pg["ix"]) == len(po["ix"]) > 0

        def order(p):
            return np.lexsort((np.round(p["x"] * s.ppc[0] * 2), np.round(p["y"] * s.ppc[1] * 2),
                               p["ix"], p["iy"]))
        a, b = order(pg), order(po)
        assert np.array_equal(pg["ix"][a], po["ix"][b])
        assert np.array_equal(pg["iy"][a], po["iy"][b])
        t = 1e-15 if fp64 else 1e-7
        for c in ("x", "y"):
            assert np.abs(pg[c][a] - po[c][b]).max() <= t
        for c in ("ux", "uy", "uz"):
            assert np.abs(pg[c][a] - po[c][b]).max() <= (1e-14 if fp64 else 1e-6) * (
                1 + np.abs(po[c]).max())


def test_laser_initial_fields_match_oracle():
    w = lwfa(nx=400, ny=64, lx=8.0, ly=12.8, steps=1, x_plasma=6.0)
    w.laser = LaserSpec(2.0, 10.0, 4.0, 2.0, 3.0, 5.0, 6.4, math.pi / 3)
    sim = Simulation(w)
    o = oracle_from_workload(w)
    add_species(o, w, load=True)
    fg, fo = sim.get_fields(), o.get_fields()
    assert np.abs(fo).max() > 10
    assert np.abs(fg - fo).max() <= 2e-6 * np.abs(fo).max()


def test_multi_step_migration_then_teacher_forced_step():
    # fast particles in a small box: many tile crossings per step
    w = two_species(40, 36, 4.0, 3.6, filter_passes=1, filter_compensate=True)
    rng = np.random.default_rng(11)
    parts, f = random_state(w, rng, uth=0.8, famp=0.1)
    sim, o = setup_pair(w, parts, f)
    n0 = [sim.count(k) for k in range(2)]
    sim.step(25)
    assert [sim.count(k) for k in range(2)] == n0
    assert sim.status() == 0
    om = oracle_mirror(sim, w)
    step_both(sim, om)
    compare_state(sim, om, w, False, "after 25 steps")


def test_graph_replay_equals_direct_launches():
    w = two_species(40, 36, 4.0, 3.6, filter_passes=1, filter_compensate=True)
    rng = np.random.default_rng(12)
    parts, f = random_state(w, rng)
    a, _ = setup_pair(w, parts, f)
    b, _ = setup_pair(w, parts, f)
    a.step(10)
    for _ in range(10):
        b.deposit()
        b.field_advance()
    # the current is summed in fixed point, independent of particle order, so
    # both launch paths give bitwise identical fields and particle sets
    assert [a.count(k) for k in range(2)] == [b.count(k) for k in range(2)] == \
        [len(p["ix"]) for p in parts]
    assert np.array_equal(a.get_fields(), b.get_fields())
    keys = ("uz", "uy", "ux", "y", "x", "iy", "ix")
    for k in range(2):
        pa, pb = a.get_particles(k), b.get_particles(k)
        oa = np.lexsort([pa[c] for c in keys])
        ob = np.lexsort([pb[c] for c in keys])
        for c in keys:
            assert np.array_equal(pa[c][oa], pb[c][ob]), c


@pytest.mark.parametrize("window", [False, True])
def test_filtered_current_requests_change_nothing(window):
    """The step filters J inside its field-solver launch; a request for the
    filtered current filters the stored J on its own.  Requests between the
    steps must leave the run bit for bit as it was, and each must return the
    current that step's solver used: the one of a run that filters in a
    launch of its own (the batched path) over the same steps."""
    if window:
        w = two_species(60, 20, 1.2, 4.0, dt=0.014, moving_window=True, filter_passes=1,
                        filter_compensate=True)
    else:
        w = two_species(40, 36, 4.0, 3.6, filter_passes=2, filter_compensate=True)
    rng = np.random.default_rng(31)
    parts, f = random_state(w, rng)
    a, _ = setup_pair(w, parts, f)
    b, _ = setup_pair(w, parts, f)
    jf = []
    for _ in range(12):
        a.step(1)
        jf.append(a.get_current(True))
        jf.append(a.get_current(True))
    b.step(12)
    assert np.array_equal(a.get_fields(), b.get_fields())
    assert np.array_equal(a.get_current(False), b.get_current(False))
    assert np.array_equal(jf[-1], b.get_current(True))
    for x, y in zip(jf[0::2], jf[1::2]):
        assert np.array_equal(x, y)
    if not window:
        # a batch of one filters in the tile-form launch of its own
        from paper_2106_12485_amd import Batch
        c, _ = setup_pair(w, parts, f)
        bt = Batch(1, c.layout()["ntx"] * c.layout()["nty"])
        for n in range(12):
            bt.step([c], 1)
            assert np.array_equal(c.get_current(True), jf[2 * n]), n
        assert np.array_equal(c.get_fields(), b.get_fields())
        bt.close()


def test_set_get_roundtrip_is_exact():
    w = two_species(40, 36, 4.0, 3.6)
    rng = np.random.default_rng(13)
    parts, f = random_state(w, rng)
    sim, _ = setup_pair(w, parts, f)
    assert np.array_equal(sim.get_fields(), f)
    for k, p in enumerate(parts):
        q = sim.get_particles(k)
        a = np.lexsort((p["x"], p["y"], p["ix"], p["iy"]))
        b = np.lexsort((q["x"], q["y"], q["ix"], q["iy"]))
        for c in ("ix", "iy", "x", "y", "ux", "uy", "uz"):
            assert np.array_equal(np.asarray(p[c])[a], q[c][b]), c


def test_thermal_64x64_invariants_and_oracle_parity():
    """The 64x64 thermal plasma (16 ppc, uth 0.1, 100 steps): teacher-forced
    one-step parity at steps 0, 50 and 99; Gauss and continuity residuals at
    FP32 round-off every 10 steps; free-running energy against the oracle's
    every 10 steps, within max(1e-4, 10x the oracle's own spread under a
    permutation of the particle order) of the initial energy."""
    w = thermal64()
    sim = Simulation(w)
    o = oracle_from_workload(w)
    add_species(o, w, load=True)
    # the same oracle run with its particles in another order: round-off of
    # the current sums only, the paper's yardstick for equally correct results
    op = oracle_from_workload(w)
    add_species(op, w, load=True)
    p = op.get_particles(0)
    perm = np.random.default_rng(5).permutation(len(p["ix"]))
    op.set_particles(0, {k: v[perm] for k, v in p.items()})
    assert sim.count(0) == o.count(0) == 65536
    e0g, e0o = sim.energy(), o.energy()
    W0 = e0o["total"]
    assert abs(e0g["total"] - W0) / W0 < 1e-6
    dev, spread = [], []

    def energies(eg):
        eo = o.energy()["total"]
        dev.append(abs(eg - eo) / W0)
        spread.append(abs(op.energy()["total"] - eo) / W0)

    for n in range(100):
        if n in (0, 50, 99):
            om = oracle_mirror(sim, w)
            step_both(sim, om)
            compare_state(sim, om, w, False, "step %d" % n)
        else:
            sim.step(1)
        o.step(1)
        op.step(1)
        if n % 10 == 9:
            e = sim.energy()
            scale = e["rho_max"]
            # FP32 round-off of rho (~64 terms per node) and of the E updates
            assert e["gauss_res_max"] < 1e-4 * max(scale, 1.0), e
            energies(e["total"])
    # continuity residual needs two diagnostics one step apart
    sim.energy()
    sim.step(1)
    o.step(1)
    op.step(1)
    e = sim.energy()
    assert 0 <= e["cont_res_max"] < 2e-4 * e["rho_max"] / w.dt, e
    energies(e["total"])
    bound = max(1e-4, 10 * max(spread))
    assert max(dev) < bound, (dev, spread)


def test_capacity_overflow_is_reported():
    w = thermal64()
    with pytest.raises(PicError) as ei:
        Simulation(w, capacity_factor=0.5)
    assert ei.value.code == PIC_E_CAPACITY
    # slots exactly equal to the initial load of a full tile: net inflow into
    # any tile overflows and the device flag is raised
    sim = Simulation(w, capacity_factor=1.0)
    sim.step(20)
    assert sim.status() == PIC_E_CAPACITY
    assert sim.energy()["status"] == PIC_E_CAPACITY


def test_particle_count_beyond_the_slots_is_refused_before_any_read():
    # a count above the species' slots is refused before the arrays are read
    # or any host buffer is sized by it; the simulation carries on
    from paper_2106_12485_amd import pic
    w = thermal64()
    sim = Simulation(w)
    one_i = np.zeros(1, np.int32)
    one_d = np.zeros(1)
    rc = pic.lib().pic_set_particles(sim._h, 0, 1 << 61, pic._ip(one_i), pic._ip(one_i),
                                     *[pic._dp(one_d)] * 5, sim._sp())
    assert rc == PIC_E_CAPACITY
    assert "slots" in pic.lib().pic_last_error().decode()
    sim.step(3)
    assert sim.status() == 0 and sim.count(0) == 65536


def test_lwfa_window_run_counts_and_teacher_forced_shift():
    # reduced laser-wakefield geometry with the moving window
    w = lwfa(nx=300, ny=32, lx=6.0, ly=6.4, steps=40, x_plasma=4.0, ppc=(2, 2))
    w.laser = LaserSpec(2.0, 10.0, 1.5, 1.0, 2.0, 3.0, 3.2, math.pi / 2)
    sim = Simulation(w)
    o = oracle_from_workload(w)
    add_species(o, w, load=True)
    assert sim.count(0) == o.count(0)
    for n in range(30):
        if n in (0, 13, 27):
            om = oracle_mirror(sim, w)
            step_both(sim, om)
            compare_state(sim, om, w, False, "window step %d" % n)
        else:
            sim.step(1)
    e = sim.energy()
    assert e["nshift"] == int(30 * w.dt / w.dx + 1e-9)
    o.step(30)
    assert o.nshift == e["nshift"]
    # cold plasma: the count changes only through the columns that leave and enter
    assert abs(sim.count(0) - o.count(0)) <= 8


def _full_size_parity(w, nsteps, deposit="reduction"):
    sim = Simulation(w, deposit=deposit)
    n0 = sim.count(0)
    assert n0 > 0
    sim.step(nsteps)
    assert sim.status() == 0
    om = oracle_mirror(sim, w)
    om.set_threads(min(16, os.cpu_count() or 1))
    step_both(sim, om)
    return compare_state(sim, om, w, False, w.name)


def _mirror_step(sim, w, what):
    om = oracle_mirror(sim, w)
    om.set_threads(min(16, os.cpu_count() or 1))
    step_both(sim, om)
    return compare_state(sim, om, w, False, what)


def _energy_run(w, checkpoints, tf_steps, oracle_steps, bounds):
    """Run workload w over its whole length on the FP32 path and, beside it,
    on the FP64 GPU path, both from the library's own load.
      - total energy of the FP32 run against a free-running FP64 oracle run
        from its own load, every 10 steps over the first oracle_steps steps;
      - FP32 against FP64 GPU total energy, and the drift of both, at the
        checkpoints;
      - a teacher-forced step against the oracle after each step count in
        tf_steps (the step is one of the run's own);
      - device status at every checkpoint.
    bounds: (FP32 vs oracle, FP32 vs FP64 GPU, absolute drift of either),
    each relative to the initial total energy W(0).  Returns the two
    simulations, the initial counts and the history."""
    s32 = Simulation(w)
    s64 = Simulation(w, fp64=True)
    o = oracle_from_workload(w)
    add_species(o, w, load=True)
    o.set_threads(min(16, os.cpu_count() or 1))
    ns = len(w.species)
    n0 = [s32.count(k) for k in range(ns)]
    assert n0 == [s64.count(k) for k in range(ns)] == [o.count(k) for k in range(ns)]
    W0 = o.energy()["total"]
    assert abs(s32.energy()["total"] / W0 - 1) < 1e-6
    assert abs(s64.energy()["total"] / W0 - 1) < 1e-12
    b_ora, b_64, b_drift = bounds
    dev_ora, hist = [], []
    events = sorted(set(checkpoints) | set(tf_steps) | set(range(10, oracle_steps + 1, 10)))
    done = 0

    def advance(k):
        s32.step(k)
        s64.step(k)
        if done < oracle_steps:
            o.step(k)

    for n in events:
        assert n >= done, (n, done)
        if n > done:
            advance(n - done)
            done = n
        if n <= oracle_steps and n % 10 == 0:
            dev_ora.append(abs(s32.energy()["total"] - o.energy()["total"]) / W0)
        if n in checkpoints:
            a, b = s32.energy(), s64.energy()
            hist.append((n, a["total"] / W0 - 1, b["total"] / W0 - 1,
                         abs(a["total"] - b["total"]) / W0))
            print("step %4d  drift32 %+.3e  drift64 %+.3e  |32-64| %.3e  gauss %.2e  cont %.2e"
                  % (n, hist[-1][1], hist[-1][2], hist[-1][3], a["gauss_res_max"],
                     a["cont_res_max"]), flush=True)
            assert a["status"] == 0 and b["status"] == 0, n
        if n in tf_steps:
            om = oracle_mirror(s32, w)
            om.set_threads(min(16, os.cpu_count() or 1))
            s64.step(1)
            if done < oracle_steps:
                o.step(1)
            step_both(s32, om)
            compare_state(s32, om, w, False, "%s after %d steps" % (w.name, n))
            om.close()
            done += 1
    o.close()
    print("energy vs oracle, worst over %d steps: %.3e" % (oracle_steps, max(dev_ora)), flush=True)
    assert max(dev_ora) < b_ora, dev_ora
    assert max(h[3] for h in hist) < b_64, hist
    assert max(max(abs(h[1]), abs(h[2])) for h in hist) < b_drift, hist
    assert s32.status() == 0 and s64.status() == 0
    return s32, s64, n0, hist


@pytest.mark.timeout(900)
def test_clouds_1024_whole_run_energy_and_teacher_forced_steps():
    """The two-cloud run (16.8M particles) over its stated 1000 steps: no tile
    or outbox runs out of slots while the clouds interpenetrate; total energy
    against the oracle over a 30-step prefix (bound 1e-4 of W(0), the paper's
    round-off yardstick, as for the thermal run), FP32 against FP64 GPU and the
    drift of both every 100 steps; teacher-forced steps as the 6th, 501st and
    1000th steps; particle counts conserved (periodic box)."""
    w = clouds1024()
    s32, s64, n0, hist = _energy_run(
        w, checkpoints=range(100, 1001, 100), tf_steps=(5, 500, 999), oracle_steps=30,
        bounds=(1e-4, 1e-3, 2e-2))
    assert [s32.count(k) for k in range(2)] == n0 == [s64.count(k) for k in range(2)]
    e = s32.energy()
    assert e["step"] == 1000


def test_clouds_1024_thousand_steps_without_a_settle():
    """The two-cloud run's 1000 steps in one call, so that no host read
    settles the pending leavers in between.  Near step 770 dense bunches of
    the two-stream instability sweep into tiles at about 8 times the inflow
    seen at the last periodic layout check; the pushes then ask for a
    relayout at the step end, and no segment runs out of slots."""
    s = Simulation(clouds1024())
    n0 = s.energy()["n_particles"]
    s.step(1000)
    assert s.status() == 0
    e = s.energy()
    assert e["status"] == 0 and e["step"] == 1000
    assert np.array_equal(e["n_particles"], n0)


@pytest.mark.parametrize("deposit", ["reduction", "commutative"])
def test_timed_steps_match_the_graph_and_time_every_push(deposit):
    """pic_timing: the same 20 steps launched directly, with HIP events
    around each kernel class (one push launch with the reduction deposit,
    five with the commutative one), end with the fields bitwise those of the
    graph replay (the current sums are exact integers); one push time per
    step, each positive, their sum below the steps' wall time."""
    import time
    import torch
    w = thermal64()
    a, b = Simulation(w, deposit=deposit), Simulation(w, deposit=deposit)
    a.step(20)
    b.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(20)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    tk = b.timing_read()
    b.timing(False)
    ms, n = tk["push_deposit"]
    assert n == 20 and 0 < ms < wall_ms
    assert tk["yee"][1] == 20
    assert np.array_equal(a.get_fields(), b.get_fields())
    ea, eb = a.energy(), b.energy()
    assert ea["step"] == eb["step"] == 20 and ea["status"] == eb["status"] == 0
    assert np.array_equal(ea["n_particles"], eb["n_particles"])
    np.testing.assert_allclose(eb["ke"], ea["ke"], rtol=1e-12)


@pytest.mark.timeout(900)
def test_lwfa_2000x256_whole_run_energy_and_teacher_forced_steps():
    """The 2000 x 256 laser-wakefield run over its stated 500 steps: total
    energy against a free-running oracle over all 500 steps (the cold plasma
    is driven by the laser, not chaotic), FP32 against FP64 GPU every 50
    steps, teacher-forced steps at 12, 250 and 500 steps, window shifts and
    particle counts against the oracle's."""
    w = lwfa()
    s32, s64, n0, hist = _energy_run(
        w, checkpoints=range(50, 501, 50), tf_steps=(12, 250, 499), oracle_steps=500,
        bounds=(1e-4, 1e-4, 5e-2))
    e = s32.energy()
    assert e["step"] == 500 and e["nshift"] == int(500 * w.dt / w.dx + 1e-9)


@pytest.mark.timeout(900)
def test_weibel_512_full_size_teacher_forced():
    # electron and positron clouds, 256 particles per cell each (134M particles)
    w = weibel512()
    errs = _full_size_parity(w, 3)
    assert errs["J"] < TOL_STEP_FP32


@pytest.mark.timeout(900)
def test_weibel_512_paper_length_run():
    """The paper's Weibel run over its whole length, 500 steps, then a
    teacher-forced step against the oracle.

    Pins along the way (eps = 2^-24):
      - a periodic box loses no particle;
      - the counter-streaming clouds are unstable to filamentation, whose
        growth rate (about u_fl / gamma^(3/2) of the plasma frequency, 0.5 here)
        lifts the magnetic energy from the noise level at step 20 by far more
        than 100x by step 500;
      - field plus kinetic energy changes only by the scheme's numerical
        heating: under 1% over the run;
      - no tile runs out of slots although the filaments pile particles up
        (status stays 0);
      - Gauss and continuity residuals stay at FP32 rounding, with the bounds
        of the precision study (E0 the largest |E| seen).
    """
    w = weibel512()
    sim = Simulation(w)
    n0 = [sim.count(k) for k in range(2)]
    assert n0 == [512 * 512 * 256] * 2
    hist = {0: sim.energy()}
    done = 0
    for n in (20, 100, 250, 499, 500):
        sim.step(n - done)
        done = n
        hist[n] = sim.energy()
        print("step %3d  E %.4e  B %.4e  KE %.6e  total %.9e  gauss %.2e  cont %.2e" % (
            n, hist[n]["e_energy"], hist[n]["b_energy"], float(np.sum(hist[n]["ke"])),
            hist[n]["total"], hist[n]["gauss_res_max"], hist[n]["cont_res_max"]), flush=True)
    assert sim.status() == 0
    assert [sim.count(k) for k in range(2)] == n0
    assert [int(v) for v in hist[500]["n_particles"]] == n0
    assert hist[500]["b_energy"] > 100 * hist[20]["b_energy"] > 0
    assert abs(hist[500]["total"] / hist[0]["total"] - 1) < 0.01
    eps = 2.0 ** -24
    dmin = min(w.lx / w.nx, w.ly / w.ny)
    e0 = float(np.abs(sim.get_fields()[:3]).max())
    e = hist[500]
    rho = e["rho_max"]
    assert 0 <= e["gauss_res_max"] <= 2 * eps * (e0 / dmin) * math.sqrt(500) + eps * rho, e
    assert 0 <= e["cont_res_max"] <= 4 * eps * rho * (1 / w.dt + 2 / dmin), e
    om = oracle_mirror(sim, w)
    om.set_threads(min(16, os.cpu_count() or 1))
    step_both(sim, om)
    errs = compare_state(sim, om, w, False, w.name)
    assert errs["J"] < TOL_STEP_FP32


# ---------------------------------------------------------------------------
# the commutative deposit: four checkerboard colours add straight into J
# ---------------------------------------------------------------------------
COMMUTATIVE_CASES = {
    # name: (workload, fp64); even tile counts, ragged last tiles
    "ragged_56x56_comp": (two_species(56, 56, 5.6, 5.6, filter_passes=1, filter_compensate=True),
                          False),
    # the narrowest last tile the commutative deposit accepts: 3 cells
    "last_tile_3_51x51": (two_species(51, 51, 5.1, 5.1, filter_passes=1), False),
    "two_tiles_24x32": (two_species(24, 32, 2.4, 3.2, filter_passes=1), False),
    "fp64_64x32": (two_species(64, 32, 6.4, 3.2, filter_passes=2), True),
}


@pytest.mark.parametrize("name", sorted(COMMUTATIVE_CASES))
def test_commutative_deposit_one_step_matches_oracle(name):
    w, fp64 = COMMUTATIVE_CASES[name]
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    parts, f = random_state(w, rng)
    sim, o = setup_pair(w, parts, f, fp64=fp64, deposit="commutative")
    step_both(sim, o)
    compare_state(sim, o, w, fp64, name)
    assert sim.status() == 0


def test_commutative_deposit_migration_then_teacher_forced_step():
    w = two_species(56, 56, 5.6, 5.6, filter_passes=1, filter_compensate=True)
    rng = np.random.default_rng(21)
    parts, f = random_state(w, rng)
    sim, _ = setup_pair(w, parts, f, deposit="commutative")
    a, _ = setup_pair(w, parts, f, deposit="commutative")
    sim.step(15)
    for _ in range(15):
        a.deposit()
        a.field_advance()
    # colour order is fixed, so graph replay and direct launches agree bitwise
    assert np.array_equal(sim.get_fields(), a.get_fields())
    assert [sim.count(k) for k in range(2)] == [len(p["ix"]) for p in parts]
    om = oracle_mirror(sim, w)
    step_both(sim, om)
    compare_state(sim, om, w, False, "commutative after 15 steps")


def test_clouds_1024_commutative_full_size_teacher_forced():
    # 600 steps first: the cloud fronts move into empty tiles, whose particle
    # segments the layout check (k_order) must grow in this mode too
    errs = _full_size_parity(clouds1024(), 600, deposit="commutative")
    assert errs["J"] < TOL_STEP_FP32


@pytest.mark.timeout(900)
def test_lwfa_2000x512_paper_scale_run():
    # the paper's LWFA size, all 4000 steps, then a teacher-forced step
    w = lwfa2000x512()
    sim = Simulation(w)
    sim.step(w.steps)
    e = sim.energy()
    assert e["status"] == 0 and e["step"] == w.steps
    assert e["nshift"] == int(w.steps * w.dt / w.dx + 1e-9)
    # the window has left the vacuum behind: plasma (16 per cell) fills the box,
    # up to the particles the wake moved across the window's edges
    full = w.nx * w.ny * 16
    assert 0.95 * full < e["n_particles"][0] < 1.02 * full
    om = oracle_mirror(sim, w)
    om.set_threads(min(16, os.cpu_count() or 1))
    step_both(sim, om)
    compare_state(sim, om, w, False, w.name)


# ---------------------------------------------------------------------------
# floating-point edge cases of the move and of the gather (FP32 offsets)
# ---------------------------------------------------------------------------
def edge_particles(w, rng, fp64):
    """Particles placed on the edges of the cell update and of the deposit
    split, plus random fillers.  With zero fields the momenta are unchanged
    by the push, so the displacement is dt/dx * u / gamma to within rounding.
    Returns the particle dict; d = dt/dx = dt/dy."""
    d = w.dt / w.dx
    assert abs(w.dt / w.dy - d) < 1e-15
    tiny = 2.0 ** -31
    below1 = 1.0 - 2.0 ** -24          # the largest FP32 offset below 1
    rows = []

    def add(ix, iy, x, y, ddx, ddy, uz=0.0):
        # proper velocity that moves by (ddx, ddy) cells: v = dd / d, u = v gamma
        vx, vy = ddx / d, ddy / d
        g = 1.0 / math.sqrt(1.0 - vx * vx - vy * vy)
        rows.append((ix, iy, x, y, vx * g, vy * g, uz))

    for ix, iy in ((5, 7), (15, 16), (16, 15), (0, 0), (w.nx - 1, w.ny - 1)):
        # x + dx in (-2^-25, 0): adding 1 rounds to exactly 1 in FP32
        add(ix, iy, tiny, 0.3, -1e-8, 0.0)
        add(ix, iy, 0.3, tiny, 0.0, -1e-8)
        # landing on exactly 1.0 in FP32 (a tie rounded to even): the offset
        # below 1 moved by 3/4 of its ulp; the oracle stays just below 1
        add(ix, iy, below1, 0.6, 0.75 * 2.0 ** -24, 0.0)
        add(ix, iy, 0.6, below1, 0.0, 0.75 * 2.0 ** -24)
        # moving right across the edge from just below it
        add(ix, iy, below1, 0.2, 0.3, 0.1)
        # exact corner crossings: both edges at the same path fraction
        add(ix, iy, 0.75, 0.75, 0.45, 0.45)
        add(ix, iy, 0.25, 0.25, -0.45, -0.45)
        add(ix, iy, 0.75, 0.25, 0.45, -0.45)
        add(ix, iy, 0.25, 0.75, -0.45, 0.45, uz=0.3)
        # no motion along one axis, or none at all
        add(ix, iy, 0.3, 0.9, 0.0, 0.3)
        add(ix, iy, 0.9, 0.3, 0.3, 0.0, uz=-0.2)
        add(ix, iy, 0.4, 0.6, 0.0, 0.0)
        # starting exactly on the cell's lower edges
        add(ix, iy, 0.0, 0.5, -0.2, 0.0)
        add(ix, iy, 0.5, 0.0, 0.0, 0.2)
        add(ix, iy, 0.0, 0.0, 0.1, -0.1)
    a = np.array(rows)
    n_fill = 2000
    fill = random_particles(rng, w.nx, w.ny, n_fill, uth=0.3)
    p = dict(ix=np.concatenate([a[:, 0], fill["ix"]]).astype(np.int32),
             iy=np.concatenate([a[:, 1], fill["iy"]]).astype(np.int32))
    for k, c in zip(("x", "y", "ux", "uy", "uz"), range(2, 7)):
        p[k] = np.concatenate([a[:, c], fill[k]])
    return p if fp64 else round_to_f32(p)


@pytest.mark.parametrize("fp64", [False, True])
def test_move_edge_cases_match_oracle(fp64):
    """One step from particles placed on the edges of the cell update: an
    offset that rounds to exactly 1 after a small negative move, a landing on
    exactly 1.0, exact corner crossings, no motion along an axis, starts on
    the lower edges, at tile borders and across the periodic seam; zero
    fields, so every displacement is the one chosen."""
    w = Workload("edges", 40, 36, 4.0, 3.6, 0.07, 1,
                 [SpeciesSpec(-1.0, 1.0, ppc=(2, 2))], filter_passes=1)
    rng = np.random.default_rng(77)
    p = edge_particles(w, rng, fp64)
    f = np.zeros((6, w.ny, w.nx))
    sim, o = setup_pair(w, [p], f, fp64=fp64)
    step_both(sim, o)
    compare_state(sim, o, w, fp64, "move edges")
    assert sim.status() == 0


@pytest.mark.parametrize("fp64", [False, True])
def test_gather_ties_and_cell_corners_match_oracle(fp64):
    """Particles at offsets 1/2 (where each staggered component's bilinear
    weight switches between its two neighbouring grid points: both give the
    same value), on cell corners and just below 1, in random fields."""
    w = Workload("ties", 40, 36, 4.0, 3.6, 0.07, 1,
                 [SpeciesSpec(-1.0, 1.0, ppc=(2, 2))], filter_passes=1)
    rng = np.random.default_rng(78)
    offs = np.array([0.5, 0.0, 1.0 - 2.0 ** -24, 0.25, 0.75])
    ox, oy = np.meshgrid(offs, offs)
    n_cell = 60
    ix = rng.integers(0, w.nx, n_cell)
    iy = rng.integers(0, w.ny, n_cell)
    m = ox.size
    p = dict(ix=np.repeat(ix, m).astype(np.int32), iy=np.repeat(iy, m).astype(np.int32),
             x=np.tile(ox.ravel(), n_cell), y=np.tile(oy.ravel(), n_cell),
             ux=0.3 * rng.standard_normal(m * n_cell), uy=0.3 * rng.standard_normal(m * n_cell),
             uz=0.3 * rng.standard_normal(m * n_cell))
    if not fp64:
        p = round_to_f32(p)
    f = (0.2 * rng.standard_normal((6, w.ny, w.nx))).astype(np.float32).astype(np.float64)
    sim, o = setup_pair(w, [p], f, fp64=fp64)
    step_both(sim, o)
    compare_state(sim, o, w, fp64, "gather ties")
