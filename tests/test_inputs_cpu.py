"""The seeded synthetic inputs match the recipes they state (CPU only)."""
import math

import numpy as np

from inputs import clouds1024, lwfa2000x512, lwfa8000, serving_requests, thermal64, weibel512


def test_serving_stream_recipe():
    a = serving_requests(n_requests=400, rate=50.0)
    b = serving_requests(n_requests=400, rate=50.0)
    assert [(t, w.name, w.species) for t, w in a] == [(t, w.name, w.species) for t, w in b]
    grids, ppcs, kinds, uths, drifts = set(), set(), [], [], []
    for _, w in a:
        assert w.nx == w.ny and w.lx == w.ly == 0.1 * w.nx and w.dt == 0.07
        assert w.steps == 200
        grids.add(w.nx)
        ppcs.add(w.species[0].ppc)
        uths.append(w.species[0].uth[0])
        assert all(s.uth == (w.species[0].uth[0],) * 3 for s in w.species)
        if len(w.species) == 2:
            kinds.append(1)
            s0, s1 = w.species
            assert s0.density == s1.density == 0.5 and s0.ufl[0] == -s1.ufl[0] >= 0.0
            drifts.append(s0.ufl[0])
        else:
            kinds.append(0)
            assert w.species[0].density == 1.0 and w.species[0].ufl == (0.0, 0.0, 0.0)
    assert grids == {64, 128, 256, 512}
    assert ppcs == {(2, 2), (4, 4), (8, 8)}
    assert 0.01 <= min(uths) and max(uths) <= 0.2
    assert 0.0 <= min(drifts) and max(drifts) <= 0.5
    assert abs(np.mean(kinds) - 0.5) < 4 * 0.5 / math.sqrt(len(kinds))
    # Poisson arrivals: exponential gaps of mean 1/rate
    t = np.array([t for t, _ in a])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps >= 0)
    assert abs(gaps.mean() - 1 / 50.0) < 4 * (1 / 50.0) / math.sqrt(len(gaps))
    assert all(t == 0.0 for t, _ in serving_requests(n_requests=10))


def test_benchmark_workloads_have_the_stated_sizes():
    w = clouds1024()
    assert (w.nx, w.ny, w.lx, w.ly, w.dt) == (1024, 1024, 102.4, 102.4, 0.07)
    n = sum(w.nx * w.ny * s.ppc[0] * s.ppc[1] *
            (min(s.x_hi, w.lx) - max(s.x_lo, 0.0)) / w.lx for s in w.species)
    assert round(n) == 16_777_216
    assert [s.ufl[0] for s in w.species] == [0.6, -0.6]
    w = weibel512()
    assert (w.nx, w.ny) == (512, 512) and len(w.species) == 2
    assert sum(w.nx * w.ny * s.ppc[0] * s.ppc[1] for s in w.species) == 134_217_728
    assert [s.qm for s in w.species] == [-1.0, 1.0]
    assert w.species[0].ufl[2] == -w.species[1].ufl[2] != 0.0
    w = lwfa2000x512()
    assert (w.nx, w.ny, w.moving_window, w.filter_compensate) == (2000, 512, True, True)
    assert w.species[0].ppc[0] * w.species[0].ppc[1] == 16 and w.steps == 4000
    w = thermal64()
    assert (w.nx, w.ny, w.species[0].ppc) == (64, 64, (4, 4))
    # the precision study keeps the 2000 x 256 run's cell and step, plasma everywhere
    w = lwfa8000()
    assert (w.nx, w.ny, w.lx, w.ly, w.dt) == (8000, 512, 160.0, 102.4, 0.014)
    assert w.nx * w.ny * w.species[0].ppc[0] * w.species[0].ppc[1] == 65_536_000
    assert w.species[0].x_lo < 0 and w.dt * math.hypot(w.nx / w.lx, w.ny / w.ly) < 1
