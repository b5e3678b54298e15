"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

Holds no arithmetic of the PIC method: only the parameters of the workloads
(grid, box, timestep, species, laser) and seeded random states (particle sets,
field planes) used to drive both the HIP path and the FP64 oracle with the
same inputs.  Random numbers that the method itself draws while loading
plasma (Maxwellian momenta) are not made here: each side implements the same
published counter-based generator (Philox4x32-10) instead.

The five workloads follow the paper's Sec. 4.1 setups at the sizes of this
build: a small thermal plasma, a laser-wakefield-like run with a moving window,
two counter-streaming electron clouds, a serving stream of independent small
periodic plasmas, and a large laser-wakefield geometry for a precision study.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

SEED_BASE = 0x5EED0000


@dataclass
class SpeciesSpec:
    qm: float = -1.0                   # charge-to-mass ratio (electrons: -1)
    density: float = 1.0               # in units of the reference density
    x_lo: float = -1e300               # lab-frame x range that is loaded
    x_hi: float = 1e300
    ppc: tuple = (4, 4)                # particles per cell along x, y
    uth: tuple = (0.0, 0.0, 0.0)       # thermal proper velocity per component
    ufl: tuple = (0.0, 0.0, 0.0)       # fluid proper velocity


@dataclass
class LaserSpec:
    a0: float
    omega0: float
    W0: float
    fwhm: float
    x_center: float
    focus: float
    axis: float
    pol: float


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    lx: float
    ly: float
    dt: float
    steps: int
    species: List[SpeciesSpec] = field(default_factory=list)
    moving_window: bool = False
    filter_passes: int = 1
    filter_compensate: bool = False
    laser: Optional[LaserSpec] = None
    seed: int = SEED_BASE
    # particle slots per tile as a multiple of the initial load (0: the
    # library's default of 3); physics that piles particles up needs more
    capacity_factor: float = 0.0

    @property
    def dx(self):
        return self.lx / self.nx

    @property
    def dy(self):
        return self.ly / self.ny

    def n_particles_initial(self) -> int:
        """Particle count of the initial load (lattice of sub-cell centres)."""
        tot = 0
        for s in self.species:
            if s.density <= 0:
                continue
            px, py = s.ppc
            xo = (np.arange(px) + 0.5) / px
            xl = (np.arange(self.nx)[:, None] + xo[None, :]) * self.dx
            inside = (xl >= s.x_lo) & (xl < s.x_hi)
            tot += int(inside.sum()) * py * self.ny
        return tot


def thermal64() -> Workload:
    """2D periodic thermal plasma, 64x64 cells, 16 ppc, uth = 0.1."""
    return Workload("thermal_64x64", 64, 64, 6.4, 6.4, 0.07, 100,
                    [SpeciesSpec(-1.0, 1.0, ppc=(4, 4), uth=(0.1, 0.1, 0.1))],
                    seed=SEED_BASE + 0)


def lwfa(nx=2000, ny=256, lx=40.0, ly=51.2, dt=0.014, ppc=(4, 2), steps=500,
         x_plasma=20.0, seed=SEED_BASE + 1, name="lwfa_2000x256") -> Workload:
    """Laser-wakefield-like run: moving window, cold electrons beyond x_plasma,
    Gaussian pulse a0 = 2, w0 = 10, W0 = 4, FWHM 2, s-polarised (pi/2),
    focused at x = 20, compensated binomial filter."""
    return Workload(name, nx, ny, lx, ly, dt, steps,
                    [SpeciesSpec(-1.0, 1.0, x_lo=x_plasma, ppc=ppc)],
                    moving_window=True, filter_passes=1, filter_compensate=True,
                    laser=LaserSpec(2.0, 10.0, 4.0, 2.0, 16.0, 20.0, ly / 2, math.pi / 2),
                    seed=seed)


def clouds1024() -> Workload:
    """Two counter-streaming electron clouds (+-0.6 c along x), each in its own
    half of a periodic 1024^2 box, 16 ppc each, uth = 0.05."""
    L = 102.4
    return Workload("clouds_1024x1024", 1024, 1024, L, L, 0.07, 1000,
                    [SpeciesSpec(-1.0, 1.0, 0.0, L / 2, (4, 4), (0.05,) * 3, (0.6, 0.0, 0.0)),
                     SpeciesSpec(-1.0, 1.0, L / 2, L, (4, 4), (0.05,) * 3, (-0.6, 0.0, 0.0))],
                    seed=SEED_BASE + 2)


def lwfa8000() -> Workload:
    """Config-2 cell size and timestep on an 8000x512 grid, 16 ppc, plasma
    filling the whole box (65,536,000 particles)."""
    return lwfa(nx=8000, ny=512, lx=160.0, ly=102.4, dt=0.014, ppc=(4, 4), steps=200,
                x_plasma=-1e300, seed=SEED_BASE + 4, name="lwfa_8000x512")


def lwfa2000x512() -> Workload:
    """The paper's LWFA size: 2000x512 cells, 16 ppc, 4000 steps, with the
    cell size and step of the 2000x256 run (box 40 x 102.4)."""
    return lwfa(nx=2000, ny=512, lx=40.0, ly=102.4, dt=0.014, ppc=(4, 4), steps=4000,
                seed=SEED_BASE + 6, name="lwfa_2000x512")


def weibel512() -> Workload:
    """Electron and positron clouds streaming along +-z through each other
    (Weibel instability): 512^2 periodic cells of 0.1, 16 x 16 particles per
    cell per species (134,217,728 particles), u_fl,z = +-0.6, u_th = 0.1."""
    L = 51.2
    # The filaments pinch: over the 500 steps the fullest tile reaches 3.8x
    # its initial load while others empty; the particle segments follow the
    # counts, so the default pool of twice the load suffices.
    return Workload("weibel_512x512", 512, 512, L, L, 0.07, 500,
                    [SpeciesSpec(-1.0, 1.0, ppc=(16, 16), uth=(0.1,) * 3, ufl=(0.0, 0.0, 0.6)),
                     SpeciesSpec(1.0, 1.0, ppc=(16, 16), uth=(0.1,) * 3, ufl=(0.0, 0.0, -0.6))],
                    seed=SEED_BASE + 5)


WORKLOADS = {
    "thermal_64x64": thermal64,
    "lwfa_2000x256": lwfa,
    "clouds_1024x1024": clouds1024,
    "lwfa_8000x512": lwfa8000,
    "weibel_512x512": weibel512,
    "lwfa_2000x512": lwfa2000x512,
}


def serving_requests(n_requests=64, seed=SEED_BASE + 3, grids=(64, 128, 256, 512),
                     ppcs=((2, 2), (4, 4), (8, 8)), steps=200, rate=None):
    """Stream of independent periodic plasmas for the serving loop.

    Each request: grid n^2 with n uniform over `grids`, cell size 0.1,
    dt = 0.07, ppc uniform over `ppcs`; kind thermal or two-stream with
    probability 1/2; uth ~ U[0.01, 0.2]; two-stream drift U ~ U[0, 0.5].
    Arrival times are a Poisson process of the given rate (requests per
    second; None = all at t = 0)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        n = int(rng.choice(grids))
        ppc = tuple(int(v) for v in ppcs[int(rng.integers(len(ppcs)))])
        uth = float(rng.uniform(0.01, 0.2))
        two = bool(rng.random() < 0.5)
        U = float(rng.uniform(0.0, 0.5))
        if two:
            sp = [SpeciesSpec(-1.0, 0.5, ppc=ppc, uth=(uth,) * 3, ufl=(U, 0.0, 0.0)),
                  SpeciesSpec(-1.0, 0.5, ppc=ppc, uth=(uth,) * 3, ufl=(-U, 0.0, 0.0))]
        else:
            sp = [SpeciesSpec(-1.0, 1.0, ppc=ppc, uth=(uth,) * 3)]
        w = Workload("req%03d_%dx%d" % (r, n, n), n, n, 0.1 * n, 0.1 * n, 0.07, steps, sp,
                     seed=seed + 1000 + r)
        if rate:
            t += float(rng.exponential(1.0 / rate))
        out.append((t, w))
    return out


# ---------------------------------------------------------------------------
# seeded random states for unit and parity tests
# ---------------------------------------------------------------------------
def random_particles(rng, nx, ny, n, uth=0.1, ufl=(0.0, 0.0, 0.0), x_range=None):
    """n particles at uniformly random positions, Gaussian momenta."""
    if x_range is None:
        ix = rng.integers(0, nx, n)
    else:
        ix = rng.integers(x_range[0], x_range[1], n)
    iy = rng.integers(0, ny, n)
    p = dict(ix=ix.astype(np.int32), iy=iy.astype(np.int32),
             x=rng.random(n), y=rng.random(n),
             ux=ufl[0] + uth * rng.standard_normal(n),
             uy=ufl[1] + uth * rng.standard_normal(n),
             uz=ufl[2] + uth * rng.standard_normal(n))
    return p


def random_fields(rng, nx, ny, amp=0.05):
    """Six smooth-ish random field planes (Ex Ey Ez Bx By Bz), shape (6, ny, nx)."""
    f = amp * rng.standard_normal((6, ny, nx))
    return f


def with_species(w: Workload, **kw) -> Workload:
    return replace(w, **kw)
