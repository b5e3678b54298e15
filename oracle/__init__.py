"""FP64 CPU oracle of the 2D EM-PIC timestep -- TEST INFRASTRUCTURE ONLY.

This package wraps ``pic_oracle.c`` (plain C, FP64, global arrays, particles in
array order) with ctypes.  It exists to check the HIP path: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product library never loads it and shares no code with it.

The method it follows is the four-stage PIC cycle of the paper's Sec. 2.2
(Fig. 1): bilinear field interpolation, leapfrog/Boris push, exact
charge-conserving (Villasenor-Buneman) current deposition with an optional
binomial filter, and Yee FDTD field advance; plus the Sec. 4.1 LWFA extras
(laser-initialised fields, compensated filter, moving window, immobile ions).
The readings taken where the paper is silent are listed at the top of
``pic_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAX_SPECIES = 8


def build(force: bool = False) -> str:
    """Compile pic_oracle.c into liboracle.so with gcc (host code only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
             "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _declare(_lib)
    return _lib


_P = C.c_void_p
_D = C.c_double
_I = C.c_int
_LL = C.c_longlong
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int)
_UP = C.POINTER(C.c_uint32)


def _declare(L):
    L.orc_create.restype = _P
    L.orc_create.argtypes = [_I, _I, _D, _D, _D, _I, _I, _I, C.c_ulonglong]
    L.orc_destroy.argtypes = [_P]
    L.orc_add_species.restype = _I
    L.orc_add_species.argtypes = [_P, _D, _D, _D, _D, _I, _I, _DP, _DP, _I]
    L.orc_count.restype = _LL
    L.orc_count.argtypes = [_P, _I]
    L.orc_qp.restype = _D
    L.orc_qp.argtypes = [_P, _I]
    L.orc_iter.restype = _LL
    L.orc_iter.argtypes = [_P]
    L.orc_nshift.restype = _I
    L.orc_nshift.argtypes = [_P]
    L.orc_set_iter.argtypes = [_P, _LL, _I]
    L.orc_set_particles.restype = _I
    L.orc_set_particles.argtypes = [_P, _I, _LL, _IP, _IP, _DP, _DP, _DP, _DP, _DP]
    L.orc_get_particles.restype = _I
    L.orc_get_particles.argtypes = [_P, _I, _IP, _IP, _DP, _DP, _DP, _DP, _DP]
    L.orc_set_fields.argtypes = [_P, _DP]
    L.orc_get_fields.argtypes = [_P, _DP]
    L.orc_get_current.argtypes = [_P, _I, _DP]
    L.orc_set_current.argtypes = [_P, _DP]
    L.orc_add_laser.argtypes = [_P, _D, _D, _D, _D, _D, _D, _D, _D]
    L.orc_gather.argtypes = [_P, _I, _I, _D, _D, _DP]
    L.orc_boris.argtypes = [_D, _D, _DP, _DP, _DP]
    for name in ("orc_push_deposit", "orc_filter", "orc_yee", "orc_field_advance"):
        getattr(L, name).argtypes = [_P]
    L.orc_step.argtypes = [_P, _I]
    L.orc_set_threads.argtypes = [_P, _I]
    L.orc_charge.argtypes = [_P, _DP]
    L.orc_divergence.argtypes = [_P, _DP, _DP, _DP]
    L.orc_filter_plane.argtypes = [_P, _DP]
    L.orc_energy.argtypes = [_P, _DP]
    L.orc_philox4x32_10.argtypes = [_UP, _UP, _UP]
    L.orc_normals4.argtypes = [_UP, _DP]


def _dp(a):
    return a.ctypes.data_as(_DP)


def _ip(a):
    return a.ctypes.data_as(_IP)


def philox4x32_10(ctr, key):
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data_as(_UP), k.ctypes.data_as(_UP), o.ctypes.data_as(_UP))
    return o


def normals4(words):
    w = np.ascontiguousarray(words, dtype=np.uint32)
    o = np.zeros(4)
    lib().orc_normals4(w.ctypes.data_as(_UP), _dp(o))
    return o


def boris(qm, dt, e, b, u):
    """One relativistic Boris update of the momentum u (returns a new array)."""
    e = np.ascontiguousarray(e, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    uu = np.array(u, dtype=np.float64)
    lib().orc_boris(qm, dt, _dp(e), _dp(b), _dp(uu))
    return uu


class Species:
    def __init__(self, qm, density=1.0, x_lo=-1e300, x_hi=1e300, ppc=(1, 1),
                 uth=(0.0, 0.0, 0.0), ufl=(0.0, 0.0, 0.0)):
        self.qm = qm
        self.density = density
        self.x_lo = x_lo
        self.x_hi = x_hi
        self.ppc = tuple(ppc)
        self.uth = tuple(uth)
        self.ufl = tuple(ufl)


class OracleSim:
    """One simulation held by the FP64 oracle.

    Field planes are (ny, nx) numpy arrays (x fastest in memory); particle
    sets are dicts of arrays ix, iy (int32), x, y, ux, uy, uz (float64).
    """

    def __init__(self, nx, ny, lx, ly, dt, window=False, filter_passes=1,
                 filter_compensate=False, seed=0):
        self._L = lib()
        self.nx, self.ny = int(nx), int(ny)
        self.dx, self.dy, self.dt = lx / nx, ly / ny, dt
        self.window = bool(window)
        self._h = self._L.orc_create(self.nx, self.ny, float(lx), float(ly), float(dt),
                                     int(window), int(filter_passes),
                                     int(filter_compensate), int(seed))
        if not self._h:
            raise ValueError("bad grid")
        self.nsp = 0

    def set_threads(self, n: int):
        """n > 1: run the particle loop as the paper's parallel for (private
        current copies summed in thread order) and the grid loops over rows."""
        self._L.orc_set_threads(self._h, int(n))

    def close(self):
        if self._h:
            self._L.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up -----------------------------------------------------
    def add_species(self, sp: Species, load=True) -> int:
        uth = np.array(sp.uth, dtype=np.float64)
        ufl = np.array(sp.ufl, dtype=np.float64)
        k = self._L.orc_add_species(self._h, sp.qm, sp.density, sp.x_lo, sp.x_hi,
                                    sp.ppc[0], sp.ppc[1], _dp(uth), _dp(ufl), int(load))
        if k < 0:
            raise ValueError("too many species")
        self.nsp += 1
        return k

    def add_laser(self, a0, omega0, W0, fwhm, x_center, focus, axis, pol):
        self._L.orc_add_laser(self._h, a0, omega0, W0, fwhm, x_center, focus, axis, pol)

    def count(self, k):
        return int(self._L.orc_count(self._h, k))

    def qp(self, k):
        return float(self._L.orc_qp(self._h, k))

    @property
    def iter(self):
        return int(self._L.orc_iter(self._h))

    @property
    def nshift(self):
        return int(self._L.orc_nshift(self._h))

    def set_iter(self, it, nshift=0):
        self._L.orc_set_iter(self._h, int(it), int(nshift))

    def set_particles(self, k, p):
        ix = np.ascontiguousarray(p["ix"], dtype=np.int32)
        iy = np.ascontiguousarray(p["iy"], dtype=np.int32)
        arrs = [np.ascontiguousarray(p[n], dtype=np.float64) for n in ("x", "y", "ux", "uy", "uz")]
        n = len(ix)
        if self._L.orc_set_particles(self._h, k, n, _ip(ix), _ip(iy), *[_dp(a) for a in arrs]):
            raise ValueError("bad species")

    def get_particles(self, k):
        n = self.count(k)
        ix = np.zeros(n, np.int32)
        iy = np.zeros(n, np.int32)
        f = [np.zeros(n) for _ in range(5)]
        self._L.orc_get_particles(self._h, k, _ip(ix), _ip(iy), *[_dp(a) for a in f])
        return dict(ix=ix, iy=iy, x=f[0], y=f[1], ux=f[2], uy=f[3], uz=f[4])

    def set_fields(self, f6):
        a = np.ascontiguousarray(np.asarray(f6, dtype=np.float64).reshape(6, self.ny, self.nx))
        self._L.orc_set_fields(self._h, _dp(a))

    def get_fields(self):
        a = np.zeros((6, self.ny, self.nx))
        self._L.orc_get_fields(self._h, _dp(a))
        return a

    def set_current(self, j3):
        a = np.ascontiguousarray(np.asarray(j3, dtype=np.float64).reshape(3, self.ny, self.nx))
        self._L.orc_set_current(self._h, _dp(a))

    def get_current(self, filtered=True):
        a = np.zeros((3, self.ny, self.nx))
        self._L.orc_get_current(self._h, int(filtered), _dp(a))
        return a

    # -- the cycle ----------------------------------------------------
    def gather(self, ix, iy, x, y):
        o = np.zeros(6)
        self._L.orc_gather(self._h, int(ix), int(iy), float(x), float(y), _dp(o))
        return o

    def push_deposit(self):
        self._L.orc_push_deposit(self._h)

    def filter(self):
        self._L.orc_filter(self._h)

    def yee(self):
        self._L.orc_yee(self._h)

    def field_advance(self):
        self._L.orc_field_advance(self._h)

    def step(self, n=1):
        self._L.orc_step(self._h, int(n))

    # -- diagnostics --------------------------------------------------
    def charge(self):
        a = np.zeros((self.ny, self.nx))
        self._L.orc_charge(self._h, _dp(a))
        return a

    def divergence(self, fx, fy):
        fx = np.ascontiguousarray(fx, dtype=np.float64)
        fy = np.ascontiguousarray(fy, dtype=np.float64)
        d = np.zeros((self.ny, self.nx))
        self._L.orc_divergence(self._h, _dp(fx), _dp(fy), _dp(d))
        return d

    def filter_plane(self, plane):
        a = np.array(plane, dtype=np.float64, order="C").reshape(self.ny, self.nx)
        self._L.orc_filter_plane(self._h, _dp(a))
        return a

    def energy(self):
        o = np.zeros(3 + MAX_SPECIES)
        self._L.orc_energy(self._h, _dp(o))
        return dict(e_energy=o[0], b_energy=o[1], ke=o[2:2 + self.nsp].copy(),
                    charge=o[2 + MAX_SPECIES],
                    total=o[0] + o[1] + o[2:2 + self.nsp].sum())
