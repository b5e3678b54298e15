"""ctypes binding of libpic (include/pic.h): argument marshalling only.

Every step of the PIC cycle runs in the HIP kernels of libpic.so; PyTorch only
provides the device arena (a uint8 tensor) and the stream.  There is no CPU
fallback: if the library is missing or no GPU is present, construction fails.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")
MAX_SPECIES = 4
NK = 7
KERNEL_NAMES = ("push_deposit", "settle", "fold", "filter", "yee", "window", "order")

PIC_OK, PIC_E_ARG, PIC_E_CFL, PIC_E_NOMEM, PIC_E_CAPACITY, PIC_E_HIP, PIC_E_STATE = \
    0, -1, -2, -3, -4, -5, -6
PIC_E_CANCELLED = -7


class SpeciesCfg(C.Structure):
    _fields_ = [("q_over_m", C.c_double), ("density", C.c_double), ("x_lo", C.c_double),
                ("x_hi", C.c_double), ("ppc_x", C.c_int), ("ppc_y", C.c_int),
                ("uth", C.c_double * 3), ("ufl", C.c_double * 3)]


class LaserCfg(C.Structure):
    _fields_ = [("on", C.c_int), ("a0", C.c_double), ("omega0", C.c_double), ("W0", C.c_double),
                ("fwhm", C.c_double), ("x_center", C.c_double), ("focus", C.c_double),
                ("axis", C.c_double), ("pol_angle", C.c_double)]


class Cfg(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("lx", C.c_double), ("ly", C.c_double),
                ("dt", C.c_double), ("moving_window", C.c_int), ("filter_passes", C.c_int),
                ("filter_compensate", C.c_int), ("n_species", C.c_int),
                ("sp", SpeciesCfg * MAX_SPECIES), ("laser", LaserCfg), ("fp64", C.c_int),
                ("seed", C.c_ulonglong), ("load", C.c_int), ("capacity_factor", C.c_double),
                ("deposit_mode", C.c_int)]


class Diag(C.Structure):
    _fields_ = [("e_energy", C.c_double), ("b_energy", C.c_double),
                ("ke", C.c_double * MAX_SPECIES), ("total", C.c_double), ("charge", C.c_double),
                ("gauss_res_max", C.c_double), ("cont_res_max", C.c_double),
                ("rho_max", C.c_double), ("t", C.c_double),
                ("n_particles", C.c_longlong * MAX_SPECIES), ("step", C.c_longlong),
                ("nshift", C.c_int), ("status", C.c_int)]


class Request(C.Structure):
    _fields_ = [("cfg", Cfg), ("nsteps", C.c_int), ("arrival_s", C.c_double),
                ("cancel_s", C.c_double)]


class Result(C.Structure):
    _fields_ = [("admit_s", C.c_double), ("done_s", C.c_double), ("diag", Diag),
                ("status", C.c_int)]


class ServeOpts(C.Structure):
    _fields_ = [("batched", C.c_int), ("chunk_steps", C.c_int), ("max_batch", C.c_int),
                ("rate_ratio", C.c_int), ("cancel", C.POINTER(C.c_int)),
                ("max_particles", C.c_longlong), ("lone_particles", C.c_longlong)]


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libpic error %d: %s" % (code, msg))
        self.code = code


_lib = None

_P = C.c_void_p
_I = C.c_int
_LL = C.c_longlong
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int)
_LLP = C.POINTER(C.c_longlong)


def lib():
    """Load libpic.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpic.so is not built (%s); run __graft_entry__.build()"
                               % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        L.pic_mem_bytes.restype = C.c_size_t
        L.pic_mem_bytes.argtypes = [C.POINTER(Cfg)]
        L.pic_init.restype = _I
        L.pic_init.argtypes = [C.POINTER(Cfg), _P, C.c_size_t, _P, C.POINTER(_P)]
        for name in ("pic_deposit", "pic_field_advance", "pic_status"):
            getattr(L, name).restype = _I
            getattr(L, name).argtypes = [_P, _P]
        L.pic_step.restype = _I
        L.pic_step.argtypes = [_P, _I, _P]
        L.pic_energy.restype = _I
        L.pic_energy.argtypes = [_P, C.POINTER(Diag), _P]
        L.pic_free.restype = _I
        L.pic_free.argtypes = [_P]
        L.pic_set_particles.restype = _I
        L.pic_set_particles.argtypes = [_P, _I, _LL, _IP, _IP, _DP, _DP, _DP, _DP, _DP, _P]
        L.pic_particle_count.restype = _LL
        L.pic_particle_count.argtypes = [_P, _I, _P]
        L.pic_get_particles.restype = _I
        L.pic_get_particles.argtypes = [_P, _I, _LL, _LLP, _IP, _IP, _DP, _DP, _DP, _DP, _DP, _P]
        L.pic_set_fields.restype = _I
        L.pic_set_fields.argtypes = [_P, _DP, _P]
        L.pic_get_fields.restype = _I
        L.pic_get_fields.argtypes = [_P, _DP, _P]
        L.pic_get_current.restype = _I
        L.pic_get_current.argtypes = [_P, _I, _DP, _P]
        L.pic_set_time.restype = _I
        L.pic_set_time.argtypes = [_P, _LL, _I, _P]
        L.pic_timing.restype = _I
        L.pic_timing.argtypes = [_P, _I, _P]
        L.pic_timing_read.restype = _I
        L.pic_timing_read.argtypes = [_P, _DP, _LLP, _I, _P]
        L.pic_layout.restype = _I
        L.pic_layout.argtypes = [_P, _LLP, _I]
        L.pic_batch_mem_bytes.restype = C.c_size_t
        L.pic_batch_mem_bytes.argtypes = [_I, _LL]
        L.pic_batch_create.restype = _I
        L.pic_batch_create.argtypes = [_P, C.c_size_t, _I, _LL, C.POINTER(_P)]
        L.pic_batch_step.restype = _I
        L.pic_batch_step.argtypes = [_P, C.POINTER(_P), _I, _I, _P]
        L.pic_batch_free.restype = _I
        L.pic_batch_free.argtypes = [_P]
        L.pic_batch_step_static.restype = _I
        L.pic_batch_step_static.argtypes = [C.POINTER(_P), _I, _I, _P]
        L.pic_serve.restype = _I
        L.pic_serve.argtypes = [C.POINTER(Request), _I, _P, C.c_size_t, C.POINTER(ServeOpts),
                                C.POINTER(Result), _DP, _LL, _LLP, _P]
        L.pic_strerror.restype = C.c_char_p
        L.pic_strerror.argtypes = [_I]
        L.pic_last_error.restype = C.c_char_p
        L.pic_last_error.argtypes = []
        _lib = L
    return _lib


def _check(rc):
    if rc != PIC_OK:
        L = lib()
        raise PicError(rc, "%s (%s)" % (L.pic_strerror(rc).decode(), L.pic_last_error().decode()))
    return rc


DEPOSIT_MODES = {"reduction": 0, "commutative": 1}


def make_cfg(w, fp64=False, load=True, capacity_factor=0.0, deposit="reduction") -> Cfg:
    """Fill the C configuration from a workload description (any object with
    nx, ny, lx, ly, dt, species, moving_window, filter_passes,
    filter_compensate, laser, seed and optionally capacity_factor
    attributes)."""
    c = Cfg()
    c.nx, c.ny = int(w.nx), int(w.ny)
    c.lx, c.ly, c.dt = float(w.lx), float(w.ly), float(w.dt)
    c.moving_window = int(bool(getattr(w, "moving_window", False)))
    c.filter_passes = int(getattr(w, "filter_passes", 1))
    c.filter_compensate = int(bool(getattr(w, "filter_compensate", False)))
    sp = list(w.species)
    if len(sp) > MAX_SPECIES:
        raise ValueError("at most %d species" % MAX_SPECIES)
    c.n_species = len(sp)
    for k, s in enumerate(sp):
        t = c.sp[k]
        t.q_over_m = float(s.qm)
        t.density = float(s.density)
        t.x_lo = float(max(s.x_lo, -1e300))
        t.x_hi = float(min(s.x_hi, 1e300))
        t.ppc_x, t.ppc_y = int(s.ppc[0]), int(s.ppc[1])
        for i in range(3):
            t.uth[i] = float(s.uth[i])
            t.ufl[i] = float(s.ufl[i])
    las = getattr(w, "laser", None)
    if las is not None:
        c.laser.on = 1
        for f in ("a0", "omega0", "W0", "fwhm", "x_center", "focus", "axis"):
            setattr(c.laser, f, float(getattr(las, f)))
        c.laser.pol_angle = float(las.pol)
    c.fp64 = int(bool(fp64))
    c.seed = int(getattr(w, "seed", 0)) & 0xFFFFFFFFFFFFFFFF
    c.load = int(bool(load))
    # an explicit factor wins over the workload's own
    c.capacity_factor = float(capacity_factor or getattr(w, "capacity_factor", 0.0))
    c.deposit_mode = DEPOSIT_MODES[deposit]
    return c


def mem_bytes(w, fp64=False, capacity_factor=0.0, deposit="reduction") -> int:
    cfg = make_cfg(w, fp64=fp64, capacity_factor=capacity_factor, deposit=deposit)
    n = lib().pic_mem_bytes(C.byref(cfg))
    if n == 0:
        raise PicError(PIC_E_ARG, lib().pic_last_error().decode())
    return int(n)


def _dp(a):
    return a.ctypes.data_as(_DP)


def _ip(a):
    return a.ctypes.data_as(_IP)


class Simulation:
    """One simulation resident in a device arena owned by this object."""

    def __init__(self, w, fp64=False, load=True, capacity_factor=0.0, device="cuda",
                 stream=None, arena=None, deposit="reduction"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libpic needs a GPU; none is visible")
        L = lib()
        self.cfg = make_cfg(w, fp64=fp64, load=load, capacity_factor=capacity_factor,
                            deposit=deposit)
        self.nx, self.ny = self.cfg.nx, self.cfg.ny
        self.n_species = self.cfg.n_species
        nbytes = L.pic_mem_bytes(C.byref(self.cfg))
        if nbytes == 0:
            raise PicError(PIC_E_ARG, L.pic_last_error().decode())
        self.nbytes = int(nbytes)
        if arena is None:
            arena = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.arena = arena
        self.stream = stream if stream is not None else torch.cuda.current_stream(arena.device)
        self._h = _P()
        _check(L.pic_init(C.byref(self.cfg), _P(arena.data_ptr()), arena.numel(), self._sp(),
                          C.byref(self._h)))

    def _sp(self):
        return _P(self.stream.cuda_stream)

    def close(self):
        if getattr(self, "_h", None):
            lib().pic_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the cycle -------------------------------------------------------
    def deposit(self):
        _check(lib().pic_deposit(self._h, self._sp()))

    def field_advance(self):
        _check(lib().pic_field_advance(self._h, self._sp()))

    def step(self, n=1):
        _check(lib().pic_step(self._h, int(n), self._sp()))

    def status(self):
        return lib().pic_status(self._h, self._sp())

    def energy(self):
        d = Diag()
        _check(lib().pic_energy(self._h, C.byref(d), self._sp()))
        ns = self.n_species
        return dict(e_energy=d.e_energy, b_energy=d.b_energy, ke=np.array(d.ke[:ns]),
                    total=d.total, charge=d.charge, gauss_res_max=d.gauss_res_max,
                    cont_res_max=d.cont_res_max, rho_max=d.rho_max, t=d.t,
                    n_particles=np.array(d.n_particles[:ns]), step=d.step, nshift=d.nshift,
                    status=d.status)

    # -- state in / out ---------------------------------------------------
    def set_particles(self, k, p):
        ix = np.ascontiguousarray(p["ix"], dtype=np.int32)
        iy = np.ascontiguousarray(p["iy"], dtype=np.int32)
        f = [np.ascontiguousarray(p[n], dtype=np.float64) for n in ("x", "y", "ux", "uy", "uz")]
        _check(lib().pic_set_particles(self._h, int(k), len(ix), _ip(ix), _ip(iy),
                                       *[_dp(a) for a in f], self._sp()))

    def count(self, k):
        n = lib().pic_particle_count(self._h, int(k), self._sp())
        if n < 0:
            _check(int(n))
        return int(n)

    def get_particles(self, k):
        n = self.count(k)
        ix = np.zeros(n, np.int32)
        iy = np.zeros(n, np.int32)
        f = [np.zeros(n) for _ in range(5)]
        got = C.c_longlong(0)
        _check(lib().pic_get_particles(self._h, int(k), n, C.byref(got), _ip(ix), _ip(iy),
                                       *[_dp(a) for a in f], self._sp()))
        return dict(ix=ix, iy=iy, x=f[0], y=f[1], ux=f[2], uy=f[3], uz=f[4])

    def set_fields(self, f6):
        a = np.ascontiguousarray(np.asarray(f6, dtype=np.float64).reshape(6, self.ny, self.nx))
        _check(lib().pic_set_fields(self._h, _dp(a), self._sp()))

    def get_fields(self):
        a = np.zeros((6, self.ny, self.nx))
        _check(lib().pic_get_fields(self._h, _dp(a), self._sp()))
        return a

    def get_current(self, filtered=True):
        a = np.zeros((3, self.ny, self.nx))
        _check(lib().pic_get_current(self._h, int(filtered), _dp(a), self._sp()))
        return a

    def set_time(self, it, nshift=0):
        _check(lib().pic_set_time(self._h, int(it), int(nshift), self._sp()))

    # -- measurement --------------------------------------------------------
    def timing(self, enable=True):
        _check(lib().pic_timing(self._h, int(enable), self._sp()))

    def timing_read(self):
        ms = np.zeros(NK)
        n = np.zeros(NK, dtype=np.int64)
        _check(lib().pic_timing_read(self._h, _dp(ms), n.ctypes.data_as(_LLP), NK, self._sp()))
        return {KERNEL_NAMES[k]: (float(ms[k]), int(n[k])) for k in range(NK)}

    def layout(self):
        a = np.zeros(7, dtype=np.int64)
        _check(lib().pic_layout(self._h, a.ctypes.data_as(_LLP), 7))
        keys = ("tile_x", "tile_y", "ntx", "nty", "nx_storage", "pool", "cap_out")
        return dict(zip(keys, (int(v) for v in a)))


def cfl_limit(dx, dy):
    return 1.0 / math.sqrt(1.0 / dx ** 2 + 1.0 / dy ** 2)


def _diag_dict(d, ns):
    return dict(e_energy=d.e_energy, b_energy=d.b_energy, ke=np.array(d.ke[:ns]),
                total=d.total, charge=d.charge, gauss_res_max=d.gauss_res_max,
                cont_res_max=d.cont_res_max, rho_max=d.rho_max, t=d.t,
                n_particles=np.array(d.n_particles[:ns]), step=d.step, nshift=d.nshift,
                status=d.status)


class Batch:
    """Device workspace that steps several Simulations with shared launches."""

    def __init__(self, max_sims, max_tiles, device="cuda"):
        import torch
        L = lib()
        n = L.pic_batch_mem_bytes(int(max_sims), int(max_tiles))
        if n == 0:
            raise PicError(PIC_E_ARG, "bad batch sizes")
        self.arena = torch.empty(int(n), dtype=torch.uint8, device=device)
        self._h = _P()
        _check(L.pic_batch_create(_P(self.arena.data_ptr()), int(n), int(max_sims),
                                  int(max_tiles), C.byref(self._h)))

    def step(self, sims, nsteps=1, stream=None):
        import torch
        arr = (_P * len(sims))(*[s._h for s in sims])
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().pic_batch_step(self._h, arr, len(sims), int(nsteps), _P(st.cuda_stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().pic_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_step_static(sims, nsteps=1, stream=None):
    """pic_batch_step_static: step `sims` together with no batch object (the
    library's own device array holds the descriptors; nothing is allocated)."""
    import torch
    arr = (_P * len(sims))(*[s._h for s in sims])
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().pic_batch_step_static(arr, len(sims), int(nsteps), _P(st.cuda_stream)))


def serve(requests, budget_bytes, batched=True, chunk_steps=10, max_batch=0, device="cuda",
          max_step_records=1 << 16, rate_ratio=1, cancel_flags=None, max_particles=0,
          lone_particles=0):
    """Serve `requests` = [(arrival_s, workload, nsteps[, cancel_s]), ...]
    through the native continuous-batching loop within an HBM budget of
    budget_bytes.  cancel_flags: None, or an int32 numpy array of one flag per
    request that another thread may set while this call runs (nonzero cancels
    the request).  max_particles (batched): a request joins a running set only
    while the set's initial particle loads stay within it (0: no limit);
    lone_particles: that limit for a request with no other queued request
    behind it (0: max_particles).
    Returns per-request times / diagnostics and the per-step batch times."""
    import torch
    n = len(requests)
    reqs = (Request * n)()
    for i, rq in enumerate(requests):
        arr, w, nsteps = rq[:3]
        reqs[i].cfg = make_cfg(w)
        reqs[i].nsteps = int(nsteps)
        reqs[i].arrival_s = float(arr)
        reqs[i].cancel_s = float(rq[3]) if len(rq) > 3 and rq[3] is not None else 0.0
    out = (Result * n)()
    flags = None
    if cancel_flags is not None:
        assert cancel_flags.dtype == np.int32 and cancel_flags.size >= n
        assert cancel_flags.flags["C_CONTIGUOUS"]
        flags = cancel_flags.ctypes.data_as(C.POINTER(C.c_int))
    opts = ServeOpts(int(bool(batched)), int(chunk_steps), int(max_batch), int(rate_ratio), flags,
                     int(max_particles), int(lone_particles))
    arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device=device)
    step_ms = np.zeros(max_step_records)
    nsteps_out = C.c_longlong(0)
    st = torch.cuda.current_stream()
    _check(lib().pic_serve(reqs, n, _P(arena.data_ptr()), arena.numel(), C.byref(opts), out,
                           _dp(step_ms), len(step_ms), C.byref(nsteps_out), _P(st.cuda_stream)))
    res = []
    for i, rq in enumerate(requests):
        arr, w = rq[0], rq[1]
        r = out[i]
        res.append(dict(arrival_s=float(arr), admit_s=r.admit_s, done_s=r.done_s,
                        latency_s=r.done_s - float(arr), status=r.status,
                        diag=_diag_dict(r.diag, len(w.species))))
    k = min(int(nsteps_out.value), len(step_ms))
    return dict(results=res, step_ms=step_ms[:k].copy())
