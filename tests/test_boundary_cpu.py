"""CPU checks of the C ABI boundary: the built library loads, exports every
function include/pic.h declares, and its host-side validation (configuration,
Courant limit, arena size) answers without touching a GPU."""
import ctypes as C
import math
import os
import re

import pytest

from inputs import clouds1024, lwfa, lwfa8000, thermal64, weibel512

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")
LIB = os.path.join(ROOT, "paper_2106_12485_amd", "libpic.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(pic_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libpic():
    if not os.path.exists(LIB):
        from paper_2106_12485_amd import build
        build.build(force=False)
    from paper_2106_12485_amd import pic
    return pic.lib()


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("pic_init", "pic_step", "pic_deposit", "pic_field_advance", "pic_energy",
              "pic_mem_bytes", "pic_free", "pic_set_particles", "pic_get_particles",
              "pic_set_fields", "pic_get_fields", "pic_get_current", "pic_status"):
        assert n in names


def test_library_exports_every_declared_symbol(libpic):
    for n in declared_functions():
        assert hasattr(libpic, n), n


def test_mem_bytes_of_the_workloads(libpic):
    from paper_2106_12485_amd import mem_bytes
    for w in (thermal64(), lwfa(), clouds1024(), lwfa8000(), weibel512()):
        n = mem_bytes(w)
        # at least the particle state of the initial load
        assert n > w.n_particles_initial() * 24
        assert mem_bytes(w, fp64=True) > n
    # clouds: 2 species x 2 particle buffers x (2 x 8,388,608 + 64 x 4096)
    # slots x 24 B dominate (about 1.64 GB); the outboxes (a quarter of a full
    # tile, 1024 slots per tile, at 25 B) add about 0.42 GB
    n = mem_bytes(clouds1024())
    assert 2.0e9 < n < 2.4e9


def test_validation_rejects_bad_configurations(libpic):
    from paper_2106_12485_amd import pic
    w = thermal64()
    good = pic.make_cfg(w)
    assert libpic.pic_mem_bytes(C.byref(good)) > 0

    def bad(**kw):
        c = pic.make_cfg(w)
        for k, v in kw.items():
            setattr(c, k, v)
        assert libpic.pic_mem_bytes(C.byref(c)) == 0
        return libpic.pic_last_error().decode()

    assert "Courant" in bad(dt=0.1 / math.sqrt(2) * 1.0001)
    assert "nx" in bad(nx=1)
    # cell indices are packed in 16 bits each (unsigned): 65535 is the largest
    # extent, 65518 with the moving window (its storage adds an 18-cell gap)
    assert "65535" in bad(nx=65536, lx=6553.6)
    assert "65535" in bad(ny=65536, ly=6553.6)
    c = pic.make_cfg(w)
    c.nx, c.lx, c.ny, c.ly = 65535, 6553.5, 65535, 6553.5
    assert libpic.pic_mem_bytes(C.byref(c)) > 0
    c = pic.make_cfg(w)
    c.nx, c.lx, c.moving_window = 65518, 6551.8, 1
    assert libpic.pic_mem_bytes(C.byref(c)) > 0
    assert "65518" in bad(nx=65519, lx=6551.9, moving_window=1)
    # a one-cell last tile is accepted (the fold then searches two tiles each
    # way), except by the commutative deposit, whose colours would overlap
    c = pic.make_cfg(w)
    c.nx, c.lx, c.ny, c.ly = 33, 3.3, 49, 4.9
    assert libpic.pic_mem_bytes(C.byref(c)) > 0
    assert "3 cells" in bad(deposit_mode=1, nx=49, lx=4.9)
    assert "n_species" in bad(n_species=5)
    assert "filter" in bad(filter_passes=0, filter_compensate=1)
    assert "filter" in bad(filter_passes=4, filter_compensate=1)
    c = pic.make_cfg(w)
    c.sp[0].ppc_x = 0
    assert libpic.pic_mem_bytes(C.byref(c)) == 0
    # the commutative deposit needs an even number of tiles per axis, periodic
    assert "commutative" in bad(deposit_mode=1, nx=48, lx=4.8)
    assert "commutative" in bad(deposit_mode=1, moving_window=1)
    assert "deposit_mode" in bad(deposit_mode=2)
    c = pic.make_cfg(w, deposit="commutative")
    assert libpic.pic_mem_bytes(C.byref(c)) > 0


def test_init_error_codes_before_any_device_work(libpic):
    from paper_2106_12485_amd import pic
    w = thermal64()
    h = C.c_void_p()
    c = pic.make_cfg(w)
    c.dt = 0.2
    assert libpic.pic_init(C.byref(c), C.c_void_p(256), 1 << 40, None, C.byref(h)) == pic.PIC_E_CFL
    c = pic.make_cfg(w)
    need = libpic.pic_mem_bytes(C.byref(c))
    assert libpic.pic_init(C.byref(c), C.c_void_p(256), need - 1, None,
                           C.byref(h)) == pic.PIC_E_NOMEM
    assert libpic.pic_init(C.byref(c), C.c_void_p(260), need, None,
                           C.byref(h)) == pic.PIC_E_ARG
    assert not h.value
    assert libpic.pic_strerror(pic.PIC_E_CAPACITY) == b"particle capacity exceeded"


def test_binding_fails_loudly_without_a_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2106_12485_amd import Simulation
    with pytest.raises(RuntimeError):
        Simulation(thermal64())


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_traffic_is_null_unless_the_profile_matches_the_sources(tmp_path, monkeypatch):
    # the roofline's measured traffic is reported only while the committed
    # counter summary was taken on the current kernel sources and build flags
    import hashlib
    import bench
    pkg = os.path.join(ROOT, "paper_2106_12485_amd")

    def sha(*p):
        return hashlib.sha256(open(os.path.join(pkg, *p), "rb").read()).hexdigest()

    good = {"kernel_source_sha256": sha("csrc", "pic_kernels.hip"),
            "header_source_sha256": sha("csrc", "pic_dev.h"),
            "build_source_sha256": sha("build.py"),
            "traffic_bytes_per_launch": "123456789"}

    def write(vals):
        f = tmp_path / "traffic.md"
        f.write_text("# summary\n\n" + "".join("    %s %s\n" % kv for kv in vals.items()))
        monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(f))

    write(good)
    assert bench.measured_traffic() == 123456789.0
    for key in ("kernel_source_sha256", "header_source_sha256", "build_source_sha256"):
        write(dict(good, **{key: "0" * 64}))
        assert bench.measured_traffic() is None, key
    write({k: v for k, v in good.items() if k != "traffic_bytes_per_launch"})
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None


def test_product_code_does_not_reach_the_oracle():
    # the oracle is test infrastructure: no module of the package imports it,
    # and bench.py reaches it only from its CPU-baseline leg
    import ast
    pkg = os.path.join(ROOT, "paper_2106_12485_amd")

    def imports(tree):
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                yield from (a.name.split(".")[0] for a in node.names)
            elif isinstance(node, ast.ImportFrom) and node.module:
                yield node.module.split(".")[0]

    for name in os.listdir(pkg):
        if name.endswith(".py"):
            tree = ast.parse(open(os.path.join(pkg, name)).read())
            assert "oracle" not in set(imports(tree)), name
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    users = [f.name for f in tree.body if isinstance(f, ast.FunctionDef)
             and "oracle" in set(imports(f))]
    assert users == ["oracle_for"], users
    # ... and only the CPU-baseline legs call that loader
    callers = sorted(f.name for f in tree.body if isinstance(f, ast.FunctionDef)
                     and any(isinstance(n, ast.Call) and getattr(n.func, "id", "") == "oracle_for"
                             for n in ast.walk(f)))
    assert callers == ["cpu_baseline", "cpu_coverage"], callers
    assert "oracle" not in {m for n in tree.body if not isinstance(n, ast.FunctionDef)
                            for m in imports(n)}


def test_oracle_and_hip_sources_share_no_code():
    # neither side includes a file of the other
    import re
    inc = re.compile(r'#\s*include\s*"([^"]+)"')
    csrc = os.path.join(ROOT, "paper_2106_12485_amd", "csrc")
    for name in os.listdir(csrc):
        for f in inc.findall(open(os.path.join(csrc, name)).read()):
            assert "oracle" not in f, (name, f)
    for f in inc.findall(open(os.path.join(ROOT, "oracle", "pic_oracle.c")).read()):
        assert not f.startswith("pic") or f.startswith("pic_oracle"), f


def test_binding_marshals_every_configuration_field():
    # the binding only copies the workload into the C struct: field by field
    from inputs import lwfa, weibel512
    from paper_2106_12485_amd import pic
    w = lwfa()
    c = pic.make_cfg(w, fp64=True, load=False, capacity_factor=2.5)
    assert (c.nx, c.ny, c.lx, c.ly, c.dt) == (w.nx, w.ny, w.lx, w.ly, w.dt)
    assert (c.moving_window, c.filter_passes, c.filter_compensate) == (1, w.filter_passes, 1)
    assert (c.fp64, c.load, c.capacity_factor, c.deposit_mode) == (1, 0, 2.5, 0)
    assert c.seed == w.seed and c.n_species == len(w.species)
    s, t = w.species[0], c.sp[0]
    assert (t.q_over_m, t.density, t.x_lo, t.ppc_x, t.ppc_y) == (s.qm, s.density, s.x_lo,
                                                                  s.ppc[0], s.ppc[1])
    assert t.x_hi == min(s.x_hi, 1e300)
    assert list(t.uth) == list(s.uth) and list(t.ufl) == list(s.ufl)
    L = w.laser
    assert c.laser.on == 1 and (c.laser.a0, c.laser.omega0, c.laser.W0, c.laser.fwhm,
                                c.laser.x_center, c.laser.focus, c.laser.axis,
                                c.laser.pol_angle) == (L.a0, L.omega0, L.W0, L.fwhm,
                                                       L.x_center, L.focus, L.axis, L.pol)
    # the workload's own capacity factor unless one is given; the other deposit
    w = weibel512()
    assert pic.make_cfg(w).capacity_factor == w.capacity_factor
    assert pic.make_cfg(w, capacity_factor=4.0).capacity_factor == 4.0
    assert pic.make_cfg(w, deposit="commutative").deposit_mode == 1
    assert pic.make_cfg(w).laser.on == 0
