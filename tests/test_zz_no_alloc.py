"""pic_batch_step_static (the batched step that allocates nothing) against
pic_batch_step on the same simulations: the same kernels over the same work
lists, so fields, current and particles must be bitwise equal.  Two calls in
a row, the second on a smaller set, so the shared device array is re-staged
with fewer simulations and tiles than the call before left in it."""
import numpy as np
import pytest

from inputs import SpeciesSpec, Workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2106_12485_amd import (PIC_E_ARG, Batch, PicError, Simulation,  # noqa: E402
                                  batch_step_static)

KEYS = ("uz", "uy", "ux", "y", "x", "iy", "ix")


def same_particles(a, b):
    oa = np.lexsort([a[c] for c in KEYS])
    ob = np.lexsort([b[c] for c in KEYS])
    return all(np.array_equal(a[c][oa], b[c][ob]) for c in KEYS)


def workloads():
    sp = [SpeciesSpec(-1.0, 0.5, ppc=(4, 4), uth=(0.05,) * 3, ufl=(0.3, 0, 0)),
          SpeciesSpec(-1.0, 0.5, ppc=(4, 4), uth=(0.05,) * 3, ufl=(-0.3, 0, 0))]
    return [
        Workload("thermal_64x48", 64, 48, 6.4, 4.8, 0.07, 20,
                 [SpeciesSpec(-1.0, 1.0, ppc=(2, 2), uth=(0.15,) * 3)], filter_passes=1,
                 seed=21),
        Workload("twostream_96x64", 96, 64, 9.6, 6.4, 0.07, 20, sp, filter_passes=1, seed=22),
        Workload("thermal_40x36", 40, 36, 4.0, 3.6, 0.07, 20,
                 [SpeciesSpec(-1.0, 1.0, ppc=(3, 3), uth=(0.2,) * 3)], filter_passes=1,
                 seed=23),
    ]


def assert_same(a, b):
    assert np.array_equal(a.get_fields(), b.get_fields())
    assert np.array_equal(a.get_current(False), b.get_current(False))
    for k in range(a.n_species):
        assert same_particles(a.get_particles(k), b.get_particles(k))


def test_static_batch_equals_batch_object_twice_second_smaller():
    ws = workloads()
    ref = [Simulation(w) for w in ws]
    got = [Simulation(w) for w in ws]
    ntiles = sum(s.layout()["ntx"] * s.layout()["nty"] for s in ref)
    b = Batch(4, ntiles)
    # call 1: all three simulations
    print("no-alloc call 1: 3 simulations, %d tiles" % ntiles, flush=True)
    b.step(ref, 12)
    batch_step_static(got, 12)
    torch.cuda.synchronize()
    for r, g in zip(ref, got):
        assert_same(r, g)
        assert g.status() == 0
    # call 2: a smaller set (the last simulation only, fewer tiles)
    print("no-alloc call 2: 1 simulation", flush=True)
    b.step(ref[2:], 9)
    batch_step_static(got[2:], 9)
    torch.cuda.synchronize()
    for r, g in zip(ref, got):
        assert_same(r, g)
    e_r, e_g = ref[2].energy(), got[2].energy()
    assert e_r["step"] == e_g["step"] == 21
    assert e_r["total"] == e_g["total"]
    for s in ref + got:
        s.close()
    b.close()


def test_static_batch_refuses_sets_beyond_its_maximum():
    from paper_2106_12485_amd.pic import lib  # noqa: F401
    w = Workload("big_2048x2048", 2048, 2048, 204.8, 204.8, 0.07, 1,
                 [SpeciesSpec(-1.0, 0.0, ppc=(1, 1), uth=(0.0,) * 3)], seed=24)
    s = Simulation(w, load=False)  # 16384 tiles ...
    s2 = Simulation(workloads()[2], load=False)  # ... plus 9 exceed the maximum
    with pytest.raises(PicError) as e:
        batch_step_static([s, s2], 1)
    assert e.value.code == PIC_E_ARG
    s.close()
    s2.close()
