"""Host-side checks of the C ABI (no GPU needed, no compute calls)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT


def _declared():
    text = open(os.path.join(ROOT, "include", "pgg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pgg_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def pgg():
    from paper_1704_08098_amd import pgg as mod
    if not os.path.exists(mod.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    mod.load()
    return mod


def test_every_declared_symbol_is_exported(pgg):
    lib = ctypes.CDLL(pgg.LIB_PATH)
    names = _declared()
    assert "pgg_init" in names and "pgg_sweep" in names and "pgg_density" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(pgg.EXPORTS) == names


def test_params_struct_layout(pgg):
    # uint32 L; double r, K, p0; uint64 seed; uint32 layout, kernel, tile, group
    assert ctypes.sizeof(pgg.PggParams) == 64
    assert pgg.PggParams.seed.offset == 32
    assert pgg.PggParams.group.offset == 52
    assert pgg.PggParams.schedule.offset == 56
    assert pgg.PggParams.game.offset == 60


def test_device_bytes(pgg):
    assert pgg.pgg_device_bytes(pgg.make_params(100, 3.8, layout="int8")) == 100 * 100
    # bits: rows padded to 64 bits -> 2 words of 64 bits for L = 100
    assert pgg.pgg_device_bytes(pgg.make_params(100, 3.8, layout="bits")) == 100 * 16
    assert pgg.pgg_device_bytes(pgg.make_params(4096, 3.8, layout="bits")) == 4096 * 512
    assert pgg.pgg_device_bytes(pgg.make_params(102, 3.8)) == 0


@pytest.mark.parametrize("kw", [dict(L=6), dict(L=0), dict(L=32772), dict(K=0.0), dict(K=-1.0),
                                dict(r=float("nan")), dict(r=-0.5), dict(p0=1.5),
                                dict(p0=float("nan")), dict(layout=7),
                                dict(layout="int8", kernel="rowband"),
                                dict(layout="bits", kernel="colour"), dict(kernel=9),
                                dict(L=32768, kernel="rowband_staged"),
                                dict(layout="int8", kernel="rowband_staged"),
                                dict(layout="int8", kernel="strip"),
                                dict(L=32768, kernel="strip"),
                                dict(kernel="strip", tile=2),
                                dict(kernel="strip", tile=101),
                                dict(kernel="rowband", tile=26),
                                dict(L=60, kernel="segment"), dict(kernel="segment", tile=48),
                                dict(kernel="segment", tile=96), dict(layout="int8", L=60, kernel="segment"),
                                dict(kernel="segment", group=3), dict(kernel="segment", group=16),
                                dict(kernel="rowband", group=4), dict(layout="int8", L=60, group=4),
                                dict(L=32768, kernel="segment", tile=32736),
                                dict(L=100, kernel="segment", tile=50),
                                dict(L=480, kernel="segment_pair"), dict(L=516, kernel="segment_pair"),
                                dict(L=512, kernel="segment_pair", tile=480),
                                dict(L=512, kernel="segment_pair", group=4),
                                dict(layout="int8", L=480, kernel="segment_pair"),
                                dict(layout="int8", kernel="colour", group=2),
                                dict(L=32768, kernel="segment", tile=16384, group=8),
                                dict(schedule=2), dict(L=100, schedule="tiled"), dict(L=92, schedule="tiled", layout="int8"),
                                dict(L=96, schedule="tiled", kernel="segment"), dict(L=96, schedule="tiled", tile=32),
                                dict(L=96, schedule="tiled", group=4),
                                dict(L=32, kernel="resident"), dict(L=544, kernel="resident"),
                                dict(L=100, kernel="resident"), dict(L=240, kernel="resident"),
                                dict(L=128, kernel="resident", tile=32), dict(L=128, kernel="resident", group=2), dict(L=128, kernel="resident", group=32),
                                dict(L=128, schedule="tiled", kernel="resident")])
def test_init_rejects_invalid_parameters_before_touching_the_device(pgg, kw):
    args = dict(L=100, r=3.8, K=0.5, p0=0.5, seed=1, layout="bits", kernel="auto")
    args.update(kw)
    p = pgg.make_params(**args)
    with pytest.raises(pgg.PggError) as e:
        pgg.pgg_init(p)
    assert e.value.status == pgg.PGG_E_INVAL
    assert "invalid parameters" in pgg.load().pgg_last_error().decode()


@pytest.mark.parametrize("layout", ["int8", "bits"])
def test_init_rejects_a_misaligned_caller_buffer_before_touching_the_device(pgg, layout):
    p = pgg.make_params(100, 3.8, layout=layout)
    h = pgg.ctypes.c_void_p()
    lib = pgg.load()
    st = lib.pgg_init(pgg.ctypes.byref(p), pgg.ctypes.c_void_p(0x10002), 1 << 20, None, pgg.ctypes.byref(h))
    assert st == pgg.PGG_E_INVAL and not h.value
    assert "aligned" in lib.pgg_last_error().decode()


def test_null_handle_is_rejected(pgg):
    lib = pgg.load()
    assert lib.pgg_sweep(None, 1, None) == pgg.PGG_E_INVAL
    assert lib.pgg_coop_count(None, None) == pgg.PGG_E_INVAL
    lib.pgg_destroy(None)  # no-op


def test_engine_has_no_cpu_fallback():
    # The product modules never import the oracle.
    pkg = os.path.join(ROOT, "paper_1704_08098_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "pgg_ref_" not in text, f


@pytest.mark.parametrize("bad", [dict(L=60), dict(L=130), dict(r=-1.0), dict(K=0.0), dict(p0=2.0),
                                 dict(schedule="tiled"), dict(schedule=5)])
def test_ensemble_calls_reject_invalid_replicas_before_touching_the_device(pgg, bad):
    reps = [dict(L=128, r=3.8, seed=1), dict(L=256, r=3.7, seed=2)]
    reps[1].update(bad)
    with pytest.raises(pgg.PggError) as e:
        pgg.Ensemble(reps)
    assert e.value.status == pgg.PGG_E_INVAL
    with pytest.raises(pgg.PggError) as e:
        pgg.ensemble_autotune(reps)
    assert e.value.status == pgg.PGG_E_INVAL
    assert "replica 1" in pgg.load().pgg_last_error().decode()


def test_tiled_ensemble_rules(pgg):
    # every replica one schedule; L % 8 == 0 for the tiled one; nothing to autotune
    for reps in ([dict(L=128, r=3.8, seed=1, schedule="tiled"), dict(L=132, r=3.8, seed=2, schedule="tiled")],
                 [dict(L=128, r=3.8, seed=1, schedule="tiled"), dict(L=128, r=3.8, seed=2)]):
        with pytest.raises(pgg.PggError) as e:
            pgg.Ensemble(reps)
        assert e.value.status == pgg.PGG_E_INVAL and "replica 1" in pgg.load().pgg_last_error().decode()
    with pytest.raises(pgg.PggError) as e:
        pgg.ensemble_autotune([dict(L=128, r=3.8, seed=1, schedule="tiled")])
    assert e.value.status == pgg.PGG_E_INVAL
    with pytest.raises(pgg.PggError) as e:
        pgg.Ensemble([dict(L=128, r=3.8, seed=1, schedule="tiled")], tiles=[64])
    assert e.value.status == pgg.PGG_E_INVAL
    assert "the tiled schedule needs L % 8 == 0 and tile 0" in str(e.value)


def test_ensemble_autotune_rejects_bad_arguments(pgg):
    reps = [dict(L=128, r=3.8, seed=1)]
    for probe in (0, 4097):
        with pytest.raises(pgg.PggError) as e:
            pgg.ensemble_autotune(reps, probe_sweeps=probe)
        assert e.value.status == pgg.PGG_E_INVAL
    lib = pgg.load()
    assert lib.pgg_ensemble_autotune(None, 1, 4, None, None, None, None) == pgg.PGG_E_INVAL


def test_plan_validates_before_touching_the_device(pgg):
    lib = pgg.load()
    k, t = ctypes.c_uint32(), ctypes.c_uint32()
    p = pgg.make_params(L=102, r=3.8)  # L not a multiple of 4
    assert lib.pgg_plan(ctypes.byref(p), ctypes.byref(k), ctypes.byref(t)) == pgg.PGG_E_INVAL
    p = pgg.make_params(L=128, r=3.8)
    assert lib.pgg_plan(ctypes.byref(p), None, ctypes.byref(t)) == pgg.PGG_E_INVAL
