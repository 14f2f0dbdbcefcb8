"""CPU checks of the C ABI: the library loads, exports every declared symbol, and its host
logic (parameter layout, validation, error codes) behaves, without touching a GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

from workload import configs, params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmd.h")


@pytest.fixture(scope="module")
def fmd():
    from paper_2606_26089_amd import fmd as m
    if not os.path.exists(m.LIB_PATH):
        pytest.skip("libfmdet.so not built")
    m.lib()
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fmd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_documented_calls():
    names = declared_functions()
    for must in ("fmd_simulate", "fmd_model_create", "fmd_model_destroy", "fmd_param_count",
                 "fmd_last_error", "fmd_velocity", "fmd_noise", "fmd_pack_padded"):
        assert must in names


def test_library_exports_every_declared_symbol(fmd):
    L = ctypes.CDLL(fmd.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.parametrize("cfg", [configs.SMALL_MODEL, configs.BASE_MODEL,
                                 configs.BASE_MODEL.with_precision(configs.BF16)])
def test_param_count_matches_layout(fmd, cfg):
    assert fmd.param_count(cfg) == params.count(cfg)


@pytest.mark.parametrize("change", [dict(d_model=60), dict(n_heads=5), dict(mlp_ratio=2),
                                    dict(t_embed_dim=16), dict(f_truth=8), dict(n_max=0),
                                    dict(precision=7), dict(d_model=512, n_heads=4)])
def test_invalid_configs(fmd, change):
    c = dict(vars(configs.SMALL_MODEL))
    c.update(change)
    assert fmd.param_count(c) == 0
    with pytest.raises(fmd.FmdError) as e:
        fmd.Model(c, np.zeros(10, dtype=np.float32))
    assert e.value.status in (fmd.E_INVALID, fmd.E_UNSUPPORTED)


def test_wrong_parameter_count_is_rejected_before_any_device_work(fmd):
    flat = params.draw(configs.SMALL_MODEL, 0)
    with pytest.raises(fmd.FmdError) as e:
        fmd.Model(configs.SMALL_MODEL, flat[:-1])
    assert e.value.status == fmd.E_INVALID and "parameter vector" in str(e.value)


@pytest.fixture
def field(fmd):
    m = fmd.Model.linear_field(0.5, 0.25)      # touches no device until it runs
    yield m
    m.close()


def _sched(**kw):
    d = dict(scheme=configs.EULER, n_steps=4, t0=0.0, t1=1.0)
    d.update(kw)
    return d


@pytest.mark.parametrize("offsets,msg", [([1, 3], "offsets[0]"), ([0, 3, 2], "decrease")])
def test_bad_offsets(fmd, field, offsets, msg):
    feat = np.zeros((4, 9), dtype=np.float32)
    with pytest.raises(fmd.FmdError) as e:
        field.simulate(offsets, feat, 0, _sched())
    assert e.value.status == fmd.E_INVALID and msg in str(e.value)


@pytest.mark.parametrize("sched,msg", [(_sched(n_steps=0), "n_steps"), (_sched(scheme=9), "scheme"),
                                       (_sched(t1=0.0), "t0 and t1"),
                                       (_sched(t1=float("nan")), "t0 and t1")])
def test_bad_schedule(fmd, field, sched, msg):
    with pytest.raises(fmd.FmdError) as e:
        field.simulate([0, 2], np.zeros((2, 9), dtype=np.float32), 0, sched)
    assert e.value.status == fmd.E_INVALID and msg in str(e.value)


def test_empty_batches_need_no_device(fmd, field):
    out = field.simulate([0, 0, 0], np.zeros((0, 9), dtype=np.float32), 0, _sched())
    assert out.shape == (0, 9)
    out = field.simulate([0], np.zeros((0, 9), dtype=np.float32), 0, _sched())
    assert out.shape == (0, 9)


def test_null_model_and_errors_are_reported(fmd):
    L = fmd.lib()
    ev = fmd.EventsIn(0, None, None, 0)
    s = fmd.Schedule(0, 1, 0.0, 1.0)
    o = fmd.EventsOut(None, 0)
    st = L.fmd_simulate(None, ctypes.byref(ev), 0, ctypes.byref(s), ctypes.byref(o), None)
    assert st == fmd.E_INVALID
    assert b"null model" in L.fmd_last_error()
    assert L.fmd_noise(0, None, 1, 9, None, None) == fmd.E_INVALID
    assert L.fmd_event_observables(None, None, None, None, None) == fmd.E_INVALID
    bad = np.array([0, 3, 1], dtype=np.int64)
    ev2 = fmd.EventsIn(2, bad.ctypes.data_as(fmd.P_int64), None, 0)
    assert L.fmd_event_observables(ctypes.byref(ev2), None, None, None, None) == fmd.E_INVALID
    assert b"offsets decrease" in L.fmd_last_error()
    zero = np.zeros(1, dtype=np.int64)
    ev0 = fmd.EventsIn(0, zero.ctypes.data_as(fmd.P_int64), None, 0)
    assert L.fmd_event_observables(ctypes.byref(ev0), None, None, None, None) == fmd.OK
    oo = np.zeros(3, dtype=np.int64)
    assert L.fmd_truth_select(None, 0.5, 128, oo.ctypes.data_as(fmd.P_int64), None, None) == fmd.E_INVALID
    assert L.fmd_truth_select(ctypes.byref(ev0), 0.0, 128, oo.ctypes.data_as(fmd.P_int64), None,
                              None) == fmd.E_INVALID
    assert L.fmd_truth_select(ctypes.byref(ev0), 0.5, -1, oo.ctypes.data_as(fmd.P_int64), None,
                              None) == fmd.E_INVALID
    assert L.fmd_truth_select(ctypes.byref(ev0), 0.5, 128, oo.ctypes.data_as(fmd.P_int64), None,
                              None) == fmd.OK
    assert L.fmd_pack_padded(None, None, 1, 4, 9, None, None, None) == fmd.E_INVALID
    assert L.fmd_debug_gemm(0, 4, 60, 32, None, None, None, 0, None, None, 0, None, -1, None) == fmd.E_INVALID
    assert L.fmd_model_destroy(None) == fmd.OK
    assert L.fmd_kernel_name(None, fmd.K_GEMM_UP) == b"k_gemm_up"


def test_binding_refuses_a_missing_library(monkeypatch, fmd):
    monkeypatch.setattr(fmd, "_lib", None)
    monkeypatch.setattr(fmd, "LIB_PATH", "/nonexistent/libfmdet.so")
    with pytest.raises(RuntimeError, match="missing"):
        fmd.lib()


def test_server_argument_checks_without_a_device(fmd, field):
    L = fmd.lib()
    cfg = fmd.ServerConfig(1 << 30, 0, 0)
    out = ctypes.c_void_p()
    assert L.fmd_server_create(None, ctypes.byref(cfg), ctypes.byref(out)) == fmd.E_INVALID
    assert L.fmd_server_create(field._h, ctypes.byref(cfg), ctypes.byref(out)) == fmd.E_UNSUPPORTED
    assert L.fmd_server_destroy(None) == fmd.OK
    rid = ctypes.c_uint64()
    assert L.fmd_server_submit(None, None, 0, None, ctypes.byref(rid)) == fmd.E_INVALID


@pytest.mark.parametrize("reco,msg", [([1, 2, 3], r"reco offsets\[0\]"), ([0, 3, 2], "decrease"),
                                      ([0, 2, 3], "no truth particle")])
def test_reco_offsets_are_validated_on_the_host(fmd, field, reco, msg):
    feat = np.zeros((2, 9), dtype=np.float32)
    with pytest.raises(fmd.FmdError, match=msg):
        field.simulate([0, 2, 2], feat, 0, _sched(), reco_offsets=reco)


def test_reco_offsets_without_slots_need_no_device(fmd, field):
    feat = np.zeros((5, 9), dtype=np.float32)
    out = field.simulate([0, 2, 5], feat, 0, _sched(), reco_offsets=[0, 0, 0])
    assert out.shape == (0, 9)
    with pytest.raises(ValueError):
        field.simulate([0, 2, 5], feat, 0, _sched(), reco_offsets=[0, 1])
