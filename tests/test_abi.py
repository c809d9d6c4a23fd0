"""C ABI checks that need no GPU: the library loads, exports every declared symbol,
validates its arguments synchronously, sizes workspaces, and builds e^{-dtau K} on the
host (model setup) in agreement with the oracle's eigen-decomposition."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_1802_06177_amd import _abi
import paper_1802_06177_amd as slmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(not os.path.exists(_abi.LIB_PATH), reason="library not built")


def _declared():
    txt = open(os.path.join(ROOT, "include", "slmc.h")).read()
    return sorted(set(re.findall(r"\b(slmc_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_exactly_the_binding_exports():
    assert sorted(_abi.EXPORTS) == _declared()


def test_every_declared_symbol_is_exported():
    L = _abi.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert slmc.version() >= 10000


def test_expk_matches_oracle_eigh():
    for (Lx, Ly, t, mu, dt) in ((4, 4, 1.0, 0.0, 0.1), (2, 3, 1.0, 0.3, 0.1), (6, 4, 0.7, -0.2, 0.05),
                                (16, 16, 1.0, 0.0, 0.1), (20, 20, 1.0, 0.0, 0.1)):
        m = slmc.model(Lx, Ly, 10, 5, t=t, mu=mu, dtau=dt)
        E = slmc.expk(m)
        Eo = oracle.expk(oracle.hopping_matrix(Lx, Ly, t, mu), dt)
        assert np.max(np.abs(E - Eo)) < 1e-14


def _call_logdet(models, n_items, opt=None, ws_bytes=0, **batch):
    arr = (_abi.Model * len(models))(*models)
    ba = slmc._BatchArgs(n_items, batch.get("model_idx"), batch.get("x_off"), batch.get("g_off"))
    opt = opt or slmc.options()
    vp = C.c_void_p
    dummy = vp(16)   # never dereferenced: validation fails first
    return _abi.lib().slmc_logdet(arr, len(models), C.byref(ba.batch), C.byref(opt), dummy, dummy,
                                  dummy, dummy, dummy if ws_bytes else None, ws_bytes, None)


def test_validation_errors_are_synchronous_codes():
    L = _abi.lib()
    good = slmc.model(4, 4, 40, 10)
    assert _call_logdet([slmc.model(1, 4, 40, 10)], 2) == _abi.SLMC_E_SHAPE
    assert b"Lx" in L.slmc_last_error()
    assert _call_logdet([slmc.model(32, 32, 40, 10)], 2) == _abi.SLMC_E_SHAPE      # N > 448
    assert _call_logdet([slmc.model(4, 4, 40, 0)], 2) == _abi.SLMC_E_ARG          # n_s < 1
    assert _call_logdet([slmc.model(4, 4, 40, 41)], 2) == _abi.SLMC_E_ARG         # n_s > Ltau
    assert _call_logdet([slmc.model(4, 4, 40, 10, dtau=-0.1)], 2) == _abi.SLMC_E_ARG
    assert _call_logdet([slmc.model(4, 4, 40, 10, lam=float("nan"))], 2) == _abi.SLMC_E_ARG
    assert _call_logdet([good], 2, opt=slmc.options(precision=7)) == _abi.SLMC_E_ARG
    assert _call_logdet([good], 2, opt=slmc.options(acc_chunk=3)) == _abi.SLMC_E_ARG
    assert _call_logdet([good], 2, opt=slmc.Options(0, 0, 0, 4)) == _abi.SLMC_E_ARG      # unknown flag
    assert _call_logdet([good], 2, opt=slmc.options(residual_steps=2)) == _abi.SLMC_E_ARG
    assert _call_logdet([good], 2, ws_bytes=0) == _abi.SLMC_E_WORKSPACE
    need = slmc.workspace_bytes(good, 2)
    assert _call_logdet([good], 2, ws_bytes=need - 1) == _abi.SLMC_E_WORKSPACE
    assert _call_logdet([good, good], 2) == _abi.SLMC_E_ARG                     # needs model_idx
    assert _call_logdet([good, good], 2, model_idx=[0, 2], x_off=[0, 640]) == _abi.SLMC_E_ARG
    assert _call_logdet([good], 2, x_off=[0, -5]) == _abi.SLMC_E_ARG
    assert _call_logdet([good], 0, ws_bytes=0) == _abi.SLMC_OK                  # empty batch


def test_sweep_and_accept_validation():
    L = _abi.lib()
    vp = C.c_void_p(16)
    odd = slmc.model(4, 4, 41, 1)
    eff = slmc.eff_model(Jk=1.0, Js=(0.1, 0.1, 0.1))
    assert L.slmc_eff_sweep(C.byref(odd), C.byref(eff), 2, vp, 1, 1, 0, vp, None) == _abi.SLMC_E_SHAPE
    ten = slmc.model(10, 10, 40, 10)
    assert L.slmc_eff_sweep(C.byref(ten), C.byref(eff), 2, vp, 1, 1, 0, vp, None) == _abi.SLMC_E_SHAPE
    ok = slmc.model(12, 12, 40, 10)
    assert L.slmc_eff_sweep(C.byref(ok), C.byref(eff), 2, None, 1, 1, 0, vp, None) == _abi.SLMC_E_ARG
    assert L.slmc_eff_sweep(C.byref(ok), C.byref(eff), -1, vp, 1, 1, 0, vp, None) == _abi.SLMC_E_ARG
    opt = slmc.options()
    need = L.slmc_accept_workspace_bytes(C.byref(ok), 4, C.byref(opt))
    assert need > 0
    rc = L.slmc_cumulative_accept(C.byref(ok), C.byref(eff), C.byref(opt), 4, vp, vp, vp, vp, 1, 0,
                                  vp, vp, None, None, vp, need - 1, None)
    assert rc == _abi.SLMC_E_WORKSPACE
    rc = L.slmc_cumulative_accept(C.byref(ok), C.byref(eff), C.byref(opt), 0, vp, vp, vp, vp, 1, 0,
                                  vp, vp, None, None, vp, need, None)
    assert rc == _abi.SLMC_E_ARG
    rc = L.slmc_log_weight(C.byref(ok), C.byref(opt), 4, vp, vp, None, vp, need - 1, None)
    assert rc == _abi.SLMC_E_WORKSPACE
    rc = L.slmc_log_weight(C.byref(ok), C.byref(opt), 4, None, vp, None, vp, need, None)
    assert rc == _abi.SLMC_E_ARG


def test_workspace_grows_with_batch_and_sums_over_models():
    m1, m2 = slmc.model(8, 8, 80, 10), slmc.model(12, 12, 120, 10)
    a = slmc.workspace_bytes(m1, 10)
    b = slmc.workspace_bytes(m1, 20)
    assert 0 < a < b
    both = slmc.workspace_bytes([m1, m2], 30, model_idx=[0] * 10 + [1] * 20,
                                x_off=np.arange(30) * 20000)
    assert both == a + slmc.workspace_bytes(m2, 20)


def test_profile_hooks_without_gpu_work():
    slmc.profile_reset()
    out = slmc.profile_read()
    assert set(out) == {"seg_chain", "wy_apply", "qr", "vupd", "lu", "lu_solve", "residual",
                        "eff_sweep"}
    assert all(v == (0.0, 0) for v in out.values())
    L = _abi.lib()
    ms, n = C.c_double(), C.c_int64()
    assert L.slmc_profile_read(9, C.byref(ms), C.byref(n)) == _abi.SLMC_E_ARG


def test_binding_refuses_cpu_tensors():
    import torch
    x = torch.zeros((2, 40, 16), dtype=torch.float64)
    with pytest.raises(TypeError):
        slmc.logdet(slmc.model(4, 4, 40, 10), x)


def test_binding_rejects_mis_shaped_tensors_before_any_call():
    # the C ABI takes raw pointers; the binding checks every size first (on CPU tensors the
    # shape check fires before the device check)
    import torch
    m = slmc.model(4, 4, 40, 10)
    f64 = dict(dtype=torch.float64)
    with pytest.raises(ValueError):
        slmc.logdet(m, torch.zeros((2, 40, 15), **f64))
    with pytest.raises(ValueError):
        slmc.green(m, torch.zeros((2, 40, 16), **f64), G=torch.zeros((2, 16, 15), **f64))
    with pytest.raises(ValueError):     # packed item past the end of x
        slmc.logdet(m, torch.zeros(2 * 640 - 1, **f64), x_off=[0, 640], n_items=2)
    with pytest.raises(ValueError):     # n_items larger than x holds
        slmc.logdet(m, torch.zeros(640, **f64), n_items=2)
    m2 = slmc.model(6, 6, 30, 10)
    with pytest.raises(ValueError):     # model index out of range
        slmc.green([m, m2], torch.zeros(2000, **f64), model_idx=[0, 2], x_off=[0, 640],
                   g_off=[0, 256], n_items=2, G=torch.zeros(2000, **f64))
    with pytest.raises(ValueError):     # G too small for the packed items
        slmc.green([m, m2], torch.zeros(1720, **f64), model_idx=[0, 1], x_off=[0, 640],
                   g_off=[0, 256], n_items=2, G=torch.zeros(1551, **f64))
    with pytest.raises(ValueError):
        slmc.eff_sweep(m, slmc.eff_model(), torch.zeros((2, 39, 16), **f64), 1, 1, 0)
    with pytest.raises(ValueError):
        slmc.eff_energy(m, slmc.eff_model(), torch.zeros((2, 40), **f64))
    with pytest.raises(ValueError):
        slmc.log_weight(m, torch.zeros((2, 16, 40), **f64))
    x = torch.zeros((3, 40, 16), **f64)
    with pytest.raises(ValueError):
        slmc.cumulative_accept(m, slmc.eff_model(), x, torch.zeros((2, 40, 16), **f64),
                               torch.zeros(3, **f64), torch.zeros(3, **f64), 1, 0)
    with pytest.raises(ValueError):
        slmc.cumulative_accept(m, slmc.eff_model(), x, x.clone(), torch.zeros(2, **f64),
                               torch.zeros(3, **f64), 1, 0)
    with pytest.raises(ValueError):
        slmc.cumulative_accept(m, slmc.eff_model(), x, x.clone(), torch.zeros(3, **f64),
                               torch.zeros(3, **f64), 1, 0, G_prop=torch.zeros((3, 16, 17), **f64))
    # well-shaped CPU tensors get past the shape checks and are refused as CPU tensors
    with pytest.raises(TypeError):
        slmc.green([m, m2], torch.zeros(1720, **f64), model_idx=[0, 1], x_off=[0, 640],
                   g_off=[0, 256], n_items=2, G=torch.zeros(1552, **f64))


def test_tuning_lookup_defaults_without_gpu_work(tmp_path, monkeypatch):
    # no tuning yet: the defaults; a cache file is read at the first lookup after a clear
    m = slmc.model(6, 6, 30, 10)
    t, tuned = slmc.tuning(m, 8, slmc.options("int8x5"))
    assert not tuned and t["schedule"] == "default" and t["seg_ahead"] == 2 and t["gate"] == 1
    f = tmp_path / "tune.txt"
    f.write_text("6 6 30 10 5 8 2 3 0 1 1 1.250000\n")
    monkeypatch.setenv("SLMC_TUNE_CACHE", str(f))
    slmc.cache_clear()
    try:
        t, tuned = slmc.tuning(m, 7, slmc.options("int8x5"))   # batch 7 rounds up to 8
        assert tuned and t == {"schedule": "gated", "seg_ahead": 3, "gate": 0, "seg_mode": 1, "seg_cb": 1,
                               "ms_per_call": 1.25}
        assert not slmc.tuning(m, 9, slmc.options("int8x5"))[1]
        assert not slmc.tuning(m, 8, slmc.options("fp64"))[1]
    finally:
        monkeypatch.delenv("SLMC_TUNE_CACHE")
        slmc.cache_clear()
    assert not slmc.tuning(m, 8, slmc.options("int8x5"))[1]
