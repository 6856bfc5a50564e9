"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/rzf.h, and validates arguments before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2512_16543_amd import rzf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rzf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rzf_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert "rzf_init" in names and "rzf_update" in names and "rzf_full" in names
    assert "rzf_sum_rate" in names
    L = rzf.lib()
    for n in names:
        assert hasattr(L, n), n
    # the binding wraps every declared function
    assert set(names) <= set(rzf._SIGS)


def test_graph_entry_points_check_arguments():
    L = rzf.lib()
    out = ctypes.c_void_p()
    assert L.rzf_graph_update(None, 1, None, 0.9, None, ctypes.byref(out)) == rzf.RZF_E_INVALID
    assert L.rzf_graph_full(None, 1, None, None, ctypes.byref(out)) == rzf.RZF_E_INVALID
    assert L.rzf_graph_launch(None) == rzf.RZF_E_INVALID
    assert L.rzf_graph_destroy(None) == rzf.RZF_E_INVALID
    e = rzf.TuneEntry(64, 256, 32, 64, 4)
    assert L.rzf_tune_table(None, 1, ctypes.byref(e)) == rzf.RZF_E_INVALID


def test_tuning_table_file_is_well_formed():
    # the committed autotuner table: every entry in range with valid knobs
    path = rzf.TUNING_PATH
    if not os.path.exists(path):
        pytest.skip("no tuning table written yet")
    entries = rzf.load_tuning(path)
    assert entries
    for e in entries:
        assert 1 <= e["K"] <= 256 and 1 <= e["N"] <= 4096
        assert e["precoder_rows"] in (32, 64, 256) and e["batch_precoder_rows"] in (32, 64, 256)
        assert 0 <= e["rate_splits"] <= 8


def test_params_default_values():
    p = rzf.default_params()
    assert (p.k_init, p.p, p.i_max, p.switch_ratio, p.reset_period, p.P) == (2, 5, 0, 0.5, 0, 1.0)
    assert (p.seed, p.track_id, p.kinit_policy) == (0, 0, rzf.KINIT_FIXED)
    assert rzf.lib().rzf_params_default(None) == rzf.RZF_E_INVALID


def test_track_bytes():
    assert rzf.track_bytes(0, 10) == 0
    assert rzf.track_bytes(257, 10) == 0
    # large tracks carry the blocked kernels' workspace
    assert rzf.track_bytes(65, 10) > rzf.track_bytes(64, 10) + 3 * 65 * 65 * 8
    assert rzf.track_bytes(4, 0) == 0
    b = rzf.track_bytes(64, 256)
    assert b >= 8 * (64 * 64 * 3 + 64 * 256) + 16 * 64 * 64
    assert rzf.track_bytes(64, 512) > b


def test_status_strings():
    for s in range(7):
        assert rzf.status_string(s)
    assert rzf.status_string(rzf.RZF_E_NOT_HPD) == "Gram matrix not positive definite"


def test_null_arguments_rejected_without_device():
    L = rzf.lib()
    assert L.rzf_sync(None) == rzf.RZF_E_INVALID
    assert L.rzf_ctx_destroy(None) == rzf.RZF_E_INVALID
    assert L.rzf_ctx_create(0, None, None, 1 << 20, None) == rzf.RZF_E_INVALID
    out = ctypes.c_void_p()
    assert L.rzf_init(None, 4, 4, None, 4, 1.0, None, ctypes.byref(out)) == rzf.RZF_E_INVALID
    assert L.rzf_update(None, None, 4, 0.9, None, 4, None) == rzf.RZF_E_INVALID
    assert L.rzf_full(None, 4, 4, None, 4, 1.0, 1.0, None, 4) == rzf.RZF_E_INVALID
    assert L.rzf_sum_rate(None, 4, 4, None, 4, None, 4, 1.0, 0.1, None, None) == rzf.RZF_E_INVALID
    assert L.rzf_get_inverse(None, None) == rzf.RZF_E_INVALID
    assert L.rzf_track_destroy(None) == rzf.RZF_E_INVALID
    assert L.rzf_debug_sketch(None, 0, 0, 0, 0, 4, 4, None, None) == rzf.RZF_E_INVALID
    r = ctypes.c_double()
    assert L.rzf_tune_switch(None, 64, 256, 0, ctypes.byref(r), None, None, None) == rzf.RZF_E_INVALID
    n = ctypes.c_size_t(0)
    assert L.rzf_track_export(None, None, ctypes.byref(n)) == rzf.RZF_E_INVALID
    blob = ctypes.create_string_buffer(64)
    assert L.rzf_track_import(None, blob, 64, ctypes.byref(out)) == rzf.RZF_E_INVALID
    assert L.rzf_server_params_default(None) == rzf.RZF_E_INVALID
    sp = rzf.server_params()
    assert (sp.max_batch, sp.max_wait_us, sp.tol, sp.mode, sp.max_inflight) == (512, 1000.0, 0.999, 0, 2)
    assert L.rzf_server_create(None, ctypes.byref(sp), ctypes.byref(out)) == rzf.RZF_E_INVALID
    assert L.rzf_server_submit(None, None, None, 4, None, 4, 0) == rzf.RZF_E_INVALID
    assert L.rzf_server_drain(None) == rzf.RZF_E_INVALID
    assert L.rzf_server_destroy(None) == rzf.RZF_E_INVALID


def test_ctx_create_arena_too_small():
    out = ctypes.c_void_p()
    assert rzf.lib().rzf_ctx_create(0, None, None, 1024, ctypes.byref(out)) == rzf.RZF_E_NOMEM


def test_no_cpu_fallback_when_library_missing(monkeypatch, tmp_path):
    monkeypatch.setattr(rzf, "_lib", None)
    monkeypatch.setattr(rzf, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        rzf.lib()


def test_params_check_ranges():
    ok = rzf.default_params()
    assert rzf.params_check(ok, 64) == rzf.RZF_OK
    assert rzf.params_check(ok, 0) == rzf.RZF_E_SHAPE
    assert rzf.params_check(ok, 257) == rzf.RZF_E_SHAPE
    assert rzf.lib().rzf_params_check(None, 8) == rzf.RZF_E_INVALID
    # k_init and p are bounded by RZF_KMAX (a huge value would overflow d = k0 + p)
    for kw in (dict(k_init=0), dict(k_init=257), dict(k_init=2**31 - 1), dict(p=-1), dict(p=257),
               dict(p=2**31 - 1), dict(i_max=65), dict(switch_ratio=0.0), dict(switch_ratio=1.5),
               dict(P=0.0), dict(kinit_policy=2), dict(early_fallback=2), dict(precision=3),
               dict(error_feedback=2), dict(reset_period=-1)):
        assert rzf.params_check(rzf.default_params(**kw), 64) == rzf.RZF_E_INVALID, kw
    assert rzf.params_check(rzf.default_params(k_init=256, p=256), 256) == rzf.RZF_OK


def test_switch_ratio_within_woodbury_workspace():
    # Alg. 2 takes Woodbury for k_est <= floor(ratio K); the workspace holds
    # min(K, max(32, K / 2)) ranks, and a ratio beyond it is refused, not capped
    def check(ratio, K):
        return rzf.params_check(rzf.default_params(switch_ratio=ratio), K)
    for K in (1, 16, 32):
        assert check(1.0, K) == rzf.RZF_OK          # every rank fits
    assert check(0.5, 64) == rzf.RZF_OK and check(0.5, 256) == rzf.RZF_OK
    assert check(32.5 / 64, 64) == rzf.RZF_OK     # floor = 32
    assert check(33 / 64, 64) == rzf.RZF_E_INVALID
    assert check(1.0, 33) == rzf.RZF_E_INVALID     # 33 > 32
    assert check(48 / 96, 96) == rzf.RZF_OK and check(49 / 96, 96) == rzf.RZF_E_INVALID
    assert check(0.75, 256) == rzf.RZF_E_INVALID


def test_full_noalloc_argument_checks_without_device():
    # refused before anything reaches a device (the pointers are never read)
    L = rzf.lib()
    fake = ctypes.c_void_p(256)
    assert L.rzf_full_noalloc(None, 4, 4, None, 4, 1.0, 1.0, fake, 4, None) == rzf.RZF_E_INVALID
    assert L.rzf_full_noalloc(None, 257, 4, fake, 4, 1.0, 1.0, fake, 257, None) == rzf.RZF_E_SHAPE
    assert L.rzf_full_noalloc(None, 4, 4097, fake, 4097, 1.0, 1.0, fake, 4, None) == rzf.RZF_E_SHAPE
    assert L.rzf_full_noalloc(None, 0, 4, fake, 4, 1.0, 1.0, fake, 4, None) == rzf.RZF_E_SHAPE
    assert L.rzf_full_noalloc(None, 4, 8, fake, 7, 1.0, 1.0, fake, 4, None) == rzf.RZF_E_SHAPE
    assert L.rzf_full_noalloc(None, 4, 8, fake, 8, 1.0, 1.0, fake, 3, None) == rzf.RZF_E_SHAPE
    assert L.rzf_full_noalloc(None, 4, 8, fake, 8, -1.0, 1.0, fake, 4, None) == rzf.RZF_E_INVALID
    assert L.rzf_full_noalloc(None, 4, 8, fake, 8, float("nan"), 1.0, fake, 4, None) == rzf.RZF_E_INVALID
    assert L.rzf_full_noalloc(None, 4, 8, fake, 8, 1.0, 0.0, fake, 4, None) == rzf.RZF_E_INVALID
