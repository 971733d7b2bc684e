"""Host-side checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad input before touching a device."""
import ctypes
import os

import pytest

from paper_2406_01322_amd import psms

pytestmark = pytest.mark.skipif(not os.path.exists(psms.LIB_PATH), reason="libpsms.so not built")


def test_library_exports_every_header_symbol():
    names = psms.header_functions()
    assert len(names) >= 14
    L = psms.lib()
    missing = [nm for nm in names if not hasattr(L, nm)]
    assert missing == []
    assert set(names) == set(psms._SIGS)


def test_workspace_bytes_grows_with_n_and_precision():
    b32 = psms.workspace_bytes(psms.make_params(32, 100, 1, 0.05, 20, 1e-3))
    b64 = psms.workspace_bytes(psms.make_params(64, 100, 1, 0.05, 20, 1e-3))
    b128 = psms.workspace_bytes(psms.make_params(128, 100, 1, 0.05, 20, 1e-3))
    b128m = psms.workspace_bytes(psms.make_params(128, 100, 1, 0.05, 20, 1e-3, precision="mixed"))
    assert 0 < b32 < b64 < b128
    assert b128m < b128
    assert b32 % 256 == 0


@pytest.mark.parametrize("field,value", [("re", 0.0), ("we", -1.0), ("ch", float("nan")), ("pe", 0.0),
                                         ("dt", -1e-3), ("n", 100), ("n", 0), ("precision", 7), ("cube", 2), ("cube", -1)])
def test_invalid_params_rejected(field, value):
    p = psms.make_params(32, 100, 1, 0.05, 20, 1e-3)
    setattr(p, field, value)
    b = ctypes.c_size_t(0)
    code = psms.lib().psms_workspace_bytes(ctypes.byref(p), ctypes.byref(b))
    assert code == -1
    assert len(psms.lib().psms_last_error()) > 0


def test_channel_geometry_reports_not_supported():
    p = psms.make_params(32, 100, 1, 0.05, 20, 1e-3, geometry=psms.CHANNEL)
    b = ctypes.c_size_t(0)
    assert psms.lib().psms_workspace_bytes(ctypes.byref(p), ctypes.byref(b)) == -4


def test_create_rejects_small_or_misaligned_workspace_before_the_device():
    L = psms.lib()
    p = psms.make_params(32, 100, 1, 0.05, 20, 1e-3)
    need = psms.workspace_bytes(p)
    ctx = ctypes.c_void_p()
    assert L.psms_create(ctypes.byref(ctx), ctypes.byref(p), ctypes.c_void_p(4096), need - 1, None) == -2
    assert L.psms_create(ctypes.byref(ctx), ctypes.byref(p), ctypes.c_void_p(4096 + 8), need, None) == -2
    assert L.psms_create(ctypes.byref(ctx), ctypes.byref(p), None, need, None) == -2
    assert ctx.value is None


def test_null_context_calls_fail_cleanly():
    L = psms.lib()
    assert L.psms_step(None, 1) == -1
    assert L.psms_init_state(None, None, None) == -1
    d = psms.Diag()
    assert L.psms_diagnostics(None, ctypes.byref(d)) == -1
    assert L.psms_version().startswith(b"psms")
