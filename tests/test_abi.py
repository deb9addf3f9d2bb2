"""The C ABI without a GPU: the library loads, exports what include/pwa.h
declares, validates arguments and reports a missing device cleanly."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1108_5673_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pwa.h")


def _header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pwa_[a-z_]+)\s*\(", text)))


def _lib():
    if not os.path.exists(_native.LIBRARY):
        pytest.skip("libpwa.so not built")
    return _native.lib()


def test_header_and_binding_agree():
    assert _header_functions() == sorted(_native.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = _lib()
    for name in _header_functions():
        assert hasattr(L, name), name


def test_header_compiles_as_c():
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        with open(src, "w") as f:
            f.write('#include "pwa.h"\nint main(void){pwa_info i; (void)i; return PWA_OK;}\n')
        subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                        "-c", src, "-o", os.path.join(d, "t.o")], check=True)


def _build(L, data, n, w, mc, n_acc, n_gen, flags):
    h = ctypes.c_void_p(123)
    st = L.pwa_build_table(data, n, w, mc, n_acc, n_gen, flags, None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("case", [
    dict(n=0), dict(w=0), dict(w=65), dict(flags=0), dict(flags=3), dict(flags=1 << 12),
    dict(n_gen=0), dict(n_acc=-1), dict(mc_null=True), dict(n_acc=5, n_gen=4),
    dict(flags=_native.PWA_FORM_AMPLITUDE | _native.PWA_INPUT_IS_TABLE),
    dict(flags=_native.PWA_FORM_AMPLITUDE, w=129), dict(data_null=True),
])
def test_invalid_arguments_rejected_before_device_use(case):
    L = _lib()
    a = np.ones((4, 4), np.complex64)
    data = None if case.get("data_null") else a.ctypes.data
    mc = None if case.get("mc_null") else a.ctypes.data
    st, h = _build(L, data, case.get("n", 4), case.get("w", 4), mc, case.get("n_acc", 2),
                   case.get("n_gen", 4), case.get("flags", _native.PWA_FORM_TABLE))
    assert st == _native.PWA_ERR_INVALID
    assert h.value is None
    assert _native.last_error()


def test_null_out_pointer_rejected():
    L = _lib()
    a = np.ones((4, 4), np.complex64)
    assert L.pwa_build_table(a.ctypes.data, 4, 4, None, 0, 1, 1, None, None) == _native.PWA_ERR_INVALID


def test_null_model_calls_rejected():
    L = _lib()
    v = np.zeros(8)
    out = ctypes.c_double()
    assert L.pwa_nll(None, v.ctypes.data, ctypes.byref(out), None) == _native.PWA_ERR_INVALID
    assert L.pwa_nll_grad(None, v.ctypes.data, ctypes.byref(out), v.ctypes.data, None) == \
        _native.PWA_ERR_INVALID
    assert L.pwa_model_info(None, None) == _native.PWA_ERR_INVALID
    assert L.pwa_nll_batched(None, 0, None, None, None, None, None) == _native.PWA_OK
    assert L.pwa_nll_batched(None, 1, None, None, None, None, None) == _native.PWA_ERR_INVALID
    L.pwa_free(None)


def test_no_device_reported_cleanly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except Exception:
        pass
    L = _lib()
    a = np.ones((4, 4), np.complex64)
    st, h = _build(L, a.ctypes.data, 4, 4, None, 0, 1, _native.PWA_FORM_TABLE)
    assert st == _native.PWA_ERR_NO_DEVICE
    assert h.value is None
    assert "device" in _native.last_error()


def test_model_refuses_to_run_without_library(monkeypatch):
    import paper_1108_5673_amd as pwa
    monkeypatch.setattr(_native, "LIBRARY", "/nonexistent/libpwa.so")
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        pwa.Model(np.ones((4, 2), np.complex64))
