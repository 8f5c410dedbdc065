"""CPU-side checks of the C ABI: the library loads, exports every entry point
declared in include/gp.h, and rejects invalid arguments before any device
work (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2403_12797_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("gp_fit", "gp_predict", "gp_submit", "gp_poll", "gp_ctx_create", "gp_ctx_destroy",
                 "gp_model_free", "gp_model_get", "gp_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = B.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(B.EXPORTED) == sorted(_declared())


def test_null_arguments_rejected():
    lib = B.load()
    out = C.c_void_p()
    prm = B.make_params(2, 4, 0.1, 1.0, 1.0)
    assert lib.gp_fit(None, C.byref(prm), None, None, 10, None, C.byref(out)) == B.GP_EINVAL
    assert "NULL" in B.last_error()
    assert lib.gp_predict(None, None, None, 0, None, None, None) == B.GP_EINVAL
    assert lib.gp_model_get(None, 0, None, 0) == B.GP_EINVAL
    assert lib.gp_model_info(None, None, None, None, None, None) == B.GP_EINVAL
    assert lib.gp_poll(None, 1, 0, None) == B.GP_EINVAL
    assert lib.gp_submit(None, None, None) == B.GP_EINVAL
    assert lib.gp_ctx_create(0, 0, None) == B.GP_EINVAL
    assert lib.gp_ctx_destroy(None) == B.GP_OK
    assert lib.gp_model_free(None) == B.GP_OK


def test_ctx_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert B.load().gp_ctx_create(0, 0, C.byref(h)) == B.GP_EDEVICE
    assert h.value is None
