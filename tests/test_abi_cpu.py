"""CPU-side checks of the C ABI: the library loads, exports every function
include/cm.h declares, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(cm_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def cm():
    import paper_2012_07145_amd as cm
    return cm


def test_header_declares_the_boundary():
    names = _declared_functions()
    for f in ("cm_eval_batch", "cm_topk_per_query", "cm_model_create", "cm_workspace_create"):
        assert f in names


def test_library_exports_every_declared_symbol(cm):
    from paper_2012_07145_amd import _lib
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(_lib.EXPORTS) <= set(_declared_functions())


def test_version(cm):
    assert cm.cm_version() == (0 << 16) | 1


def test_invalid_arguments_are_rejected_before_device_work(cm):
    from paper_2012_07145_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.cm_model_create(None, None, ctypes.byref(h)) == _lib.CM_EINVAL
    bad = _lib.cm_model_desc(56, 40, 24, 31, 8)
    blob = (ctypes.c_float * 4184)()
    assert L.cm_model_create(ctypes.byref(bad), blob, ctypes.byref(h)) == _lib.CM_EINVAL
    assert b"56/40/24/32/8" in L.cm_last_error()
    good = _lib.cm_model_desc(56, 40, 24, 32, 8)
    blob[7] = float("nan")
    assert L.cm_model_create(ctypes.byref(good), blob, ctypes.byref(h)) == _lib.CM_EINVAL
    wd = _lib.cm_workspace_desc(0, 1, 1, 1, 8)
    assert L.cm_workspace_create(ctypes.byref(wd), ctypes.byref(h)) == _lib.CM_EINVAL
    wd = _lib.cm_workspace_desc(1, 1, 1, 1, 257)
    assert L.cm_workspace_create(ctypes.byref(wd), ctypes.byref(h)) == _lib.CM_EINVAL
    assert L.cm_eval_batch(None, 0, None, None, None, None) == _lib.CM_EINVAL
    assert L.cm_topk_per_query(None, None, 8, None, None, None, None) == _lib.CM_EINVAL
    assert L.cm_model_destroy(None) == _lib.CM_EINVAL
    assert L.cm_workspace_destroy(None) == _lib.CM_EINVAL


def test_binding_refuses_wrong_parameter_count(cm):
    import numpy as np
    with pytest.raises(ValueError):
        cm.cm_model_create(np.zeros(10, np.float32))
