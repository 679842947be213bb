"""The C ABI library loads and exports every function include/mpsl.h declares
(CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpsl.h")
LIB = os.path.join(ROOT, "paper_1407_3868_amd", "libmpsl.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpsl_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.isfile(LIB):
        pytest.fail("libmpsl.so is not built: run paper_1407_3868_amd/build.py")
    from paper_1407_3868_amd import _lib
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared()
    for must in ["mpsl_create", "mpsl_set_layers", "mpsl_set_geometry", "mpsl_set_contour",
                 "mpsl_apply_dev", "mpsl_m2l_dev", "mpsl_m2s_dev", "mpsl_reflect_dev", "mpsl_s2l_dev",
                 "mpsl_sapply_dev", "mpsl_solve", "mpsl_eval_field", "mpsl_rhs"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_1407_3868_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared()


def test_status_strings(lib):
    lib.mpsl_status_string.restype = ctypes.c_char_p
    assert lib.mpsl_status_string(0) == b"ok"
    assert lib.mpsl_status_string(-5) == b"invalid geometry"


def test_create_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    rc = lib.mpsl_create(ctypes.byref(h), 0, 0)
    assert rc != 0 and not h.value
