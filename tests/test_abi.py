"""The C-ABI library loads and exports every entry point its header declares (no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "exx.h")
LIB = os.path.join(ROOT, "paper_2304_05505_amd", "libexx.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:exx_status|const\s+char\s*\*)\s*(exx_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2304_05505_amd import build

        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_build_entry_points():
    syms = declared_symbols()
    for name in ("exx_isdf_fit", "exx_coulomb_V", "exx_build_K", "exx_create", "exx_destroy"):
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol(lib):
    from paper_2304_05505_amd import exx

    assert sorted(exx.EXPORTED) == declared_symbols()


def test_null_handle_paths_need_no_device(lib):
    lib.exx_last_error.restype = ctypes.c_char_p
    lib.exx_last_error.argtypes = [ctypes.c_void_p]
    assert lib.exx_last_error(None) == b"null handle"
    lib.exx_create.argtypes = [ctypes.c_void_p, ctypes.c_int]
    assert lib.exx_create(None, 0) == -1  # EXX_ERR_ARG
    lib.exx_destroy.argtypes = [ctypes.c_void_p]
    assert lib.exx_destroy(None) == -1
    # the calls beyond the build reject a null handle before touching the device
    vp = ctypes.c_void_p
    lib.exx_exchange_gradient.argtypes = [vp, vp, ctypes.c_int] + [vp] * 10
    assert lib.exx_exchange_gradient(None, None, 0, *([None] * 10)) == -1
    lib.exx_build_robust.argtypes = [vp, vp, ctypes.c_int] + [vp] * 9
    assert lib.exx_build_robust(None, None, 0, *([None] * 9)) == -1
