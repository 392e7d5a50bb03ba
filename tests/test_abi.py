"""CPU checks of the C ABI: the built library loads and exports every function the
header declares, the binding's table matches the header, and argument errors that
need no device are reported."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2607_05920_amd as fhe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fhe_mi355x.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fhe_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_table():
    assert header_functions() == sorted(fhe.EXPORTS)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fhe.LIB_PATH):
        pytest.skip("library not built")
    return fhe.load_library()


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", fhe.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (fhe_[a-z0-9_]+)$", out, flags=re.M))
    missing = set(header_functions()) - exported
    assert not missing, missing
    for name in header_functions():
        assert getattr(lib, name) is not None


def test_strerror_and_argument_errors_without_device(lib):
    assert lib.fhe_strerror(0) == b"ok"
    assert lib.fhe_strerror(-3) == b"beyond context limits or key level"
    h = ctypes.c_void_p()
    assert lib.fhe_ctx_create(0, 0, 10, ctypes.byref(h)) == -1     # bad limit, checked before the device
    assert lib.fhe_ctx_create(0, 10, 10, None) == -1
    assert lib.fhe_prime_count(None, None) == -1
    assert lib.fhe_mul_relin(None, None, 16, 100, None, None, None, None, None, None, 1, None) == -1
    lib.fhe_ctx_destroy(None)
    lib.fhe_evk_destroy(None)


def test_binding_fails_loudly_without_library(tmp_path):
    import importlib
    saved = fhe._lib
    try:
        fhe._lib = None
        with pytest.raises(fhe.LibraryMissing):
            fhe.load_library(str(tmp_path / "absent.so"))
    finally:
        fhe._lib = saved
