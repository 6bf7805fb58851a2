"""The C-ABI library loads on the host and exports every entry point the
public header declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "minsr.h")
LIB = os.path.join(ROOT, "paper_2608_18065_amd", "libminsr.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(minsr_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_five_calls():
    names = declared_symbols()
    for n in ("minsr_create_model", "minsr_sample", "minsr_local_energy", "minsr_jacobian",
              "minsr_step"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_symbol_list_matches_header():
    import paper_2608_18065_amd as pm
    assert sorted(pm.SYMBOLS) == declared_symbols()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_errors_without_device_calls():
    import paper_2608_18065_amd as pm
    lib = pm.lib()
    # invalid descriptors are rejected on the host before any device work
    d = pm.ModelDesc(10, 1, 3, 16, 0, 0, 0, pm.F64, 1, 64, 0)
    h = ctypes.c_void_p()
    rc = lib.minsr_create_model(ctypes.byref(d), ctypes.byref(h))
    assert rc == -1
    assert b"dim" in lib.minsr_last_error()
    d = pm.ModelDesc(10, 1, 1, 48, 0, 0, 0, pm.F64, 1, 64, 0)
    assert lib.minsr_create_model(ctypes.byref(d), ctypes.byref(h)) == -6
    assert lib.minsr_destroy_model(None) == -1
