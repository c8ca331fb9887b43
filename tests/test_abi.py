"""The C-ABI library loads and exports every function include/vie.h declares (CPU only:
no compute call is made)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vie.h")
LIB = os.path.join(ROOT, "paper_1805_04791_amd", "libvie.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vie_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_four_core_calls():
    names = declared_functions()
    for core in ("vie_plan_create", "vie_apply", "vie_solve", "vie_destroy"):
        assert core in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvie.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvie.so not built")
def test_host_only_calls():
    from paper_1805_04791_amd import vie
    L = vie.load_library()
    assert L.vie_status_string(0) == b"VIE_OK"
    assert L.vie_status_string(-2).startswith(b"VIE_E_SIZE")
    assert L.vie_supported_n(128) == 1
    assert L.vie_supported_n(7) == 0
    assert L.vie_destroy(None) == 0
    assert L.vie_apply_noalloc(None, None, None, 1, 0, None) == vie.E_ARG
    # invalid problems are rejected before any device work
    p = vie.Problem()
    p.kind, p.n, p.h, p.omega, p.coef, p.precision, p.max_rhs = 1, 7, 0.1, 1.0, None, 0, 1
    h = ctypes.c_void_p()
    assert L.vie_plan_create(ctypes.byref(p), None, ctypes.byref(h)) == vie.E_ARG   # coef NULL
    p.coef = 1  # never dereferenced: the size check comes first
    assert L.vie_plan_create(ctypes.byref(p), None, ctypes.byref(h)) == vie.E_SIZE
    p.n, p.omega = 16, 0.0
    assert L.vie_plan_create(ctypes.byref(p), None, ctypes.byref(h)) == vie.E_ARG   # Helmholtz needs omega > 0
    assert not h.value
