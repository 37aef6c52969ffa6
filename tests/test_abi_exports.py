"""The C-ABI library loads on the CPU and exports every entry point of include/osa.h."""
import ctypes
import os
import re

import pytest

import paper_0710_0341_amd as osa

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "osa.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^OSA_API\s+[\w\s\*]*?\b(\w+)\s*\(", text, re.M)))


def test_header_declares_entry_points():
    names = declared_symbols()
    assert "overlap_sign_apply" in names and "osa_apply" in names
    assert set(names) == set(osa.EXPORTS)


def test_library_exports_every_symbol():
    if not os.path.exists(osa.LIB_PATH):
        pytest.fail("libosa.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(osa.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_status_strings_without_gpu():
    lib = osa.lib()
    assert lib.osa_version().startswith(b"osa")
    for s in range(-8, 2):
        assert len(lib.osa_status_string(s)) > 0


def test_argument_errors_before_device_work():
    """Invalid arguments are rejected before any device call (works without a GPU)."""
    lib = osa.lib()
    lat = osa.Lattice()
    for i in range(4):
        lat.dims[i] = 4
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(1)
    # m_w outside (-2, 0)
    assert lib.osa_create(ctypes.byref(h), ctypes.byref(lat), dummy, 0, 0.3, 0.5, None, None) == -1
    assert lib.osa_create(ctypes.byref(h), ctypes.byref(lat), dummy, 0, 0.3, -2.0, None, None) == -1
    # extent < 2
    lat.dims[2] = 1
    assert lib.osa_create(ctypes.byref(h), ctypes.byref(lat), dummy, 0, 0.3, -1.5, None, None) == -1
    lat.dims[2] = 4
    # null links, bad precision
    assert lib.osa_create(ctypes.byref(h), ctypes.byref(lat), None, 0, 0.3, -1.5, None, None) == -1
    assert lib.osa_create(ctypes.byref(h), ctypes.byref(lat), dummy, 7, 0.3, -1.5, None, None) == -1
    # one-shot: tol <= 0, aliasing source/result, negative n_defl
    est = ctypes.c_double()
    assert lib.overlap_sign_apply(ctypes.byref(lat), dummy, 0, 0.3, -1.5, dummy, 0.0, 0,
                                  ctypes.c_void_p(2), ctypes.byref(est), None) == -1
    assert lib.overlap_sign_apply(ctypes.byref(lat), dummy, 0, 0.3, -1.5, dummy, 1e-8, 0,
                                  dummy, ctypes.byref(est), None) == -1
    assert lib.overlap_sign_apply(ctypes.byref(lat), dummy, 0, 0.3, -1.5, dummy, 1e-8, -3,
                                  ctypes.c_void_p(2), ctypes.byref(est), None) == -1
    # small sign: k < 1
    assert lib.osa_small_sign(0, dummy, dummy, None, None) == -1
    # null context
    assert lib.osa_apply(None, 1, dummy, dummy, 1e-8, None) == -1
    assert lib.osa_deflate(None, 4, None) == -1


def test_allocator_hook_arguments():
    """osa_set_allocator: exactly one null function is an argument error; both
    null (the default, hipMalloc) is accepted.  No device work on either path."""
    L = osa.lib()
    alloc = osa.ALLOC_FN(lambda n, s, u: None)
    assert L.osa_set_allocator(alloc, osa.DEALLOC_FN(), None) == -1
    assert L.osa_set_allocator(osa.ALLOC_FN(), osa.DEALLOC_FN(lambda p, s, u: None), None) == -1
    assert L.osa_set_allocator(osa.ALLOC_FN(), osa.DEALLOC_FN(), None) == 0
