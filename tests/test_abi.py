"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the header declares, and rejects bad arguments before touching
the device."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "krylov_kernel.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:kk_status|const char \*)\s*(\w+)\s*\(", text)))


def test_header_declares_the_three_entry_points():
    names = declared_functions()
    for n in ("krylov_kernel_apply", "density_response_batch", "mulliken_project"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2303_03529_amd import krylov
    lib = ctypes.CDLL(krylov.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(krylov.SIGNATURES)


def test_argument_validation_without_device():
    from paper_2303_03529_amd import krylov
    L = krylov.LIB
    assert L.kk_create(None, None) == krylov.KK_EINVAL
    h = ctypes.c_void_p()
    assert L.kk_create(ctypes.byref(h), None) == krylov.KK_OK
    try:
        # every entry point refuses an unprepared handle
        assert L.density_response_batch(h, 1, ctypes.c_void_p(8), ctypes.c_void_p(8)) == krylov.KK_ENOTPREPARED
        assert L.mulliken_project(h, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8)) \
            == krylov.KK_ENOTPREPARED
        assert L.krylov_kernel_apply(h, ctypes.c_void_p(8), 4, None, ctypes.c_void_p(8), None) \
            == krylov.KK_ENOTPREPARED
        assert "kk_prepare" in krylov.last_error()
        assert L.krylov_kernel_adjoint(h, p8 := ctypes.c_void_p(8), 4, None, p8, 0, None, p8, p8, p8, p8, p8,
                                       None) == krylov.KK_ENOTPREPARED
        assert L.krylov_kernel_apply_adaptive(h, p8, 4, 0.1, None, p8, None) == krylov.KK_ENOTPREPARED
        assert L.kk_ground_state_charges(h, None, p8) == krylov.KK_ENOTPREPARED
        assert L.kk_xlbomd_update(h, p8, 1, p8, 1.0, 0.0, p8, p8) == krylov.KK_ENOTPREPARED
        off = np.array([0, 9, 18], dtype=np.int32)
        p = ctypes.c_void_p(8)
        args = [p] * 6
        # bad offsets, kT, electron count, precision, NULL arrays
        bad = np.array([0, 9, 9], dtype=np.int32)
        assert L.kk_prepare(h, 2, bad.ctypes.data_as(ctypes.c_void_p), 9, *([p] * 7), -0.4, 0.25, 16.0, 0) \
            == krylov.KK_EINVAL
        assert L.kk_prepare(h, 2, off.ctypes.data_as(ctypes.c_void_p), 18, *([p] * 7), -0.4, 0.0, 16.0, 0) \
            == krylov.KK_EINVAL
        assert L.kk_prepare(h, 2, off.ctypes.data_as(ctypes.c_void_p), 18, *([p] * 7), -0.4, 0.25, 36.0, 0) \
            == krylov.KK_EINVAL
        assert L.kk_prepare(h, 2, off.ctypes.data_as(ctypes.c_void_p), 18, *([p] * 7), -0.4, 0.25, 16.0, 7) \
            == krylov.KK_EINVAL
        assert L.kk_prepare(h, 2, off.ctypes.data_as(ctypes.c_void_p), 18, None, *args, -0.4, 0.25, 16.0, 0) \
            == krylov.KK_EINVAL
        assert "NULL" in krylov.last_error()
        assert L.kk_get_mu(h, None) == krylov.KK_ENOTPREPARED
    finally:
        assert L.kk_destroy(h) == krylov.KK_OK
    assert L.kk_destroy(None) == krylov.KK_EINVAL


def test_product_package_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2303_03529_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, flags=re.M), f
                assert "oracle/" not in text, f
