"""CPU checks of the boundary: libtft.so loads and exports every function that
include/libtft.h declares, and the Python binding lists the same names.  No
compute call is made (there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libtft.h")
LIB = os.path.join(ROOT, "paper_1001_5272_amd", "lib", "libtft.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\**\s+\**([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared()
    for must in ["tft_ctx_create", "tft_ctx_destroy", "tft_forward", "tft_inverse", "poly_mul", "tft_strerror"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libtft.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_1001_5272_amd import libtft
    assert sorted(libtft.SIGNATURES) == declared()


def test_strerror_without_device():
    lib = ctypes.CDLL(LIB)
    lib.tft_strerror.restype = ctypes.c_char_p
    lib.tft_strerror.argtypes = [ctypes.c_int]
    assert lib.tft_strerror(0) == b"ok"
    assert lib.tft_strerror(-2) == b"length or prime out of range"


def test_plan_bucket_without_device():
    # floor(4 lg n), exactly: the largest t with n^4 >= 2^t; a power of two
    # 2^k has the slot 4 * 28 + 4 + k of its own
    lib = ctypes.CDLL(LIB)
    lib.tft_plan_bucket.restype = ctypes.c_uint
    lib.tft_plan_bucket.argtypes = [ctypes.c_size_t]
    for n in [1, 2, 3, 4, 5, 7, 8, 9, 100003, (1 << 22) - 1, 1 << 22, (1 << 22) + 1, 3 << 21, 5931642, (1 << 28)]:
        if n & (n - 1) == 0:
            assert lib.tft_plan_bucket(n) == 4 * 28 + 4 + n.bit_length() - 1, n
            continue
        t = 0
        while n ** 4 >= 2 ** (t + 1):
            t += 1
        assert lib.tft_plan_bucket(n) == t, n


def test_argument_checks_without_device():
    # NULL arguments are rejected before any device call
    from paper_1001_5272_amd import libtft
    lib = ctypes.CDLL(LIB)
    lib.tft_batch_tuning_get.restype = ctypes.c_int
    lib.tft_batch_tuning_get.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    t = libtft.BatchTuning()
    assert lib.tft_batch_tuning_get(None, ctypes.byref(t)) == libtft.TFT_EINVAL
    lib.tft_calibrate.restype = ctypes.c_int
    lib.tft_calibrate.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.tft_calibrate(None, None) == libtft.TFT_EINVAL
