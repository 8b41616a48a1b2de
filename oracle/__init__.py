"""ORACLE — test infrastructure only.

ctypes wrapper around ``oracle/tft_oracle.c``, the plain CPU reference for the
in-place truncated Fourier transform of Harvey & Roche (2010) and the
polynomial products built on it.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package; the GPU
product path (``paper_1001_5272_amd``) never does, and this package imports
nothing from it.

Every array is passed as a contiguous ``numpy.uint64`` vector of residues
(signed int64 for the exact integer product).  Functions raise ``ValueError``
when the C routine reports a bad argument.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
(hand-computed fixtures in ``tests/golden/``, closed forms, library routines
and brute force); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tft_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_u64 = ctypes.c_uint64
_P = ctypes.POINTER(ctypes.c_uint64)
_PI = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no vectorisation
    assumptions); returns the library path."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                        "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        sig = {
            "or_mulmod": (_u64, [_u64, _u64, _u64]),
            "or_addmod": (_u64, [_u64, _u64, _u64]),
            "or_submod": (_u64, [_u64, _u64, _u64]),
            "or_powmod": (_u64, [_u64, _u64, _u64]),
            "or_invmod": (_u64, [_u64, _u64]),
            "or_two_adic": (ctypes.c_uint, [_u64]),
            "or_root_chain": (_u64, [_u64, _u64, ctypes.c_uint]),
            "or_rev": (_u64, [_u64, ctypes.c_uint]),
            "or_bitlen": (ctypes.c_uint, [_u64]),
            "or_omega": (_u64, [_u64, _u64, _u64]),
            "or_omega_k": (_u64, [_u64, _u64, _u64, ctypes.c_uint]),
            "or_omega_table": (ctypes.c_int, [_u64, _u64, _u64, _P]),
            "or_eval": (_u64, [_u64, _P, _u64, _u64]),
            "or_tft_direct": (ctypes.c_int, [_u64, _u64, _P, _u64, _P]),
            "or_tft_sample": (ctypes.c_int, [_u64, _u64, _P, _u64, _P, _u64, _P]),
            "or_itft_lagrange": (ctypes.c_int, [_u64, _u64, _P, _u64, _P]),
            "or_fft_padded": (ctypes.c_int, [_u64, _u64, _P, _u64, ctypes.c_uint, _P]),
            "or_ifft_pow2": (ctypes.c_int, [_u64, _u64, _P, _u64, _P]),
            "or_mul_schoolbook": (ctypes.c_int, [_u64, _P, _u64, _P, _u64, _P]),
            "or_mul_coeff": (_u64, [_u64, _P, _u64, _P, _u64, _u64]),
            "or_mul_padded": (ctypes.c_int, [_u64, _u64, _P, _u64, _P, _u64, _P]),
            "or_conv_i128": (ctypes.c_int, [_PI, _u64, _PI, _u64, _P]),
            "or_conv_coeff_i128": (ctypes.c_int, [_PI, _u64, _PI, _u64, _u64, _P]),
            "or_tft_paper": (ctypes.c_int, [_u64, _u64, _P, _u64]),
            "or_itft_paper": (ctypes.c_int, [_u64, _u64, _P, _u64]),
            "or_node_len": (_u64, [_u64, _u64, ctypes.c_uint]),
            "or_paper_counts": (ctypes.c_int, [_u64, _P, _P]),
            "or_tft_inplace": (ctypes.c_int, [_u64, _u64, _P, _u64]),
            "or_itft_inplace": (ctypes.c_int, [_u64, _u64, _P, _u64]),
            "or_mul_restricted": (ctypes.c_int, [_u64, _u64, _P, _u64, _P, _u64, _P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _vec(x) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.uint64))
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_P)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


# ---------------------------------------------------------------- scalars
def mulmod(a, b, p): return int(lib().or_mulmod(a, b, p))
def addmod(a, b, p): return int(lib().or_addmod(a, b, p))
def submod(a, b, p): return int(lib().or_submod(a, b, p))
def powmod(a, e, p): return int(lib().or_powmod(a, e, p))
def invmod(a, p): return int(lib().or_invmod(a, p))
def two_adic(p): return int(lib().or_two_adic(p))
def root_chain(p, g, j): return int(lib().or_root_chain(p, g, j))
def rev(s, k): return int(lib().or_rev(s, k))
def omega(p, g, s): return int(lib().or_omega(p, g, s))
def omega_k(p, g, s, k): return int(lib().or_omega_k(p, g, s, k))
def node_len(n, q, r): return int(lib().or_node_len(n, q, r))


def omega_table(p, g, n):
    out = np.zeros(n, dtype=np.uint64)
    _check(lib().or_omega_table(p, g, n, _ptr(out)), "omega_table")
    return out


def evaluate(p, F, z):
    F = _vec(F)
    return int(lib().or_eval(p, _ptr(F), len(F), z))


# ------------------------------------------------------------ transforms
def tft_direct(p, g, F):
    F = _vec(F)
    X = np.zeros_like(F)
    _check(lib().or_tft_direct(p, g, _ptr(F), len(F), _ptr(X)), "tft_direct")
    return X


def tft_sample(p, g, F, idx):
    F = _vec(F)
    idx = _vec(idx)
    X = np.zeros(len(idx), dtype=np.uint64)
    _check(lib().or_tft_sample(p, g, _ptr(F), len(F), _ptr(idx), len(idx), _ptr(X)), "tft_sample")
    return X


def itft_lagrange(p, g, Y):
    Y = _vec(Y)
    F = np.zeros_like(Y)
    _check(lib().or_itft_lagrange(p, g, _ptr(Y), len(Y), _ptr(F)), "itft_lagrange")
    return F


def fft_padded(p, g, F, kmin=0):
    F = _vec(F)
    X = np.zeros_like(F)
    _check(lib().or_fft_padded(p, g, _ptr(F), len(F), kmin, _ptr(X)), "fft_padded")
    return X


def ifft_pow2(p, g, X):
    X = _vec(X)
    F = np.zeros_like(X)
    _check(lib().or_ifft_pow2(p, g, _ptr(X), len(X), _ptr(F)), "ifft_pow2")
    return F


def tft_paper(p, g, F):
    X = _vec(F).copy()
    _check(lib().or_tft_paper(p, g, _ptr(X), len(X)), "tft_paper")
    return X


def itft_paper(p, g, Y):
    F = _vec(Y).copy()
    _check(lib().or_itft_paper(p, g, _ptr(F), len(F)), "itft_paper")
    return F


def tft_inplace(p, g, F):
    """Algorithm 1 with O(1) auxiliary space (no root table, no recursion)."""
    X = _vec(F).copy()
    _check(lib().or_tft_inplace(p, g, _ptr(X), len(X)), "tft_inplace")
    return X


def itft_inplace(p, g, Y):
    """Algorithm 2 with O(1) auxiliary space."""
    F = _vec(Y).copy()
    _check(lib().or_itft_inplace(p, g, _ptr(F), len(F)), "itft_inplace")
    return F


def mul_restricted(p, g, A, B):
    """Algorithm 3: the product written into its r-word output only."""
    A, B = _vec(A), _vec(B)
    X = np.zeros(len(A) + len(B) - 1, dtype=np.uint64)
    _check(lib().or_mul_restricted(p, g, _ptr(A), len(A), _ptr(B), len(B), _ptr(X)), "mul_restricted")
    return X


def paper_counts(n):
    b = np.zeros(1, dtype=np.uint64)
    c = np.zeros(1, dtype=np.uint64)
    _check(lib().or_paper_counts(n, _ptr(b), _ptr(c)), "paper_counts")
    return int(b[0]), int(c[0])


# --------------------------------------------------------------- products
def mul_schoolbook(p, A, B):
    A, B = _vec(A), _vec(B)
    C = np.zeros(len(A) + len(B) - 1, dtype=np.uint64)
    _check(lib().or_mul_schoolbook(p, _ptr(A), len(A), _ptr(B), len(B), _ptr(C)), "mul_schoolbook")
    return C


def mul_coeff(p, A, B, s):
    A, B = _vec(A), _vec(B)
    return int(lib().or_mul_coeff(p, _ptr(A), len(A), _ptr(B), len(B), s))


def mul_padded(p, g, A, B):
    A, B = _vec(A), _vec(B)
    C = np.zeros(len(A) + len(B) - 1, dtype=np.uint64)
    _check(lib().or_mul_padded(p, g, _ptr(A), len(A), _ptr(B), len(B), _ptr(C)), "mul_padded")
    return C


def _ivec(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64))


def _i128_from_lohi(lohi: np.ndarray):
    lo = lohi[0::2].astype(object)
    hi = lohi[1::2].astype(object)
    out = []
    for a, b in zip(lo, hi):
        v = (int(b) << 64) | int(a)
        if v >= 1 << 127:
            v -= 1 << 128
        out.append(v)
    return out


def conv_i128(a, b, as_lohi=False):
    """Exact signed product; returns Python ints (or the raw lo/hi pairs)."""
    a, b = _ivec(a), _ivec(b)
    r = len(a) + len(b) - 1
    out = np.zeros(2 * r, dtype=np.uint64)
    _check(lib().or_conv_i128(a.ctypes.data_as(_PI), len(a), b.ctypes.data_as(_PI), len(b), _ptr(out)),
           "conv_i128")
    return out if as_lohi else _i128_from_lohi(out)


def conv_coeff_i128(a, b, s):
    a, b = _ivec(a), _ivec(b)
    out = np.zeros(2, dtype=np.uint64)
    _check(lib().or_conv_coeff_i128(a.ctypes.data_as(_PI), len(a), b.ctypes.data_as(_PI), len(b), s,
                                    _ptr(out)), "conv_coeff_i128")
    return _i128_from_lohi(out)[0]
