import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


# (p, g) pairs used throughout: the NTT primes of the workloads plus small
# primes for exhaustive checks.  g is the generator that fixes the roots.
PRIMES = {
    "p17": (17, 3),
    "p257": (257, 3),
    "p7681": (7681, 17),
    "p12289": (12289, 11),
    "p998244353": (998244353, 3),
    "p469762049": (469762049, 3),
    "p2013265921": (2013265921, 31),
    "p1811939329": (1811939329, 13),
    "goldilocks": (2**64 - 2**32 + 1, 7),
    # other primes of 8-byte words (64-bit Montgomery arithmetic): just below
    # 2^63 with 2-adic order 32, and a 62-bit one of order 35
    "p63": (9223372006790004737, 3),
    "p62": (2478761244408938497, 5),
}
