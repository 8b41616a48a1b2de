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
}
