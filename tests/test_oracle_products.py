"""Pins for the oracle's products (section 5: the product C = A B is unique)
and for the exact integer product behind the three-prime CRT path.

Schoolbook and padded products are checked against numpy.convolve on small
values (exact in int64) and against each other; the exact signed product is
checked against Python's integers.
"""
import random

import numpy as np
import pytest

import oracle
from conftest import PRIMES


@pytest.mark.parametrize("name", ["p17", "p998244353", "goldilocks"])
def test_schoolbook_against_numpy(name):
    p, g = PRIMES[name]
    rng = np.random.default_rng(1)
    for m, nb in [(1, 1), (1, 5), (5, 1), (7, 9), (64, 3), (100, 100)]:
        A = rng.integers(0, min(p, 1000), m)
        B = rng.integers(0, min(p, 1000), nb)
        ref = [int(c) % p for c in np.convolve(A, B)]
        assert [int(c) for c in oracle.mul_schoolbook(p, A, B)] == ref
        if (m + nb - 2).bit_length() <= oracle.two_adic(p):
            assert [int(c) for c in oracle.mul_padded(p, g, A, B)] == ref
        for s in [0, m + nb - 2, (m + nb - 1) // 2]:
            assert oracle.mul_coeff(p, A, B, s) == ref[s]


@pytest.mark.parametrize("name", ["p998244353", "goldilocks", "p1811939329", "p63"])
def test_padded_product_against_schoolbook_full_range(name):
    p, g = PRIMES[name]
    rng = random.Random(2)
    for m, nb in [(1000, 1500), (33, 1), (1, 64), (129, 128), (300, 211)]:
        A = np.array([rng.randrange(p) for _ in range(m)], dtype=np.uint64)
        B = np.array([rng.randrange(p) for _ in range(nb)], dtype=np.uint64)
        C = oracle.mul_schoolbook(p, A, B)
        assert (oracle.mul_padded(p, g, A, B) == C).all()
        # evaluation identity C(z) = A(z) B(z)
        z = rng.randrange(p)
        assert oracle.evaluate(p, C, z) == oracle.evaluate(p, A, z) * oracle.evaluate(p, B, z) % p


def test_product_through_tft_and_interpolation():
    # TFT both operands in r slots, multiply pointwise, interpolate: the
    # product of section 5 (without its memory restriction)
    p, g = PRIMES["p998244353"]
    rng = random.Random(9)
    for m, nb in [(1, 1), (3, 4), (10, 7), (40, 25)]:
        r = m + nb - 1
        A = [rng.randrange(p) for _ in range(m)] + [0] * (r - m)
        B = [rng.randrange(p) for _ in range(nb)] + [0] * (r - nb)
        XA, XB = oracle.tft_direct(p, g, A), oracle.tft_direct(p, g, B)
        XC = [int(a) * int(b) % p for a, b in zip(XA, XB)]
        assert (oracle.itft_lagrange(p, g, XC) == oracle.mul_schoolbook(p, A[:m], B[:nb])).all()


@pytest.mark.parametrize("name", ["p257", "p998244353", "goldilocks"])
def test_space_restricted_product(name):
    """Algorithm 3 (section 5) gives the unique product: against the schoolbook
    product for every shape up to 24 x 24 (r = 1 .. 47: one to several
    blocks, r a power of two and one either side), against numpy.convolve on
    small values, and against the padded product at larger r."""
    p, g = PRIMES[name]
    rng = random.Random(31)
    for m in range(1, 25):
        for nb in range(1, 25):
            if (m + nb - 2).bit_length() > oracle.two_adic(p):
                continue
            A = np.array([rng.randrange(p) for _ in range(m)], dtype=np.uint64)
            B = np.array([rng.randrange(p) for _ in range(nb)], dtype=np.uint64)
            assert (oracle.mul_restricted(p, g, A, B) == oracle.mul_schoolbook(p, A, B)).all(), (m, nb)
    A, B = np.arange(1, 40), np.arange(7, 20)
    assert [int(c) for c in oracle.mul_restricted(p, g, A, B)] == [int(x) % p for x in np.convolve(A, B)]
    if p > 2**20:
        for m, nb in [(1000, 1500), (4096, 4097), (3000, 1)]:
            A = np.array([rng.randrange(p) for _ in range(m)], dtype=np.uint64)
            B = np.array([rng.randrange(p) for _ in range(nb)], dtype=np.uint64)
            assert (oracle.mul_restricted(p, g, A, B) == oracle.mul_padded(p, g, A, B)).all(), (m, nb)


def test_exact_signed_product_against_python():
    rng = random.Random(4)
    for m, nb in [(1, 1), (5, 3), (64, 64), (200, 17)]:
        a = [rng.randrange(-2**23, 2**23) for _ in range(m)]
        b = [rng.randrange(-2**23, 2**23) for _ in range(nb)]
        ref = [0] * (m + nb - 1)
        for i, x in enumerate(a):
            for j, y in enumerate(b):
                ref[i + j] += x * y
        assert oracle.conv_i128(a, b) == ref
        for s in [0, m + nb - 2, (m + nb) // 2 - 1]:
            assert oracle.conv_coeff_i128(a, b, s) == ref[s]
    # values beyond 64 bits
    a = [2**62 - 1] * 8
    b = [-(2**62) + 3] * 8
    ref = [(min(s, 7) - max(0, s - 7) + 1) * (2**62 - 1) * (-(2**62) + 3) for s in range(15)]
    assert oracle.conv_i128(a, b) == ref


def test_bad_arguments():
    with pytest.raises(ValueError):
        oracle.mul_schoolbook(17, [], [1])
    with pytest.raises(ValueError):
        oracle.mul_padded(17, 3, list(range(10)), list(range(10)))  # r = 19 > 2^4
