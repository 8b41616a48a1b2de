"""Pins for the oracle's transforms.

- tft_direct (definition F^_s = F(w_s), section 2.2) is checked against the
  hand-computed fixtures in tests/golden, monomial inputs evaluated with
  Python integers, the DFT closed forms at n = 2^k, the convolution theorem
  with numpy.convolve, and the zero-padded DFT prefix property (section 1.2).
- fft_padded (separately coded textbook FFT) must agree with tft_direct.
- itft_lagrange (unique interpolant, section 4) must invert tft_direct both
  ways and, at n = 2^k, agree with the closed-form inverse DFT.
- tft_paper / itft_paper (Algorithms 1 and 2 in recursive form) must agree
  with the definition; the tree they walk is pinned to Figure 1.
- tft_inplace / itft_inplace (the same algorithms with O(1) auxiliary space:
  roots on the fly, a stackless walk) must agree with the definition and
  invert each other.
"""
import json
import os
import random

import numpy as np
import pytest

import oracle
from conftest import PRIMES

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tft_p17.json")))


def rnd(p, n, seed):
    rng = random.Random(seed)
    return np.array([rng.randrange(p) for _ in range(n)], dtype=np.uint64)


def py_omega(p, g, s):
    k = s.bit_length()
    r = int(format(s, "0%db" % k)[::-1], 2) if k else 0
    return pow(pow(g, (p - 1) >> k, p), r, p)


def test_golden_cases():
    for c in GOLD["cases"]:
        X = oracle.tft_direct(17, 3, c["F"])
        assert [int(x) for x in X] == c["X"], c["name"]
        assert [int(x) for x in oracle.fft_padded(17, 3, c["F"])] == c["X"]
        assert [int(x) for x in oracle.tft_paper(17, 3, c["F"])] == c["X"]
        assert [int(x) for x in oracle.itft_lagrange(17, 3, c["X"])] == c["F"]
        assert [int(x) for x in oracle.itft_paper(17, 3, c["X"])] == c["F"]
        assert [int(x) for x in oracle.tft_inplace(17, 3, c["F"])] == c["X"]
        assert [int(x) for x in oracle.itft_inplace(17, 3, c["X"])] == c["F"]


@pytest.mark.parametrize("name", ["p17", "p998244353", "goldilocks", "p63"])
def test_monomials(name):
    p, g = PRIMES[name]
    n = 13 if p > 17 else 9
    for t in range(n):
        e = np.zeros(n, dtype=np.uint64)
        e[t] = 1
        X = oracle.tft_direct(p, g, e)
        assert [int(x) for x in X] == [pow(py_omega(p, g, s), t, p) for s in range(n)]


@pytest.mark.parametrize("name", ["p17", "p257", "p998244353", "goldilocks", "p63"])
def test_closed_form_inverse_dft_at_power_of_two(name):
    # n = N = 2^k: sum_s X_s w_s^(-t) = N F_t (orthogonality of N-th roots)
    p, g = PRIMES[name]
    for k in range(0, 5):
        N = 1 << k
        F = rnd(p, N, 11 + k)
        X = [int(x) for x in oracle.tft_direct(p, g, F)]
        for t in range(N):
            acc = sum(X[s] * pow(py_omega(p, g, s), (-t) % (p - 1), p) for s in range(N)) % p
            assert acc == N * int(F[t]) % p


@pytest.mark.parametrize("name", ["p257", "p12289", "p998244353"])
def test_convolution_theorem_against_numpy(name):
    # evaluation is a ring homomorphism: TFT(A) * TFT(B) = TFT(A B) when
    # deg(A B) < n; A B comes from numpy.convolve on small integer values
    p, g = PRIMES[name]
    rng = np.random.default_rng(5)
    for n in [1, 2, 3, 7, 16, 33, 100]:
        la = rng.integers(1, n + 1)
        lb = n + 1 - la if n + 1 - la >= 1 else 1
        A = rng.integers(0, 200, la)
        B = rng.integers(0, 200, lb)
        C = np.convolve(A, B) % p            # exact in int64 for these sizes
        pad = lambda v: np.concatenate([v, np.zeros(n - len(v), dtype=np.int64)]).astype(np.uint64)  # noqa
        XA, XB, XC = (oracle.tft_direct(p, g, pad(v)) for v in (A, B, C))
        assert [int(a) * int(b) % p for a, b in zip(XA, XB)] == [int(c) for c in XC]


@pytest.mark.parametrize("name", ["p17", "p12289", "p998244353", "goldilocks"])
def test_direct_equals_padded_prefix(name):
    # section 1.2: the TFT is the first n outputs of the zero-padded length-2^k DFT
    p, g = PRIMES[name]
    v = oracle.two_adic(p)
    ns = [n for n in range(1, 301) if (n - 1).bit_length() <= v]
    for n in ns:
        F = rnd(p, n, n)
        X = oracle.tft_direct(p, g, F)
        assert (oracle.fft_padded(p, g, F) == X).all(), n
    # compatibility: padding further (larger k) changes nothing
    for n in [1, 5, 6, 100, 129]:
        if (n - 1).bit_length() + 3 <= v:
            F = rnd(p, n, 99 + n)
            X = oracle.tft_direct(p, g, F)
            for extra in range(1, 4):
                assert (oracle.fft_padded(p, g, F, kmin=(n - 1).bit_length() + extra) == X).all()


def test_exhaustive_bijection_p17():
    # every input for n <= 3 over Z/17: the TFT is a bijection and the
    # interpolation inverts it exactly
    p, g = 17, 3
    for n in [1, 2, 3]:
        seen = set()
        for code in range(p ** n):
            F = [(code // p ** i) % p for i in range(n)]
            X = tuple(int(x) for x in oracle.tft_direct(p, g, F))
            seen.add(X)
            if code % 7 == 0:
                assert [int(x) for x in oracle.itft_lagrange(p, g, list(X))] == F
        assert len(seen) == p ** n


@pytest.mark.parametrize("name", ["p17", "p12289", "p998244353", "goldilocks"])
def test_itft_round_trips(name):
    p, g = PRIMES[name]
    v = oracle.two_adic(p)
    for n in [1, 2, 3, 4, 5, 6, 7, 8, 9, 15, 16, 17, 31, 64, 65, 100]:
        if (n - 1).bit_length() > v:
            continue
        F = rnd(p, n, 1000 + n)
        X = oracle.tft_direct(p, g, F)
        assert (oracle.itft_lagrange(p, g, X) == F).all()
        Y = rnd(p, n, 2000 + n)
        assert (oracle.tft_direct(p, g, oracle.itft_lagrange(p, g, Y)) == Y).all()
        if n & (n - 1) == 0:
            assert (oracle.ifft_pow2(p, g, X) == F).all()


def test_figure1_tree():
    # node (q, r) of the n = 6 tree is the strided subarray X_{q + i 2^r},
    # of length ceil((n - q) / 2^r), as drawn in Figure 1
    n = 6
    for q, r, members in GOLD["figure1_n6_nodes"]["nodes"]:
        L = oracle.node_len(n, q, r)
        assert [q + i * (1 << r) for i in range(L)] == members


@pytest.mark.parametrize("name", ["p17", "p12289", "p998244353", "goldilocks"])
def test_paper_algorithms_match_definition(name):
    p, g = PRIMES[name]
    v = oracle.two_adic(p)
    rng = random.Random(17)
    ns = list(range(1, 130)) + [rng.randrange(130, 2000) for _ in range(8)]
    for n in ns:
        if (n - 1).bit_length() > v:
            continue
        F = rnd(p, n, 3 * n + 1)
        X = oracle.tft_direct(p, g, F) if n <= 700 else oracle.fft_padded(p, g, F)
        assert (oracle.tft_paper(p, g, F) == X).all(), n
        assert (oracle.itft_paper(p, g, X) == F).all(), n
        assert (oracle.tft_inplace(p, g, F) == X).all(), n
        assert (oracle.itft_inplace(p, g, X) == F).all(), n


@pytest.mark.parametrize("name", ["p257", "p7681", "p998244353", "goldilocks"])
def test_inplace_algorithms_every_length(name):
    """Every length up to 300 (or 2^v): the O(1)-space walks equal the
    definition F^_s = F(w_s) and invert each other."""
    p, g = PRIMES[name]
    v = oracle.two_adic(p)
    for n in range(1, min(300, 1 << v) + 1):
        F = rnd(p, n, 11 * n + 5)
        X = oracle.tft_direct(p, g, F)
        assert (oracle.tft_inplace(p, g, F) == X).all(), n
        assert (oracle.itft_inplace(p, g, X) == F).all(), n


def test_paper_operation_counts():
    # closed forms for power-of-two n: (n/2) lg n butterflies and no corrections
    for k in range(0, 14):
        b, c = oracle.paper_counts(1 << k)
        assert b == (1 << k) // 2 * k and c == 0
    # n = 2^k + 1: the root (m odd) has 2^(k-1) butterflies, its odd child is
    # a full 2^(k-1) transform and its even child is the case k-1, which sums
    # to k 2^(k-1) + 1 butterflies
    for k in range(1, 14):
        b, _ = oracle.paper_counts((1 << k) + 1)
        assert b == k * (1 << (k - 1)) + 1


# Operation counts of Algorithm 1 (section 3), derived by hand from the tree
# of section 3 (node (q, r) = the strided subarray X_{q + i 2^r}, length
# m = ceil((n - q) / 2^r), even child (q, r+1), odd child (q + 2^r, r+1)).  A
# node of length m >= 2 does floor(m / 2) butterflies (eq. 1); a node of odd
# length m >= 3 does the odd-length correction v = sum_{i <= (m-3)/2}
# S_{2i+1} w_{(m-1)/2}^i, S_{m-1} += v w_{m-1}, counted as one mulmod per term
# of the sum ((m-1)/2 terms) plus the final multiply by w_{m-1}.
#
# n = 3: root (0,0) m=3: 1 butterfly, correction 1+1 = 2; (0,1) m=2: 1
#        butterfly; (1,1) m=1.                      -> 2 butterflies, 2 mulmods
# n = 5: root m=5: 2 bf, corr 2+1 = 3; (0,1) m=3: 1 bf, corr 2; (0,2) m=2: 1 bf;
#        (2,2) m=1; (1,1) m=2: 1 bf.               -> 5 butterflies, 5 mulmods
# n = 6 (the tree of Figure 1): root m=6: 3 bf; (0,1) = {X0,X2,X4} m=3: 1 bf,
#        corr 2; (0,2) = {X0,X4} m=2: 1 bf; (2,2) = {X2} leaf; (1,1) =
#        {X1,X3,X5} m=3: 1 bf, corr 2; (1,2) = {X1,X5} m=2: 1 bf; (3,2) = {X3}
#        leaf.                                     -> 7 butterflies, 4 mulmods
# n = 7: root m=7: 3 bf, corr 3+1 = 4; (0,1) m=4: 2 bf; (0,2) m=2: 1 bf;
#        (2,2) m=2: 1 bf; (1,1) m=3: 1 bf, corr 2; (1,2) m=2: 1 bf; (3,2) m=1.
#                                                  -> 9 butterflies, 6 mulmods
HAND_COUNTS = {3: (2, 2), 5: (5, 5), 6: (7, 4), 7: (9, 6)}


def test_paper_operation_counts_by_hand():
    for n, (bf, corr) in HAND_COUNTS.items():
        assert oracle.paper_counts(n) == (bf, corr), n


def test_paper_butterflies_closed_form():
    # Every position x < n sits, at tree depth r >= 1, in an odd child exactly
    # when bit r-1 of x is set (odd children at depth r are the nodes
    # (q, r) with 2^(r-1) <= q < 2^r), and a node's butterflies are the length
    # of its odd child (floor(m / 2) = ceil((n - q - 2^r) / 2^(r+1))).  So the
    # butterflies of Algorithm 1 number sum_{x < n} popcount(x) for every n;
    # this gives 13,646 at n = 2499.
    for n in list(range(1, 300)) + [2499, 4097, 12345]:
        b, _ = oracle.paper_counts(n)
        assert b == sum(bin(x).count("1") for x in range(n)), n
    assert oracle.paper_counts(2499)[0] == 13646


def test_sample_and_eval():
    p, g = PRIMES["goldilocks"]
    F = rnd(p, 1000, 4)
    X = oracle.tft_direct(p, g, F)
    idx = [0, 1, 2, 511, 999]
    assert [int(x) for x in oracle.tft_sample(p, g, F, idx)] == [int(X[i]) for i in idx]
    z = 123456789
    assert oracle.evaluate(p, F, z) == sum(int(f) * pow(z, t, p) for t, f in enumerate(F)) % p


def test_rejects_bad_lengths():
    with pytest.raises(ValueError):
        oracle.tft_direct(17, 3, [])
    with pytest.raises(ValueError):
        oracle.tft_direct(17, 3, list(range(17)))   # needs a 32nd root; v2(16) = 4
