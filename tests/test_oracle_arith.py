"""Pins for the oracle's ring arithmetic and roots (section 2.1 and 2.2).

Everything here is checked against Python's own integers (an independent
big-integer implementation), against the table of roots printed in
section 2.2, or against the identities stated there.
"""
import random

import pytest

import oracle
from conftest import PRIMES


def factor(n):
    out, d = set(), 2
    while d * d <= n:
        while n % d == 0:
            out.add(d)
            n //= d
        d += 1
    if n > 1:
        out.add(n)
    return out


@pytest.mark.parametrize("name", list(PRIMES))
def test_mulmod_matches_python(name):
    p, _ = PRIMES[name]
    rng = random.Random(7)
    edge = [0, 1, 2, p - 1, p - 2, (p - 1) // 2, (p + 1) // 2]
    vals = edge + [rng.randrange(p) for _ in range(200)]
    for a in vals:
        b = rng.choice(vals)
        assert oracle.mulmod(a, b, p) == a * b % p
        assert oracle.addmod(a, b, p) == (a + b) % p
        assert oracle.submod(a, b, p) == (a - b) % p
        if a:
            assert oracle.invmod(a, p) == pow(a, -1, p)
    for _ in range(50):
        a, e = rng.randrange(p), rng.randrange(2**63)
        assert oracle.powmod(a, e, p) == pow(a, e, p)


@pytest.mark.parametrize("name", list(PRIMES))
def test_generator_and_root_chain(name):
    p, g = PRIMES[name]
    v = oracle.two_adic(p)
    assert (p - 1) % (1 << v) == 0 and ((p - 1) >> v) % 2 == 1
    # g generates (Z/pZ)^*: g^((p-1)/q) != 1 for every prime q | p-1
    for q in factor(p - 1):
        assert pow(g, (p - 1) // q, p) != 1
    chain = [oracle.root_chain(p, g, j) for j in range(v + 1)]
    assert chain[0] == 1
    assert chain[1] == p - 1                       # w[1] = -1 (section 2.2 table)
    for j in range(v):
        assert chain[j + 1] * chain[j + 1] % p == chain[j]   # compatibility
    # w[v] has order exactly 2^v
    assert pow(chain[v], 1 << (v - 1), p) == p - 1
    for j in range(v + 1):
        assert chain[j] == pow(g, (p - 1) >> j, p)


def test_known_root_values():
    # closed forms: in Z/(2^64-2^32+1), 2^96 = -1, so the 4th roots of unity are +-2^48
    P = 2**64 - 2**32 + 1
    w2 = oracle.root_chain(P, 7, 2)
    assert w2 in (2**48, P - 2**48)
    assert w2 * w2 % P == P - 1
    # 998244353 - 1 = 2^23 * 7 * 17
    assert oracle.two_adic(998244353) == 23
    assert oracle.two_adic(P) == 32
    assert oracle.two_adic(1811939329) == 26
    assert oracle.two_adic(2013265921) == 27
    assert oracle.two_adic(469762049) == 26


def test_bit_reversal():
    for k in range(0, 12):
        seen = set()
        for s in range(1 << k):
            r = oracle.rev(s, k)
            assert r == int(format(s, "0%db" % k)[::-1] or "0", 2) if k else r == 0
            seen.add(r)
        assert seen == set(range(1 << k))


@pytest.mark.parametrize("name", ["p17", "p257", "p998244353", "goldilocks"])
def test_omega_table_of_section_2_2(name):
    p, g = PRIMES[name]
    w = lambda k: oracle.root_chain(p, g, k)  # noqa: E731
    # the printed table: w_0 = w[0], w_1 = w[1], w_2 = w[2], w_3 = w[2]^3,
    # w_4 = w[3], w_5 = w[3]^5, w_6 = w[3]^3, w_7 = w[3]^7
    expect = [1, w(1), w(2), pow(w(2), 3, p), w(3), pow(w(3), 5, p), pow(w(3), 3, p), pow(w(3), 7, p)]
    assert [oracle.omega(p, g, s) for s in range(8)] == expect
    assert expect[1] == p - 1


@pytest.mark.parametrize("name", ["p17", "p12289", "p998244353", "goldilocks"])
def test_omega_identities_and_compatibility(name):
    p, g = PRIMES[name]
    v = oracle.two_adic(p)
    S = min(1 << v, 4096)
    om = oracle.omega_table(p, g, S)
    for s in range(S // 2):
        assert int(om[2 * s + 1]) == (p - int(om[2 * s])) % p          # w_{2s+1} = -w_{2s}
        assert int(om[2 * s]) ** 2 % p == int(om[s])                      # w_{2s}^2 = w_s
        assert int(om[2 * s + 1]) ** 2 % p == int(om[s])
    # independence of k (compatible choice): same w_s for every k >= bitlen(s)
    rng = random.Random(3)
    for s in [0, 1, 2, 3, 5, 100, S - 1] + [rng.randrange(S) for _ in range(20)]:
        for k in range(max(1, s.bit_length()), min(v, s.bit_length() + 4) + 1):
            assert oracle.omega_k(p, g, s, k) == int(om[s])


@pytest.mark.parametrize("name", ["p17", "p257", "p7681"])
def test_omega_set_is_all_roots(name):
    # {w_s : s < 2^k} is exactly the set of 2^k-th roots of unity (Python pow)
    p, g = PRIMES[name]
    v = oracle.two_adic(p)
    for k in range(0, v + 1):
        N = 1 << k
        roots = {x for x in range(1, p) if pow(x, N, p) == 1}
        got = [int(x) for x in oracle.omega_table(p, g, N)]
        assert len(set(got)) == N and set(got) == roots


def test_golden_roots():
    import json
    import os
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tft_p17.json")))
    assert [oracle.root_chain(17, 3, j) for j in range(5)] == d["root_chain"]
    assert [oracle.omega(17, 3, s) for s in range(16)] == d["omega"]
