"""GPU parity: libtft's forward/inverse TFT and product against the oracle,
element by element, bit-exact (all arithmetic is exact modulo p, so the
tolerance is zero).  Inputs are seeded uniform residues (synth)."""
import numpy as np
import pytest

import oracle
import synth
from conftest import PRIMES
from gpu_util import gpu_mul_restricted, gpu_forward, gpu_inverse, gpu_mul

pytestmark = pytest.mark.gpu

libtft = pytest.importorskip("paper_1001_5272_amd.libtft")


@pytest.fixture(scope="module")
def ctxs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    out = {name: libtft.Context(*PRIMES[name]) for name in
           ["p998244353", "goldilocks", "p63", "p62", "p12289", "p7681", "p2013265921", "p469762049",
            "p1811939329"]}
    yield out
    for c in out.values():
        c.close()


def check_roundtrip(ctx, p, g, n, seed, direct=False):
    F = synth.residues(p, n, seed)
    X = gpu_forward(ctx, F)
    ref = oracle.tft_direct(p, g, F) if direct else oracle.fft_padded(p, g, F)
    bad = np.nonzero(X != ref)[0]
    assert len(bad) == 0, f"p={p} n={n}: {len(bad)} forward mismatches, first at {bad[:5]}"
    back = gpu_inverse(ctx, X)
    bad = np.nonzero(back != F)[0]
    assert len(bad) == 0, f"p={p} n={n}: {len(bad)} inverse mismatches, first at {bad[:5]}"


@pytest.mark.parametrize("name", ["p998244353", "goldilocks", "p63"])
def test_every_small_length(ctxs, name):
    p, g = PRIMES[name]
    ctx = ctxs[name]
    print(f"[gpu] every n in 1..1100 for {name}", flush=True)
    for n in range(1, 1101):
        check_roundtrip(ctx, p, g, n, seed=n, direct=(n <= 64))


@pytest.mark.parametrize("name", ["p998244353", "goldilocks", "p63"])
def test_single_workgroup_sizes(ctxs, name):
    p, g = PRIMES[name]
    ctx = ctxs[name]
    for n in [1536, 2047, 2048, 2049, 2499, 3000, 4095, 4096, 6000, 8191, 8192]:
        print(f"[gpu] {name} n={n}", flush=True)
        check_roundtrip(ctx, p, g, n, seed=7 * n)


@pytest.mark.parametrize("name", ["p998244353", "goldilocks", "p63"])
@pytest.mark.parametrize("logW", [3, 4, 5, 6, 7])
def test_two_pass_forced_small(ctxs, name, logW):
    # the two-pass schedule at sizes the oracle handles quickly: many column
    # tiles, partial tiles and every kind of last row (b = 0, 1, W-1, other)
    p, g = PRIMES[name]
    ctx = ctxs[name]
    C = 16 if ctx.word_bytes == 4 else 8
    if (1 << logW) < C:
        pytest.skip("W below one column tile")
    libtft.tft_set_plan_override(ctx, logW)
    try:
        W = 1 << logW
        # includes the split columns (a = 2^k with b > 0, and a = 2^k + 1 with b = 0),
        # a + 1 = 2^k with b > 0 (two inverse column phases), and the general
        # last row (columns c < b completed by the rank-one update), also with b = 1
        ns = sorted({W + 1, 2 * W - 1, 2 * W, 3 * W + 1, 5 * W - 1, 17 * W, 17 * W + 3, 33 * W + W // 2,
                     100 * W + 7, 1000, 2499, 4097, 16 * W + 1, 16 * W + W - 1, 32 * W + 5, 65 * W, 129 * W,
                     64 * W + W // 2, 2 * W + 1, 3 * W, 5 * W + 1, 6 * W + 2, 11 * W + W - 1, 7 * W + 3,
                     9 * W + 5, 23 * W + 1, 15 * W + W // 3, 127 * W + 1,
                     # b = W - 1 with a + 1 a power of two (one short column)
                     4 * W - 1, 8 * W - 1, 64 * W - 1, 128 * W - 1})
        for n in ns:
            if n <= W:
                continue
            print(f"[gpu] {name} logW={logW} n={n}", flush=True)
            check_roundtrip(ctx, p, g, n, seed=n + 31 * logW)
    finally:
        libtft.tft_set_plan_override(ctx, 0)


@pytest.mark.parametrize("name", ["p998244353", "goldilocks", "p63"])
@pytest.mark.parametrize("logW", [8, 9, 10])
def test_two_pass_general_b_tiles(ctxs, name, logW):
    # general last rows with more than 128 columns c < b, so the columns run
    # as tiles (not one per workgroup) beside the last row's inverse; a + 1 is
    # not a power of two (the rank-one completion) or is (two column phases)
    p, g = PRIMES[name]
    ctx = ctxs[name]
    libtft.tft_set_plan_override(ctx, logW)
    try:
        W = 1 << logW
        # a in (H, 1.25 H] for a power of two H >= 64: the column inverse splits
        # at H (70, 140, 270, 300, 520); b = 0 and 1 as well
        ns = [a * W + b for a in (5, 17, 70, 100, 140, 270, 300, 511, 520) for b in (0, 1, 129, W // 2 + 3, W - 5)]
        if logW == 8:
            # a = 1116 splits at 1024: tiles of more than 76 KiB with the
            # twiddle copy, so the planner leaves the copy out
            ns += [1116 * W + b for b in (0, 1, 129, 200)]
        for n in ns:
            print(f"[gpu] {name} logW={logW} n={n}", flush=True)
            check_roundtrip(ctx, p, g, n, seed=n + 7 * logW)
    finally:
        libtft.tft_set_plan_override(ctx, 0)


@pytest.mark.parametrize("name", ["p998244353", "goldilocks", "p63"])
def test_two_pass_planner_sizes(ctxs, name):
    p, g = PRIMES[name]
    ctx = ctxs[name]
    for n in [8193, 10000, 16383, 16384, 16385, 40000, 65535, 65536, 65537, 100003, 262145]:
        plan = libtft.tft_plan_info(ctx, n)
        print(f"[gpu] {name} n={n} plan={plan}", flush=True)
        check_roundtrip(ctx, p, g, n, seed=3 * n)


@pytest.mark.parametrize("name", ["p12289", "p7681", "p2013265921", "p469762049", "p1811939329", "p62"])
def test_other_primes(ctxs, name):
    p, g = PRIMES[name]
    ctx = ctxs[name]
    v = oracle.two_adic(p)
    top = 1 << min(v, 14)
    for n in [1, 2, 3, 5, 100, 255, 256, 257, 1000, top - 1, top, 5000, 20001]:
        if (n - 1).bit_length() > v:
            continue
        print(f"[gpu] {name} n={n}", flush=True)
        check_roundtrip(ctx, p, g, n, seed=n + 5)


@pytest.mark.parametrize("name", ["p998244353", "goldilocks", "p63"])
def test_products(ctxs, name):
    p, g = PRIMES[name]
    ctx = ctxs[name]
    # (3, 200000) .. (20000, 280000): one operand much shorter than the
    # product, so its column tiles hold only a few nonzero rows (the column
    # pass skips the stages that only copy them); r = 2^17 - 1 and 2^17: the
    # products whose rows run as one launch (b = W - 1 with a + 1 a power of
    # two, and b = 0)
    for m, nb in [(1, 1), (1, 7), (5, 1), (3, 4), (1000, 1500), (4096, 4097), (5000, 3000), (30000, 40001),
                  (3, 200000), (150000, 7), (100, 300001), (20000, 280000), (65536, 65536), (40000, 91072),
                  (65536, 65537)]:
        print(f"[gpu] {name} product {m}x{nb}", flush=True)
        A = synth.residues(p, m, 100 + m)
        B = synth.residues(p, nb, 200 + nb)
        C = gpu_mul(ctx, A, B)
        ref = oracle.mul_schoolbook(p, A, B) if m * nb <= 4_000_000 else oracle.mul_padded(p, g, A, B)
        assert (C == ref).all(), f"product {m}x{nb} mismatches at {np.nonzero(C != ref)[0][:5]}"


@pytest.mark.parametrize("name", ["p998244353", "goldilocks", "p63"])
def test_restricted_products(ctxs, name):
    # section 5's space-restricted product (Algorithm 3): X is the only memory
    # written; blocks at global index q/L include two-pass ones with q > 0
    p, g = PRIMES[name]
    ctx = ctxs[name]
    for m, nb in [(1, 1), (1, 2), (2, 2), (1, 7), (5, 1), (3, 4), (17, 16), (1000, 1500), (4096, 4097),
                  (5000, 3000), (30000, 40001), (65536, 1), (12345, 98765)]:
        print(f"[gpu] {name} restricted product {m}x{nb}", flush=True)
        A = synth.residues(p, m, 300 + m)
        B = synth.residues(p, nb, 400 + nb)
        C = gpu_mul_restricted(ctx, A, B)
        ref = oracle.mul_schoolbook(p, A, B) if m * nb <= 4_000_000 else oracle.mul_padded(p, g, A, B)
        assert (C == ref).all(), f"restricted product {m}x{nb} mismatches at {np.nonzero(C != ref)[0][:5]}"


@pytest.mark.parametrize("name", ["p998244353", "goldilocks", "p63"])
def test_restricted_tail_nodes(ctxs, name):
    # the restricted product's last positions (t = r - q < 2^18 of them) come
    # from one or two aligned nodes: single-workgroup nodes of S = 2^13 words
    # (4-byte words) or 2^12 (8-byte) when t < 2S, else nodes of size
    # 2^(ceil(lg t) - 1) transformed in two passes.  r below, at and above 2S,
    # 3S and 4S, r < 2S (the whole product from the nodes), and r around 2^18
    # (the first block of 2^17, then nodes)
    p, g = PRIMES[name]
    ctx = ctxs[name]
    S = 1 << (13 if ctx.word_bytes == 4 else 12)
    for r in [S - 3, 2 * S - 1, 2 * S, 2 * S + 1, 3 * S - 1, 3 * S, 3 * S + 1, 4 * S - 1, 5 * S + 7,
              3 * (1 << 15) + 1, (1 << 18) - 1, 1 << 18, (1 << 18) + 1, 5 * (1 << 17) + 3]:
        m = r // 3 + 1
        nb = r + 1 - m
        print(f"[gpu] {name} restricted product {m}x{nb} (r = {r}, S = {S})", flush=True)
        A = synth.residues(p, m, 500 + r)
        B = synth.residues(p, nb, 600 + r)
        C = gpu_mul_restricted(ctx, A, B)
        ref = oracle.mul_padded(p, g, A, B)
        assert (C == ref).all(), f"restricted product r={r} mismatches at {np.nonzero(C != ref)[0][:5]}"


def test_rejects_bad_arguments(ctxs):
    import torch
    ctx = ctxs["p998244353"]
    X = torch.zeros(16, dtype=torch.uint32, device="cuda")
    with pytest.raises(libtft.TftError) as e:
        libtft.tft_forward(ctx, X, 0)
    assert e.value.status == libtft.TFT_EINVAL
    big = torch.zeros(1, dtype=torch.uint32, device="cuda")
    with pytest.raises(libtft.TftError) as e:
        libtft.tft_forward(ctx, big, (1 << 23) + 1)   # needs a root of order 2^24
    assert e.value.status == libtft.TFT_ERANGE
    with pytest.raises(libtft.TftError):
        libtft.Context(998244353, 4)                   # 4 is a square: not a generator
    for p in [(1 << 63) + 29, (1 << 61) - 3, 9223372006790004739]:   # beyond 2^63, composite, composite
        with pytest.raises(libtft.TftError) as e:
            libtft.Context(p, 3)
        assert e.value.status == libtft.TFT_ERANGE


@pytest.mark.parametrize("name", ["p998244353", "goldilocks", "p63"])
def test_buffered_comparator(ctxs, name):
    # van der Hoeven-style buffered transforms (2^ceil(lg n)-word buffer): the
    # same outputs as the oracle, the inverse restores the input, for every
    # kind of last row and the single-workgroup sizes
    import torch
    p, g = PRIMES[name]
    ctx = ctxs[name]
    for n in [1, 7, 1000, 2499, 8193, 100003, 65537, 3 * 4096 + 5, (1 << 17) - 1, 40000, 262145, 300000]:
        F = synth.residues(p, n, 4 * n + 1)
        L = 1 << (n - 1).bit_length()
        buf = torch.full((L,), 3, dtype=ctx.dtype, device="cuda")
        buf[:n] = torch.from_numpy(F.astype(np.uint32 if ctx.word_bytes == 4 else np.uint64)).cuda()
        print(f"[gpu] buffered {name} n={n}", flush=True)
        libtft.tft_buffered_forward(ctx, buf, n)
        got = buf[:n].cpu().numpy().astype(np.uint64)
        assert (got == oracle.fft_padded(p, g, F)).all(), n
        libtft.tft_buffered_inverse(ctx, buf, n)
        assert (buf[:n].cpu().numpy().astype(np.uint64) == F).all(), n
