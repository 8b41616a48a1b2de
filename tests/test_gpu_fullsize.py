"""Parity at the benchmark's full sizes and launch configurations.

- Goldilocks TFT at every length of the sweep: the whole output against the
  oracle's padded FFT; the inverse restores the input.
- Products at every r of the sweep (poly_mul, the space-restricted product and
  the allocation-free product): every coefficient against the oracle's padded
  product, plus exact coefficients and the evaluation identity
  C(z) = A(z) B(z) from the oracle's direct formulas.
- The 4096-product batch: every instance against the oracle.
- The three-prime exact product at length 2^24+12345: sampled exact int128
  coefficients and C(z) = A(z) B(z) modulo 2^61-1.
"""
import os
import random

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
libtft = pytest.importorskip("paper_1001_5272_amd.libtft")
torch = pytest.importorskip("torch")

SWEEP = [1 << 22, (1 << 22) + 1, 3 << 21, (1 << 23) - 1, 1 << 23]


@pytest.fixture(scope="module")
def ctxgl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = libtft.Context(*synth.GOLDILOCKS)
    yield c
    c.close()


@pytest.mark.parametrize("n", SWEEP)
def test_sweep_lengths_full_output(ctxgl, n):
    p, g = synth.GOLDILOCKS
    print(f"[gpu] full-size TFT n={n} plan={libtft.tft_plan_info(ctxgl, n)}", flush=True)
    F = synth.residues(p, n, 2000 + SWEEP.index(n))
    X = torch.from_numpy(F).cuda()
    libtft.tft_forward(ctxgl, X)
    got = X.cpu().numpy()
    ref = oracle.fft_padded(p, g, F)
    bad = np.nonzero(got != ref)[0]
    assert len(bad) == 0, f"{len(bad)} mismatches, first {bad[:5]}"
    idx = [0, 1, n // 2, n - 1] + [random.Random(n).randrange(n) for _ in range(4)]
    assert (oracle.tft_sample(p, g, F, idx) == got[idx]).all()
    libtft.tft_inverse(ctxgl, X)
    assert (X.cpu().numpy() == F).all()


@pytest.mark.parametrize("r", SWEEP)
def test_products_at_full_size(ctxgl, r):
    p, g = synth.GOLDILOCKS
    la = (r + 2) // 2
    lb = r + 1 - la
    print(f"[gpu] full-size products r={r}", flush=True)
    A = synth.residues(p, la, 3000 + r)
    B = synth.residues(p, lb, 4000 + r)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    X = torch.empty(r, dtype=torch.uint64, device="cuda")
    Y = torch.empty(r, dtype=torch.uint64, device="cuda")
    libtft.poly_mul(ctxgl, dA, dB, X, Y)
    X2 = torch.full((r,), 5, dtype=torch.uint64, device="cuda")
    libtft.poly_mul_restricted(ctxgl, dA, dB, X2)        # output buffer only
    C, C2 = X.cpu().numpy(), X2.cpu().numpy()
    ref = oracle.mul_padded(p, g, A, B)
    bad = np.nonzero(C != ref)[0]
    assert len(bad) == 0, f"poly_mul: {len(bad)} mismatches, first {bad[:5]}"
    bad = np.nonzero(C2 != ref)[0]
    assert len(bad) == 0, f"poly_mul_restricted: {len(bad)} mismatches, first {bad[:5]}"
    rng = random.Random(r)
    for s in [0, 1, r // 2, r - 2, r - 1] + [rng.randrange(r) for _ in range(3)]:
        assert int(ref[s]) == oracle.mul_coeff(p, A, B, s), s
    z = rng.randrange(p)
    assert oracle.evaluate(p, ref, z) == oracle.evaluate(p, A, z) * oracle.evaluate(p, B, z) % p
    if r <= 1 << 22:                                     # the allocation-free product's limit
        X3 = torch.full((r,), 9, dtype=torch.uint64, device="cuda")
        libtft.poly_mul_noalloc(ctxgl, dA, dB, X3)
        assert (X3.cpu().numpy() == ref).all()


def _oracle_products(p, g, host):
    """The oracle's product of every pair, on the host's cores (the oracle
    releases the interpreter lock while it computes)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(ab):
        A, B = ab
        if len(A) * len(B) <= 1_000_000:
            return oracle.mul_schoolbook(p, A, B)
        return oracle.mul_padded(p, g, A, B)
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, host))


def test_batch_4096_every_instance():
    p, g = synth.P998
    ctx = libtft.Context(p, g)
    count = 4096
    la = synth.log_uniform_lengths(32, 32768, count, 3001)
    lb = synth.log_uniform_lengths(32, 32768, count, 3002)
    jobs, host = [], []
    for i in range(count):
        A = synth.residues_u32(p, int(la[i]), 10_000 + 2 * i)
        B = synth.residues_u32(p, int(lb[i]), 10_001 + 2 * i)
        r = len(A) + len(B) - 1
        jobs.append((torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(),
                     torch.empty(r, dtype=torch.uint32, device="cuda"), torch.empty(r, dtype=torch.uint32, device="cuda")))
        host.append((A.astype(np.uint64), B.astype(np.uint64)))
    print("[gpu] batch of 4096 products (998244353)", flush=True)
    b = libtft.Batch(ctx, jobs)
    b.run()
    torch.cuda.synchronize()
    refs = _oracle_products(p, g, host)
    for i, ref in enumerate(refs):
        got = jobs[i][2].cpu().numpy().astype(np.uint64)
        assert (got == ref).all(), f"instance {i}: {len(host[i][0])} x {len(host[i][1])}"
    b.close()
    # the batch tuner's choice of row width (it runs the batch itself), then a
    # fresh batch planned with it: every instance again
    widen = libtft.tft_autotune_batch(ctx, jobs)
    print(f"[gpu] batch tuner chose rows {widen} steps wider than balanced", flush=True)
    assert widen in (0, 1, 2)
    tuning = libtft.tft_batch_tuning_get(ctx)
    assert tuning["widen"] == widen
    assert tuning["list_col_threads"] in (128, 256) and tuning["row_mul_threads"] in (128, 256), tuning
    for _, _, X, _ in jobs:
        X.zero_()
    b = libtft.Batch(ctx, jobs)
    b.run()
    torch.cuda.synchronize()
    for i, ref in enumerate(refs):
        got = jobs[i][2].cpu().numpy().astype(np.uint64)
        assert (got == ref).all(), f"tuned batch, instance {i}"
    b.close()
    ctx.close()


def test_exact_product_full_size():
    P61 = (1 << 61) - 1
    n = (1 << 24) + 12345
    r = 2 * n - 1
    a = synth.signed24(n, 5001)
    b = synth.signed24(n, 5002)
    ctxs = [libtft.Context(pp, gg) for pp, gg in synth.CRT_PRIMES]
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    res = []
    for c in ctxs:
        A = torch.empty(n, dtype=torch.uint32, device="cuda")
        B = torch.empty(n, dtype=torch.uint32, device="cuda")
        libtft.tft_from_signed(c, da, A)
        libtft.tft_from_signed(c, db, B)
        X = torch.empty(r, dtype=torch.uint32, device="cuda")
        Y = torch.empty(r, dtype=torch.uint32, device="cuda")
        libtft.poly_mul(c, A, B, X, Y)
        res.append(X)
        del A, B, Y
    out = torch.empty(2 * r, dtype=torch.int64, device="cuda")
    libtft.tft_crt3(ctxs, res[0], res[1], res[2], out)
    o = out.cpu().numpy()
    lo, hi = o[0::2].view(np.uint64), o[1::2]
    for s in [0, 1, r // 2, r - 1, 12345, r - 7]:
        v = (int(hi[s]) << 64) | int(lo[s])
        if v >= 1 << 127:
            v -= 1 << 128
        assert v == oracle.conv_coeff_i128(a, b, s), s
    # C(z) = A(z) B(z) mod 2^61 - 1, with C reduced from int128: 2^64 = 8 mod P61
    M61 = np.uint64(P61)
    lo_r = (lo >> np.uint64(61)) + (lo & M61)
    hi_r = (hi % P61).astype(np.uint64)           # floor mod of the signed high word
    Cr = (lo_r % M61 + (hi_r * np.uint64(8)) % M61) % M61
    ar = (a % P61).astype(np.uint64)
    br = (b % P61).astype(np.uint64)
    for z in [123456789, 987654321987]:
        assert oracle.evaluate(P61, Cr, z) == oracle.evaluate(P61, ar, z) * oracle.evaluate(P61, br, z) % P61
    for c in ctxs:
        c.close()
