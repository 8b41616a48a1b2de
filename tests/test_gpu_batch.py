"""GPU parity for batched products and transforms, graph replay, and the
three-prime exact integer product.  Bit-exact against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from conftest import PRIMES

pytestmark = pytest.mark.gpu
libtft = pytest.importorskip("paper_1001_5272_amd.libtft")
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx998():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = libtft.Context(*PRIMES["p998244353"])
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctxgl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = libtft.Context(*PRIMES["goldilocks"])
    yield c
    c.close()


def make_jobs(ctx, p, lens, seed):
    dt = np.uint32 if ctx.word_bytes == 4 else np.uint64
    jobs, host = [], []
    for i, (la, lb) in enumerate(lens):
        A = synth.residues(p, la, seed + 2 * i)
        B = synth.residues(p, lb, seed + 2 * i + 1)
        r = la + lb - 1
        dA = torch.from_numpy(A.astype(dt)).cuda()
        dB = torch.from_numpy(B.astype(dt)).cuda()
        X = torch.zeros(r, dtype=ctx.dtype, device="cuda")
        Y = torch.zeros(r, dtype=ctx.dtype, device="cuda")
        jobs.append((dA, dB, X, Y))
        host.append((A, B))
    return jobs, host


def expected(p, g, A, B):
    if len(A) * len(B) <= 2_000_000:
        return oracle.mul_schoolbook(p, A, B)
    return oracle.mul_padded(p, g, A, B)


def seeded_lengths(n, lo, hi, seed):
    la = synth.log_uniform_lengths(lo, hi, n, seed)
    lb = synth.log_uniform_lengths(lo, hi, n, seed + 1)
    return list(zip(la.tolist(), lb.tolist()))


@pytest.mark.parametrize("which", ["p998244353", "goldilocks"])
def test_batch_products_match_oracle_and_solo(ctx998, ctxgl, which):
    ctx = ctx998 if which == "p998244353" else ctxgl
    p, g = PRIMES[which]
    lens = seeded_lengths(120, 1, 12000, 77) + [(1, 1), (1, 5), (7, 1), (4096, 4097), (9000, 9000), (1, 30000)]
    print(f"[gpu] batch of {len(lens)} products, {which}", flush=True)
    jobs, host = make_jobs(ctx, p, lens, 500)
    b = libtft.Batch(ctx, jobs)
    info = b.info()
    assert info["single_workgroup"] > 0 and info["two_pass"] > 0, info
    b.run()
    torch.cuda.synchronize()
    for (A, B), (_, _, X, _) in zip(host, jobs):
        got = X.cpu().numpy().astype(np.uint64)
        ref = expected(p, g, A, B)
        assert (got == ref).all(), f"batch product {len(A)}x{len(B)} differs"
    # the same instance alone gives the same words
    for k in [0, 3, len(jobs) - 3, len(jobs) - 1]:
        dA, dB, X, Y = jobs[k]
        X2 = torch.empty_like(X)
        Y2 = torch.empty_like(Y)
        libtft.poly_mul(ctx, dA, dB, X2, Y2)
        torch.cuda.synchronize()
        assert torch.equal(X, X2)
    b.close()


@pytest.mark.parametrize("which", ["p998244353", "goldilocks"])
def test_batch_products_long_rows(ctx998, ctxgl, which):
    """Products long enough that a batch row holds 2048 words: the fused row
    product then takes one row per workgroup (b > 0 and b = 0)."""
    ctx = ctx998 if which == "p998244353" else ctxgl
    p, g = PRIMES[which]
    lens = [(1 << 20, (1 << 20) + 5), (1500000, 700001), (3000, 1 << 21), (1 << 20, (1 << 20) + 1), (5, 7)]
    print(f"[gpu] batch of long products, {which}", flush=True)
    jobs, host = make_jobs(ctx, p, lens, 900)
    b = libtft.Batch(ctx, jobs)
    b.run()
    torch.cuda.synchronize()
    for (A, B), (_, _, X, _) in zip(host, jobs):
        got = X.cpu().numpy().astype(np.uint64)
        assert (got == expected(p, g, A, B)).all(), f"batch product {len(A)}x{len(B)} differs"
    b.close()


def test_batch_graph_replay(ctx998):
    p, g = PRIMES["p998244353"]
    lens = seeded_lengths(40, 16, 20000, 91)
    jobs, host = make_jobs(ctx998, p, lens, 900)
    b = libtft.Batch(ctx998, jobs)
    refs = [expected(p, g, A, B) for A, B in host]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run()                      # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.run()
    for rep in range(4):
        for (_, _, X, _) in jobs:
            X.zero_()                # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for ref, (_, _, X, _) in zip(refs, jobs):
            assert (X.cpu().numpy().astype(np.uint64) == ref).all(), f"replay {rep} differs"
    b.close()


def test_poly_mul_batch_convenience(ctxgl):
    p, g = PRIMES["goldilocks"]
    lens = seeded_lengths(30, 1, 9000, 31)
    jobs, host = make_jobs(ctxgl, p, lens, 300)
    libtft.poly_mul_batch(ctxgl, jobs)
    torch.cuda.synchronize()
    for (A, B), (_, _, X, _) in zip(host, jobs):
        assert (X.cpu().numpy().astype(np.uint64) == expected(p, g, A, B)).all()


def test_batch_products_64bit_montgomery_prime():
    # a prime of 8-byte words other than 2^64 - 2^32 + 1: the batch's
    # single-workgroup and two-pass products in 64-bit Montgomery arithmetic,
    # every product against the oracle
    p, g = PRIMES["p63"]
    ctx = libtft.Context(p, g)
    try:
        lens = seeded_lengths(60, 1, 12000, 78) + [(1, 1), (4096, 4097), (9000, 9000), (1, 30000)]
        print(f"[gpu] batch of {len(lens)} products, p63", flush=True)
        jobs, host = make_jobs(ctx, p, lens, 700)
        b = libtft.Batch(ctx, jobs)
        info = b.info()
        assert info["single_workgroup"] > 0 and info["two_pass"] > 0, info
        b.run()
        torch.cuda.synchronize()
        for (A, B), (_, _, X, _) in zip(host, jobs):
            assert (X.cpu().numpy().astype(np.uint64) == expected(p, g, A, B)).all(), (len(A), len(B))
        b.close()
    finally:
        ctx.close()


@pytest.mark.parametrize("which", ["p998244353", "goldilocks"])
def test_forward_batch(ctx998, ctxgl, which):
    ctx = ctx998 if which == "p998244353" else ctxgl
    p, g = PRIMES[which]
    ns = [1, 2, 3, 100, 2499, 8191, 8193, 20000, 65537] + synth.log_uniform_lengths(1, 30000, 20, 5).tolist()
    dt = np.uint32 if ctx.word_bytes == 4 else np.uint64
    host = [synth.residues(p, n, 40 + i) for i, n in enumerate(ns)]
    xs = [torch.from_numpy(h.astype(dt)).cuda() for h in host]
    libtft.tft_forward_batch(ctx, xs)
    torch.cuda.synchronize()
    for F, X in zip(host, xs):
        assert (X.cpu().numpy().astype(np.uint64) == oracle.fft_padded(p, g, F)).all(), len(F)


def test_convenience_calls_reuse_work_list_memory(ctxgl):
    """Consecutive convenience calls share the context's work-list memory: a
    call that grows it (40000 instances) between smaller ones, and a product
    batch after the transforms, all still match the oracle."""
    p, g = PRIMES["goldilocks"]

    def forward(ns, seed, sample):
        host = [synth.residues(p, int(n), seed + i) for i, n in enumerate(ns)]
        xs = [torch.from_numpy(h).cuda() for h in host]
        libtft.tft_forward_batch(ctxgl, xs)
        torch.cuda.synchronize()
        for i in sample:
            got = xs[i].cpu().numpy().astype(np.uint64)
            assert (got == oracle.fft_padded(p, g, host[i])).all(), (seed, i, len(host[i]))

    ns = synth.log_uniform_lengths(1, 30000, 20, 61).tolist()
    forward(ns, 600, range(len(ns)))
    many = synth.log_uniform_lengths(1, 64, 40000, 62).tolist()
    forward(many, 700, list(range(0, 40000, 97)) + [39999])
    few = [1, 5, 4096, 4097, 12345, 3, 64]
    forward(few, 800, range(len(few)))
    lens = seeded_lengths(12, 1, 9000, 63)
    jobs, host = make_jobs(ctxgl, p, lens, 900)
    libtft.poly_mul_batch(ctxgl, jobs)
    torch.cuda.synchronize()
    for (A, B), (_, _, X, _) in zip(host, jobs):
        assert (X.cpu().numpy().astype(np.uint64) == expected(p, g, A, B)).all()


@pytest.mark.parametrize("name", ["p2013265921", "p469762049", "goldilocks", "p63"])
def test_from_signed_edges(name):
    # signed 64-bit integers to residues: the extremes, small values of both
    # signs and random 64-bit values, against Python's floor modulo
    p, g = PRIMES[name]
    ctx = libtft.Context(p, g)
    try:
        rng = np.random.default_rng(9)
        v = np.concatenate([np.array([0, 1, -1, 2**63 - 1, -2**63, -2**63 + 1, p % 2**63, -(p % 2**63),
                                      2**32, -2**32, 2**32 - 1, -(2**32 - 1)], dtype=np.int64),
                            rng.integers(-2**63, 2**63 - 1, 100000, dtype=np.int64, endpoint=True)])
        dv = torch.from_numpy(v).cuda()
        X = torch.empty(len(v), dtype=ctx.dtype, device="cuda")
        libtft.tft_from_signed(ctx, dv, X)
        torch.cuda.synchronize()
        got = X.cpu().numpy().astype(np.uint64)
        want = np.array([int(x) % p for x in v.tolist()], dtype=np.uint64)
        assert (got == want).all(), np.nonzero(got != want)[0][:5]
    finally:
        ctx.close()


def test_crt3_random_residues():
    # Garner's reconstruction alone: random residue triples (and the edges 0,
    # -1, (M-1)/2, (M+1)/2) against the Chinese remainder by Python integers,
    # as the signed representative in (-M/2, M/2]
    ctxs = [libtft.Context(p, g) for p, g in synth.CRT_PRIMES]
    try:
        (p1, _), (p2, _), (p3, _) = synth.CRT_PRIMES
        M = p1 * p2 * p3
        n = 100000
        rs = [synth.residues(p, n, 8100 + i).astype(np.uint32) for i, (p, _) in enumerate(synth.CRT_PRIMES)]
        edges = [0, M - 1, (M - 1) // 2, (M + 1) // 2, p1, p1 * p2, M - p1 * p2]
        for k, v in enumerate(edges):
            for r, (p, _) in zip(rs, synth.CRT_PRIMES):
                r[k] = v % p
        dev = [torch.from_numpy(r).cuda() for r in rs]
        out = torch.empty(2 * n, dtype=torch.int64, device="cuda")
        libtft.tft_crt3(ctxs, dev[0], dev[1], dev[2], out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint64)
        e1, e2, e3 = [(M // p) * pow(M // p, -1, p) for p in (p1, p2, p3)]   # idempotents of Z/M
        for i in range(n):
            x = (int(rs[0][i]) * e1 + int(rs[1][i]) * e2 + int(rs[2][i]) * e3) % M
            if x > M // 2:
                x -= M
            v = (int(got[2 * i + 1]) << 64) | int(got[2 * i])
            if v >= 1 << 127:
                v -= 1 << 128
            assert v == x, (i, [int(r[i]) for r in rs])
    finally:
        for c in ctxs:
            c.close()


def test_exact_integer_product_crt():
    ctxs = [libtft.Context(p, g) for p, g in synth.CRT_PRIMES]
    try:
        for m, nb in [(1, 1), (5, 3), (200, 300), (3000, 5000), (20000, 12345)]:
            print(f"[gpu] crt product {m}x{nb}", flush=True)
            a = synth.signed24(m, 5001 + m)
            b = synth.signed24(nb, 5002 + nb)
            r = m + nb - 1
            da = torch.from_numpy(a).cuda()
            db = torch.from_numpy(b).cuda()
            res = []
            for c in ctxs:
                A = torch.empty(m, dtype=torch.uint32, device="cuda")
                B = torch.empty(nb, dtype=torch.uint32, device="cuda")
                libtft.tft_from_signed(c, da, A)
                libtft.tft_from_signed(c, db, B)
                X = torch.empty(r, dtype=torch.uint32, device="cuda")
                Y = torch.empty(r, dtype=torch.uint32, device="cuda")
                libtft.poly_mul(c, A, B, X, Y)
                res.append(X)
            out = torch.empty(2 * r, dtype=torch.int64, device="cuda")
            libtft.tft_crt3(ctxs, res[0], res[1], res[2], out)
            torch.cuda.synchronize()
            got = out.cpu().numpy().view(np.uint64)
            if m * nb <= 3_000_000:
                ref = oracle.conv_i128(a, b, as_lohi=True)
                assert (got == ref).all()
            else:
                for s in [0, 1, r // 3, r // 2, r - 2, r - 1]:
                    v = (int(got[2 * s + 1]) << 64) | int(got[2 * s])
                    if v >= 1 << 127:
                        v -= 1 << 128
                    assert v == oracle.conv_coeff_i128(a, b, s), s
    finally:
        for c in ctxs:
            c.close()
