"""GPU tests of the serving queue: every request's result is the same words
as the same product computed alone (tolerance zero: exact arithmetic) and as
the oracle; admission by footprint refuses (TFT_EAGAIN) what does not fit now
and never loses a request; the queue waits for the operands' producer stream."""
import time

import numpy as np
import pytest

import oracle
import synth
from conftest import PRIMES

pytestmark = pytest.mark.gpu
libtft = pytest.importorskip("paper_1001_5272_amd.libtft")
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = libtft.Context(*PRIMES["goldilocks"])
    yield c
    c.close()


def requests(p, n, seed, lo=1, hi=40000):
    la = synth.log_uniform_lengths(lo, hi, n, seed)
    lb = synth.log_uniform_lengths(lo, hi, n, seed + 1)
    out = []
    for i in range(n):
        A = synth.residues(p, int(la[i]), seed + 10 + 2 * i)
        B = synth.residues(p, int(lb[i]), seed + 11 + 2 * i)
        out.append((A, B))
    return out


def alone(ctx, dA, dB):
    r = dA.numel() + dB.numel() - 1
    X = torch.empty(r, dtype=ctx.dtype, device="cuda")
    Y = torch.empty(r, dtype=ctx.dtype, device="cuda")
    libtft.poly_mul(ctx, dA, dB, X, Y)
    torch.cuda.synchronize()
    return X


def oracle_product(p, g, A, B):
    return oracle.mul_schoolbook(p, A, B) if len(A) * len(B) < 3_000_000 else oracle.mul_padded(p, g, A, B)


@pytest.mark.parametrize("pool_words,max_inflight", [(1 << 24, 4096), (70000, 8)])
def test_served_equals_alone(ctx, pool_words, max_inflight):
    """Every request of a stream, served in a mix with others (small pool: many
    submits refused for footprint and retried), equals the same product run
    alone and the oracle, word for word."""
    p, g = PRIMES["goldilocks"]
    reqs = requests(p, 60, 123)
    dev = [(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()) for A, B in reqs]
    outs = [torch.zeros(len(A) + len(B) - 1, dtype=torch.uint64, device="cuda") for A, B in reqs]
    torch.cuda.synchronize()
    q = libtft.Queue(ctx, pool_words, max_inflight)
    print(f"[gpu] queue pool={pool_words} inflight={max_inflight}", flush=True)
    tickets, retries = [], 0
    for i, ((dA, dB), X) in enumerate(zip(dev, outs)):
        t = q.try_submit(dA, dB, X)
        while t is None:              # footprint does not fit now: wait for the oldest and retry
            retries += 1
            q.wait(next(x for x in tickets if not q.poll(x)))
            t = q.try_submit(dA, dB, X)
        tickets.append(t)
        if i % 7 == 0:
            time.sleep(0.0005)        # arrivals spread over time, overlapping work on the device
    for t in tickets:
        q.wait(t)
    st = q.stats()
    assert st["completed"] == len(reqs) and st["pending"] == 0
    assert st["rejected"] == retries
    if pool_words < 100000:
        assert retries > 0
        assert st["pool_used_max"] <= pool_words
    for t in tickets:
        assert q.completion_ns(t) > 0
    q.close()
    for (A, B), (dA, dB), X in zip(reqs, dev, outs):
        assert torch.equal(X, alone(ctx, dA, dB)), f"served {len(A)}x{len(B)} differs from alone"
    for k, (A, B) in enumerate(reqs):
        assert (outs[k].cpu().numpy() == oracle_product(p, g, A, B)).all(), f"request {k} differs from the oracle"


def test_queue_rejects(ctx):
    """Footprint admission: a product needing more workspace than the pool holds
    can never run (TFT_ERANGE); one that does not fit the free space now is
    refused with TFT_EAGAIN and queues nothing.  r = 9999 is above the
    single-workgroup limit of 8-byte words, so it needs r words of workspace."""
    p, g = PRIMES["goldilocks"]
    A = torch.from_numpy(synth.residues(p, 5000, 91)).cuda()
    B = torch.from_numpy(synth.residues(p, 5000, 92)).cuda()
    X1 = torch.zeros(9999, dtype=torch.uint64, device="cuda")
    X2 = torch.zeros(9999, dtype=torch.uint64, device="cuda")
    small = libtft.Queue(ctx, 9000, 4)
    with pytest.raises(libtft.TftError) as e:
        small.submit(A, B, X1)                       # 9999 > 9000: never fits
    assert e.value.status == libtft.TFT_ERANGE
    small.close()
    q = libtft.Queue(ctx, 15000, 4)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        torch.cuda._sleep(20_000_000)                # the first request's batch waits for this stream
    t1 = q.submit(A, B, X1, stream=s)
    assert q.try_submit(A, B, X2) is None            # its 9999 words are reserved: no room for a second
    with pytest.raises(libtft.TftError) as e:
        q.submit(A, B, X2)
    assert e.value.status == libtft.TFT_EAGAIN
    assert q.stats()["pending"] + q.stats()["inflight"] == 1
    q.wait(t1)
    t2 = q.submit(A, B, X2)                          # fits once the first has released its words
    q.wait(t2)
    assert q.stats()["rejected"] == 2
    q.close()
    ref = oracle_product(p, g, synth.residues(p, 5000, 91), synth.residues(p, 5000, 92))
    assert (X1.cpu().numpy() == ref).all() and (X2.cpu().numpy() == ref).all()


def test_queue_waits_for_producer_stream(ctx):
    """Operands written by work still running on the producer's stream: the
    queue's batch waits for that work (no host synchronisation in between),
    and the queue keeps the operand tensors alive after the caller drops them."""
    p, g = PRIMES["goldilocks"]
    reqs = requests(p, 12, 777, lo=2000, hi=30000)
    s = torch.cuda.Stream()
    q = libtft.Queue(ctx, 1 << 22, 4096)
    outs, tickets = [], []
    src = [(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()) for A, B in reqs]
    torch.cuda.synchronize()
    for sA, sB in src:
        with torch.cuda.stream(s):
            dA = torch.zeros_like(sA)
            dB = torch.zeros_like(sB)
            torch.cuda._sleep(2_000_000)             # the copies below land well after submit returns
            dA.copy_(sA, non_blocking=True)          # device to device, enqueued on s
            dB.copy_(sB, non_blocking=True)
            X = torch.zeros(len(sA) + len(sB) - 1, dtype=torch.uint64, device="cuda")
        tickets.append(q.submit(dA, dB, X, stream=s))
        outs.append(X)
        del dA, dB                                   # only the queue holds them now
    with torch.cuda.stream(s):                       # allocations that would reuse freed operand memory
        junk = [torch.full((30000,), 5, dtype=torch.uint64, device="cuda") for _ in range(24)]
    for t in tickets:
        q.wait(t)
    q.close()
    del junk
    for (A, B), X in zip(reqs, outs):
        assert (X.cpu().numpy() == oracle_product(p, g, A, B)).all()
