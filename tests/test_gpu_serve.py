"""GPU tests of the serving queue: every request's result is the same words
as the same product computed alone (tolerance zero: exact arithmetic) and as
the oracle; admission by footprint defers requests without losing any."""
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


@pytest.mark.parametrize("pool_words,max_inflight", [(1 << 24, 4096), (70000, 8)])
def test_served_equals_alone(ctx, pool_words, max_inflight):
    p, g = PRIMES["goldilocks"]
    reqs = requests(p, 60, 123)
    dev = [(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()) for A, B in reqs]
    outs = [torch.zeros(len(A) + len(B) - 1, dtype=torch.uint64, device="cuda") for A, B in reqs]
    torch.cuda.synchronize()
    q = libtft.Queue(ctx, pool_words, max_inflight)
    print(f"[gpu] queue pool={pool_words} inflight={max_inflight}", flush=True)
    tickets = []
    for i, ((dA, dB), X) in enumerate(zip(dev, outs)):
        tickets.append(q.submit(dA, dB, X))
        if i % 7 == 0:
            time.sleep(0.0005)        # arrivals spread over time, overlapping work on the device
    for t in tickets:
        q.wait(t)
    st = q.stats()
    assert st["completed"] == len(reqs) and st["pending"] == 0
    if pool_words < 100000:
        assert st["deferred"] > 0
        assert st["pool_used_max"] <= pool_words
    for t in tickets:
        assert q.completion_ns(t) > 0
    q.close()
    for (A, B), (dA, dB), X in zip(reqs, dev, outs):
        assert torch.equal(X, alone(ctx, dA, dB)), f"served {len(A)}x{len(B)} differs from alone"
    for k in [0, 5, 17, 59]:
        A, B = reqs[k]
        ref = oracle.mul_schoolbook(p, A, B) if len(A) * len(B) < 3_000_000 else oracle.mul_padded(p, g, A, B)
        assert (outs[k].cpu().numpy() == ref).all()


def test_queue_rejects(ctx):
    q = libtft.Queue(ctx, 1000, 4)
    a = torch.zeros(800, dtype=torch.uint64, device="cuda")
    X = torch.zeros(1599, dtype=torch.uint64, device="cuda")
    with pytest.raises(libtft.TftError) as e:
        q.submit(a, a, X)              # needs 1599 words of workspace, the pool has 1000
    assert e.value.status == libtft.TFT_ERANGE
    q.close()
