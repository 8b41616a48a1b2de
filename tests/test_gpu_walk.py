"""The paper's Algorithms 1 and 2 run literally, one wavefront per instance
(tft_walk_batch): bit-exact against the oracle at every length up to 300 and
at larger ones up to the 1024-word limit, and the inverse restores the input."""
import numpy as np
import pytest

import oracle
import synth
from conftest import PRIMES

pytestmark = pytest.mark.gpu

libtft = pytest.importorskip("paper_1001_5272_amd.libtft")


@pytest.mark.parametrize("name", ["p998244353", "goldilocks", "p63"])
def test_walk_matches_oracle(name):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p, g = PRIMES[name]
    ctx = libtft.Context(p, g, 0)
    dt = np.uint32 if ctx.word_bytes == 4 else np.uint64
    try:
        ns = list(range(1, 301)) + [511, 512, 513, 700, 1000, 1023, 1024]
        F = [synth.residues(p, n, 900 + n) for n in ns]
        xs = [torch.from_numpy(f.astype(dt)).cuda() for f in F]
        print(f"[gpu] walk forward {name}: {len(ns)} instances", flush=True)
        libtft.tft_walk_batch(ctx, xs)
        for n, f, x in zip(ns, F, xs):
            ref = oracle.tft_direct(p, g, f) if n <= 64 else oracle.fft_padded(p, g, f)
            got = x.cpu().numpy().astype(np.uint64)
            bad = np.nonzero(got != ref)[0]
            assert len(bad) == 0, f"walk forward n={n}: mismatches at {bad[:5]}"
        print(f"[gpu] walk inverse {name}", flush=True)
        libtft.tft_walk_batch(ctx, xs, inverse=True)
        for n, f, x in zip(ns, F, xs):
            assert (x.cpu().numpy().astype(np.uint64) == f).all(), f"walk inverse n={n}"
    finally:
        ctx.close()


def test_walk_rejects_bad_lengths():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p, g = PRIMES["goldilocks"]
    ctx = libtft.Context(p, g, 0)
    try:
        big = torch.zeros(1025, dtype=torch.uint64, device="cuda")
        with pytest.raises(libtft.TftError) as e:
            libtft.tft_walk_batch(ctx, [big])
        assert e.value.status == libtft.TFT_ERANGE
        empty = torch.zeros(0, dtype=torch.uint64, device="cuda")
        with pytest.raises(libtft.TftError) as e:
            libtft.tft_walk_batch(ctx, [empty])
        assert e.value.status == libtft.TFT_EINVAL
    finally:
        ctx.close()
