"""poly_mul_noalloc (the product with B's transform in the library's fixed
device array) against poly_mul (caller workspace), bit for bit, on two calls
in a row with the second one shorter, so that the array holds the first
call's words when the second starts; and the size limit, which is checked on
the host before anything is enqueued."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import to_dev, to_host
from paper_1001_5272_amd import libtft

pytestmark = pytest.mark.gpu

CASES = {
    # (p, g), [(m, nb) of the first, longer call; (m, nb) of the second]
    "goldilocks": ((2**64 - 2**32 + 1, 7), [(1 << 21, (1 << 21) + 1), (150001, 100003)]),   # r = 2^22 (the limit)
    "p998244353": ((998244353, 3), [(3000000, 2500017), (40000, 25000)]),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_noalloc_equals_poly_mul(name):
    (p, g), shapes = CASES[name]
    ctx = libtft.Context(p, g, 0)
    for call, (m, nb) in enumerate(shapes):
        print(f"[noalloc] {name} call {call}: m={m} nb={nb}", flush=True)
        A = synth.residues(p, m, 7100 + 2 * call)
        B = synth.residues(p, nb, 7101 + 2 * call)
        dA, dB = to_dev(ctx, A), to_dev(ctx, B)
        r = m + nb - 1
        X0 = torch.empty(r, dtype=ctx.dtype, device=dA.device)
        Y0 = torch.empty(r, dtype=ctx.dtype, device=dA.device)
        libtft.poly_mul(ctx, dA, dB, X0, Y0)
        X1 = torch.full((r,), 3, dtype=ctx.dtype, device=dA.device)
        libtft.poly_mul_noalloc(ctx, dA, dB, X1)
        ref, got = to_host(X0), to_host(X1)
        assert got.shape == ref.shape
        bad = np.nonzero(got != ref)[0]
        assert bad.size == 0, f"call {call}: {bad.size} words differ, first at {bad[:5]}"
    ctx.close()


def test_noalloc_rejects_beyond_the_limit():
    p, g = 2**64 - 2**32 + 1, 7
    ctx = libtft.Context(p, g, 0)
    A = torch.zeros(1 << 21, dtype=ctx.dtype, device="cuda:0")
    B = torch.zeros((1 << 21) + 2, dtype=ctx.dtype, device="cuda:0")     # r = 2^22 + 1
    X = torch.zeros((1 << 22) + 1, dtype=ctx.dtype, device="cuda:0")
    with pytest.raises(libtft.TftError) as e:
        libtft.poly_mul_noalloc(ctx, A, B, X)
    assert e.value.status == libtft.TFT_ERANGE
    ctx.close()
