"""Calibration and autotuning entry points: the calibration returns plausible
device ceilings, the autotuner caches a valid plan by ceil(lg n), and results
under the tuned plan still match the oracle bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import synth
from conftest import PRIMES
from paper_1001_5272_amd import libtft


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["p998244353", "goldilocks"])
def test_calibrate(name):
    p, g = PRIMES[name]
    ctx = libtft.Context(p, g, 0)
    try:
        print(f"[gpu] calibrate {name}", flush=True)
        c = libtft.tft_calibrate(ctx)
        print(c, flush=True)
        assert 1.0 < c["valu_tops"] < 200.0
        assert 1.0 < c["mad64_tops"] < 200.0
        assert 10.0 < c["butterflies_g"] < 20000.0
        assert 100.0 < c["copy_gbs"] < 20000.0
        # an exchange after every unit cannot make the butterflies faster
        for k in ("butterflies_lds_xchg_g", "butterflies_bpermute_xchg_g", "butterflies_dpp_xchg_g"):
            assert 1.0 < c[k] < 1.05 * c["butterflies_g"], (k, c)
    finally:
        ctx.close()


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["p998244353", "goldilocks"])
def test_autotune_then_parity(name):
    p, g = PRIMES[name]
    ctx = libtft.Context(p, g, 0)
    dt = np.uint32 if ctx.word_bytes == 4 else np.uint64
    try:
        n = 100003                      # two-pass for both word sizes; bucket floor(4 lg n) = 66
        bk = libtft.tft_plan_bucket(n)
        assert bk == 66
        print(f"[gpu] autotune {name} n={n}", flush=True)
        plan = libtft.tft_autotune(ctx, n)
        assert plan["kind"] == 1
        code = libtft.tft_plan_cache_get(ctx, bk)
        assert code & 31 == plan["logW"]
        assert libtft.plan_cache_dump(ctx) == {bk: code}
        for m in (n, 97000, 110000):    # every length of the bucket uses the tuned plan
            assert libtft.tft_plan_info(ctx, m)["logW"] == plan["logW"]
            assert libtft.tft_plan_info(ctx, m)["cols_per_tile"] == plan["cols_per_tile"]
            F = synth.residues(p, m, 77 + m)
            X = torch.from_numpy(F.astype(dt)).cuda()
            libtft.tft_forward(ctx, X)
            torch.cuda.synchronize()
            got = X.cpu().numpy().astype(np.uint64)
            ref = oracle.fft_padded(p, g, F)
            assert (got == ref).all(), f"forward differs at m={m} under the tuned plan"
            libtft.tft_inverse(ctx, X)
            torch.cuda.synchronize()
            assert (X.cpu().numpy().astype(np.uint64) == F).all(), f"inverse differs at m={m}"
        # a cache entry can be set by hand and cleared
        libtft.tft_plan_cache_set(ctx, bk, 0)
        assert libtft.plan_cache_dump(ctx) == {}
        libtft.plan_cache_load(ctx, {bk: code})
        assert libtft.tft_plan_cache_get(ctx, bk) == code
    finally:
        ctx.close()


def plan_code(logW, logC=0, rlog=0, smax=0):
    return logW | (logC << 5) | (rlog << 8) | (smax << 11)


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["p998244353", "goldilocks"])
def test_every_plan_knob_is_exact(name):
    """Each knob the autotuner can set -- columns per tile 8 or 16, one or two
    radix-8 units per row thread, 1, 2 or 3 stages per LDS round trip -- with
    the product and both transforms against the oracle, at lengths with
    b = 0, a general last row, b = W - 1 and a split column."""
    p, g = PRIMES[name]
    ctx = libtft.Context(p, g, 0)
    dt = np.uint32 if ctx.word_bytes == 4 else np.uint64
    codes = [plan_code(7, 3, 3, 3), plan_code(7, 4, 3, 3), plan_code(8, 0, 4, 0), plan_code(7, 0, 0, 2),
             plan_code(8, 4, 4, 1), plan_code(9, 3, 4, 2)]
    try:
        for code in codes:
            W = 1 << (code & 31)
            for n in (129 * W, 150 * W + 37, 256 * W - 1, 256 * W + W // 2):
                bk = libtft.tft_plan_bucket(n)
                libtft.tft_plan_cache_set(ctx, bk, code)
                plan = libtft.tft_plan_info(ctx, n)
                print(f"[gpu] {name} code={code:#x} n={n} plan={plan}", flush=True)
                assert plan["logW"] == code & 31
                F = synth.residues(p, n, n + code)
                X = torch.from_numpy(F.astype(dt)).cuda()
                libtft.tft_forward(ctx, X)
                torch.cuda.synchronize()
                assert (X.cpu().numpy().astype(np.uint64) == oracle.fft_padded(p, g, F)).all(), (code, n)
                libtft.tft_inverse(ctx, X)
                torch.cuda.synchronize()
                assert (X.cpu().numpy().astype(np.uint64) == F).all(), (code, n)
                la = n // 2 + 1
                A, B = synth.residues(p, la, 3 * n), synth.residues(p, n + 1 - la, 3 * n + 1)
                dA = torch.from_numpy(A.astype(dt)).cuda()
                dB = torch.from_numpy(B.astype(dt)).cuda()
                Xc = torch.empty(n, dtype=ctx.dtype, device="cuda")
                Yc = torch.empty(n, dtype=ctx.dtype, device="cuda")
                libtft.poly_mul(ctx, dA, dB, Xc, Yc)
                torch.cuda.synchronize()
                assert (Xc.cpu().numpy().astype(np.uint64) == oracle.mul_padded(p, g, A, B)).all(), (code, n)
                libtft.tft_plan_cache_set(ctx, bk, 0)
    finally:
        ctx.close()


@pytest.mark.gpu
def test_timing_select_brackets_only_selected_kernels():
    # measurement mode with a kernel mask: only the selected kernels' launches
    # are timed, the others run untimed, and results are unchanged
    p, g = PRIMES["goldilocks"]
    ctx = libtft.Context(p, g, 0)
    try:
        n = (1 << 20) + 3
        F = synth.residues(p, n, 5)
        X = torch.from_numpy(F).cuda()
        print(f"[gpu] timing select n={n}", flush=True)
        libtft.tft_timing_reset(ctx)
        libtft.tft_timing_enable(ctx, True)
        libtft.tft_forward(ctx, X)
        libtft.tft_inverse(ctx, X)
        torch.cuda.synchronize()
        every = libtft.tft_timing_read(ctx)
        assert {"col_fwd", "row_fwd", "row_inv"} <= set(every)
        libtft.tft_timing_reset(ctx)
        libtft.tft_timing_select(ctx, ["row_fwd"])
        libtft.tft_forward(ctx, X)
        libtft.tft_inverse(ctx, X)
        torch.cuda.synchronize()
        only = libtft.tft_timing_read(ctx)
        assert set(only) == {"row_fwd"} and only["row_fwd"][0] == 1
        libtft.tft_timing_select(ctx, None)
        libtft.tft_timing_enable(ctx, False)
        assert (X.cpu().numpy() == F).all()
    finally:
        ctx.close()
