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
        assert libtft.tft_plan_cache_get(ctx, bk) == plan["logW"]
        assert libtft.plan_cache_dump(ctx) == {bk: plan["logW"]}
        for m in (n, 97000, 110000):    # every length of the bucket uses the tuned width
            assert libtft.tft_plan_info(ctx, m)["logW"] == plan["logW"]
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
        libtft.plan_cache_load(ctx, {bk: plan["logW"]})
        assert libtft.tft_plan_cache_get(ctx, bk) == plan["logW"]
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
