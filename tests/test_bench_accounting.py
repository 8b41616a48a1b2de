"""The benchmark's work accounting (host only): the butterflies and words it
credits to each pass add up to the whole transform, so the roofline figures
neither drop nor double-count work."""
import math

import pytest

import bench


def plan(n, logW):
    W = 1 << logW
    return {"kind": 1, "logW": logW, "W": W, "a": n >> logW, "b": n & (W - 1)}


CASES = [(n, lw) for n in bench.SWEEP for lw in (11, 12, 13)] + [(3 * 2**20 + 77, 10), (2**21 - 1, 11)]


@pytest.mark.parametrize("n,logW", CASES)
def test_pass_butterflies_add_up(n, logW):
    P = plan(n, logW)
    fwd = bench.pass_butterflies("row_fwd", n, P) + bench.pass_butterflies("col_fwd", n, P)
    inv = sum(bench.pass_butterflies(k, n, P) for k in ("row_inv", "col_inv_short", "col_inv_long"))
    assert fwd == pytest.approx(bench.nominal_butterflies(n), rel=1e-12)
    assert inv == pytest.approx(bench.nominal_butterflies(n), rel=1e-12)


@pytest.mark.parametrize("n,logW", CASES)
def test_pass_words_cover_the_buffer(n, logW):
    P = plan(n, logW)
    for k in ("row_fwd", "row_inv", "col_fwd"):
        assert bench.pass_words(k, n, P) == n
    assert bench.pass_words("col_inv_short", n, P) + bench.pass_words("col_inv_long", n, P) == n


def test_small_plans_credit_the_single_workgroup_kernel():
    P = {"kind": 0}
    assert bench.pass_butterflies("small_fwd", 2499, P) == bench.nominal_butterflies(2499)
    assert bench.pass_butterflies("row_fwd", 2499, P) == 0.0
    assert bench.pass_words("small_inv", 2499, P) == 2499


def test_peaks():
    assert bench.VALU_PEAK_TOPS == pytest.approx(256 * 4 * 16 * 2.4e9 / 1e12)
    assert bench.nominal_butterflies(1 << 22) == (1 << 21) * 22
    assert math.isclose(bench.HBM_PEAK_GBS, 8000.0)
