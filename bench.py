"""Benchmark of the in-place truncated Fourier transform on one MI355X.

Default workload (one "step"): forward TFT then inverse TFT, in place, over
Z/pZ with p = 2^64 - 2^32 + 1 (uint64 words, generator 7) at each length of
the sweep n in {2^22, 2^22+1, 3*2^21, 2^23-1, 2^23}; uniform residues from a
fixed seed, resident in HBM before timing starts.  `value` is the nominal
butterfly rate sum_n 2 (n/2) log2 n / time (forward + inverse per length).

Also reported (outside the timed step, same process):
- per-length forward/inverse times and the step at the power of two,
  t(2^22+1) / t(2^22), against the padded radix-2 comparator;
- poly_mul at product lengths r = n (operand lengths ceil((r+1)/2) and the
  rest) against the padded product;
- the 998244353 single product 1000 x 1500 (r = 2499) latency;
- `roofline` for the kernel with the largest share of the step (found in the
  last warm-up step, which times every launch), from HIP events recorded
  around each of its launches during the timed steps; `kernels` is the
  warm-up step's table;
- `cpu_baseline`: the oracle (textbook padded FFT and its inverse, one core)
  on one length of the sweep.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TFT+ITFT Gbutterfly/s & HBM GB/s; batched mults/s + p99 latency vs plain"
SWEEP = [1 << 22, (1 << 22) + 1, 3 << 21, (1 << 23) - 1, 1 << 23]
HBM_PEAK_GBS = 8000.0
# VALU: 256 CUs x 4 SIMDs x 16 lanes = 64 32-bit lane operations per CU per
# clock at 2.4 GHz
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# 32-bit VALU operations of one butterfly mod 2^64 - 2^32 + 1 (64 x 64-bit
# product as four 32 x 32 + 64 multiply-adds, folding with 2^64 = 2^32 - 1 and
# 2^96 = -1, modular add and subtract), register moves not counted
OPS_PER_BUTTERFLY = 33
# the timed steps bracket the dominant kernel with HIP events in every
# TIMING_EVERY-th step (the first, the sixth, ...)
TIMING_EVERY = 5
ROW_KERNELS = ("row_fwd", "row_inv")
COL_KERNELS = ("col_fwd", "col_inv_short", "col_inv_long")


def nominal_butterflies(n: int) -> float:
    return (n / 2.0) * math.log2(n)


def pass_butterflies(kernel: str, n: int, plan: dict) -> float:
    """Nominal butterflies of one pass of the two-pass transform of length n:
    the rows take log2 W of the log2 n levels, the columns the rest; the two
    classes of inverse columns split the column share by their word counts."""
    if plan["kind"] != 1:
        return nominal_butterflies(n) if kernel.startswith("small") else 0.0
    lw = plan["logW"]
    total_levels = math.log2(n)
    if kernel in ROW_KERNELS:
        return (n / 2.0) * lw
    if kernel in COL_KERNELS:
        col = (n / 2.0) * max(total_levels - lw, 0.0)
        if kernel == "col_fwd":
            return col
        W, a, b = plan["W"], plan["a"], plan["b"]
        share = ((W - b) * a if kernel == "col_inv_short" else b * (a + 1)) / float(n)
        return col * share
    return 0.0


def pass_words(kernel: str, n: int, plan: dict) -> float:
    """Words one pass reads (and writes) once."""
    if plan["kind"] != 1:
        return float(n) if kernel.startswith("small") else 0.0
    if kernel in ROW_KERNELS or kernel == "col_fwd":
        return float(n)
    W, a, b = plan["W"], plan["a"], plan["b"]
    if kernel == "col_inv_short":
        return float((W - b) * a)
    if kernel == "col_inv_long":
        return float(b * (a + 1))
    if kernel == "last_inv":
        return float(W)
    return 0.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true", help="only the timed step, roofline and baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--no-autotune", action="store_true", help="plan with the built-in planner only")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the served Poisson stream")
    ap.add_argument("--plain-seconds", type=float, default=1.0, help="length of the plain FIFO comparison")
    ap.add_argument("--lengths", default="", help="comma list of transform lengths for the timed step instead of "
                    "the workload's five (for profiling other lengths; implies --no-extras --no-cpu)")
    ap.add_argument("--skip", default="", help="comma list of extras to skip: products,small,walk,sweep,batched,served,crt")
    return ap.parse_args()


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in ("tft_device.hpp", "tft_kernels.hpp"):
        with open(os.path.join(ROOT, "paper_1001_5272_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def event_time(fn, reps=5):
    import torch
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        s.record()
        fn()
        e.record()
        e.synchronize()
        ts.append(s.elapsed_time(e))
    ts.sort()
    return ts[len(ts) // 2]


def main():
    args = parse()
    global SWEEP
    if args.lengths:
        SWEEP = [int(x) for x in args.lengths.split(",") if x]
        args.no_extras = args.no_cpu = True
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1001_5272_amd import libtft

    dev = torch.device("cuda:0")
    p, g = synth.GOLDILOCKS
    ctx = libtft.Context(p, g, 0)
    print(f"[bench] inputs: {len(SWEEP)} lengths, p=2^64-2^32+1", file=sys.stderr, flush=True)
    host = {n: synth.residues(p, n, 2000 + i) for i, n in enumerate(SWEEP)}
    bufs = {n: torch.from_numpy(host[n]).to(dev) for n in SWEEP}
    torch.cuda.synchronize()

    # autotune each length (outside the timed steps): the plan cache then holds
    # the fastest column width per ceil(lg n)
    tuned = {}
    if not args.no_autotune:
        print("[bench] autotune", file=sys.stderr, flush=True)
        for n in SWEEP:
            tuned[n] = libtft.tft_autotune(ctx, n)["logW"]

    def step():
        for n in SWEEP:
            libtft.tft_forward(ctx, bufs[n])
            libtft.tft_inverse(ctx, bufs[n])

    # The last warm-up step times every launch (HIP events around each): its
    # kernel table and the dominant kernel.  Inside the timed region only the
    # dominant kernel's launches are bracketed, and only in every
    # TIMING_EVERY-th step: each bracketed launch adds two event records to the
    # stream, about 5 us of idle device each, so the step time carries a
    # fifth of the events the roofline needs.
    wstats = None
    for i in range(args.warmup):
        if i == args.warmup - 1:
            torch.cuda.synchronize()
            libtft.tft_timing_reset(ctx)
            libtft.tft_timing_enable(ctx, True)
        step()
    torch.cuda.synchronize()
    if args.warmup:
        libtft.tft_timing_enable(ctx, False)
        wstats = libtft.tft_timing_read(ctx)
        libtft.tft_timing_select(ctx, [max(wstats.items(), key=lambda kv: kv[1][1])[0]])
    libtft.tft_timing_reset(ctx)
    libtft.tft_timing_enable(ctx, False)
    bracketed = [i for i in range(args.steps) if i % TIMING_EVERY == 0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        libtft.tft_timing_enable(ctx, i % TIMING_EVERY == 0)
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    libtft.tft_timing_enable(ctx, False)
    kstats = libtft.tft_timing_read(ctx)
    libtft.tft_timing_select(ctx, None)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    bfly = sum(2 * nominal_butterflies(n) for n in SWEEP)
    words_per_step = sum(SWEEP)
    value = bfly / (ms_per_step * 1e-3) / 1e9
    # the round trip must restore the inputs exactly
    ok = all(np.array_equal(bufs[n].cpu().numpy(), host[n]) for n in SWEEP)
    if not ok:
        print("[bench] round trip did not restore the inputs", file=sys.stderr)
        sys.exit(1)

    # ---- roofline of the dominant kernel (live HIP events over the timed steps)
    dom = max(kstats.items(), key=lambda kv: kv[1][1])
    dname, (dcount, dms) = dom
    avg_ms = dms / dcount
    launches_per_step = dcount / len(bracketed)
    plans = {n: libtft.tft_plan_info(ctx, n) for n in SWEEP}
    # Algorithmic work of one launch: the butterflies of the pass it runs
    # (the nominal count split between the passes by their tree depth) and
    # the words it must read and write once, averaged over the step.
    bf_step = sum(pass_butterflies(dname, n, plans[n]) for n in SWEEP)
    words_step = sum(pass_words(dname, n, plans[n]) for n in SWEEP)
    bf_launch = bf_step / launches_per_step
    alu_achieved = bf_launch * OPS_PER_BUTTERFLY / (avg_ms * 1e-3) / 1e12
    hbm_bytes = 2 * 8 * words_step / launches_per_step
    hbm_achieved = hbm_bytes / (avg_ms * 1e-3) / 1e9
    roofline = {
        "kernel": dname, "bound": "alu", "achieved": round(alu_achieved, 2), "peak": round(VALU_PEAK_TOPS, 1),
        "unit": "Tops/s", "frac": round(alu_achieved / VALU_PEAK_TOPS, 4), "traffic": None,
        "ops_per_butterfly": OPS_PER_BUTTERFLY, "butterflies_per_launch": int(bf_launch),
        "avg_launch_us": round(avg_ms * 1e3, 2), "launches": dcount, "bracketed_steps": len(bracketed),
        "hbm": {"achieved": round(hbm_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_achieved / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": int(hbm_bytes)},
        # the whole TFT+ITFT step: algorithmic bytes (each of the n words read
        # and written once per transform) over the step time
        "step_hbm": {"achieved": round(4 * 8 * words_per_step / (ms_per_step * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(4 * 8 * words_per_step / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "alg_bytes_per_step": 4 * 8 * words_per_step},
    }
    # the same device's register-only and copy-only ceilings (outside the timed steps)
    try:
        cal = libtft.tft_calibrate(ctx)
        bf_rate = bf_launch / (avg_ms * 1e-3) / 1e9
        roofline["device_measured"] = {k: round(v, 2) for k, v in cal.items()}
        roofline["achieved_gbutterfly_s"] = round(bf_rate, 1)
        roofline["frac_of_register_butterflies"] = round(bf_rate / cal["butterflies_g"], 4)
        roofline["hbm"]["frac_of_copy"] = round(hbm_achieved / cal["copy_gbs"], 4)
    except Exception as ex:   # calibration is reported, never required
        roofline["device_measured"] = {"error": str(ex)}
    pmc_path = os.path.join(ROOT, "profiles", f"pmc_{dname}_goldilocks_sweep.json")
    if os.path.exists(pmc_path):
        try:
            pm = json.load(open(pmc_path))
            if pm.get("kernel_src_sha") == kernel_source_sha():
                roofline["traffic"] = pm.get("hbm_bytes_per_launch")
        except Exception:
            pass
    table = wstats or kstats   # every kernel of one step (the last warm-up step)
    per_kernel = {k: {"launches": c, "avg_us": round(ms * 1e3 / c, 2), "share": round(ms / sum(v[1] for v in table.values()), 3)}
                  for k, (c, ms) in table.items()}

    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Gbutterfly/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "inplace TFT+ITFT sweep, p=2^64-2^32+1, n in {2^22, 2^22+1, 3*2^21, 2^23-1, 2^23}"
                   if not args.lengths else f"inplace TFT+ITFT, p=2^64-2^32+1, n in {SWEEP}",
                   "prime": p, "generator": g, "lengths": SWEEP, "word_bytes": 8,
                   "algorithmic_hbm_gbs": round(4 * 8 * words_per_step / (ms_per_step * 1e-3) / 1e9, 1),
                   "plans": {str(n): libtft.tft_plan_info(ctx, n)["logW"] for n in SWEEP},
                   "autotuned": not args.no_autotune},
        "roofline": roofline,
        "kernels": per_kernel,
    }

    if not args.no_extras:
        skip = set(x for x in args.skip.split(",") if x)
        result.update(extras(ctx, bufs, host, p, skip))
        if "sweep" not in skip:
            result["sweep"] = length_sweep(ctx, p, autotune=not args.no_autotune)
        if "batched" not in skip:
            result["batched"] = batched_c3()
        if "served" not in skip:
            result["served"] = served_c4(ctx, args.serve_seconds, args.plain_seconds)
        if "crt" not in skip:
            result["crt"] = crt_c5()

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(p, g, host)

    print(json.dumps(result), flush=True)
    ctx.close()


def extras(ctx, bufs, host, p, skip=frozenset()):
    import numpy as np
    import torch

    import synth
    from paper_1001_5272_amd import libtft

    dev = bufs[SWEEP[0]].device
    out = {}
    per = []
    print("[bench] per-length and padded comparator", file=sys.stderr, flush=True)
    pad = torch.empty(max(1 << (n - 1).bit_length() for n in SWEEP), dtype=torch.uint64, device=dev)
    for n in SWEEP:
        X = bufs[n]
        tf = event_time(lambda: libtft.tft_forward(ctx, X), 7)
        ti = event_time(lambda: libtft.tft_inverse(ctx, X), 7)
        # restore (forward then inverse leaves X as it was only in pairs)
        X.copy_(torch.from_numpy(host[n]).to(dev))
        tpf = event_time(lambda: libtft.tft_padded_forward(ctx, X, pad), 7)
        tpi = event_time(lambda: libtft.tft_padded_inverse(ctx, X, pad), 7)
        X.copy_(torch.from_numpy(host[n]).to(dev))
        # van der Hoeven-style buffered comparator: the same transform in a
        # 2^ceil(lg n)-word buffer
        L = 1 << (n - 1).bit_length()
        pad[:n].copy_(X)
        tbf = event_time(lambda: libtft.tft_buffered_forward(ctx, pad[:L], n), 7)
        tbi = event_time(lambda: libtft.tft_buffered_inverse(ctx, pad[:L], n), 7)
        plan = libtft.tft_plan_info(ctx, n)
        per.append({"n": n, "fwd_us": round(tf * 1e3, 1), "inv_us": round(ti * 1e3, 1),
                    "tft_itft_us": round((tf + ti) * 1e3, 1),
                    "gbfly_s": round(2 * nominal_butterflies(n) / ((tf + ti) * 1e-3) / 1e9, 2),
                    "padded_fwd_us": round(tpf * 1e3, 1), "padded_inv_us": round(tpi * 1e3, 1),
                    "buffered_fwd_us": round(tbf * 1e3, 1), "buffered_inv_us": round(tbi * 1e3, 1),
                    "buffered_mem_bytes": 8 * L,
                    "logW": plan["logW"], "a": plan["a"], "b": plan["b"],
                    "mem_bytes": 8 * n, "padded_mem_bytes": 8 * (n + (1 << (n - 1).bit_length()))})
    out["per_length"] = per
    t = {d["n"]: d["tft_itft_us"] for d in per}
    tp = {d["n"]: d["padded_fwd_us"] + d["padded_inv_us"] for d in per}
    out["jump"] = {"tft_ratio_2^22+1_over_2^22": round(t[SWEEP[1]] / t[SWEEP[0]], 3),
                   "padded_ratio_2^22+1_over_2^22": round(tp[SWEEP[1]] / tp[SWEEP[0]], 3)}

    if "products" not in skip:
        out["poly_mul"] = products(ctx, p, dev)
    if "small" not in skip:
        out["small_c1"] = small_c1(dev)
    if "walk" not in skip:
        out["walk_vs_batch"] = walk_vs_batch(ctx, p)
    return out


def restricted_fold_passes(r, word_bytes=8):
    """Fold passes over A and B of poly_mul_restricted at product length r:
    one per step with at least 2^18 positions left, then one per node (two,
    or ceil(t / S) single-workgroup nodes of S words when t < 2S); and the
    same count for the step-by-step schedule (one per block, plus the last
    point)."""
    small = 1 << (13 if word_bytes == 4 else 12)
    q = passes = 0
    while r - q >= 1 << 18:
        L = 1 << ((r - q).bit_length() - 2)
        q += L
        passes += 1
    t = r - q
    passes += -(-t // small) if t < 2 * small else 2
    q = literal = 0
    while q + 1 < r:
        q += 1 << ((r - q).bit_length() - 2)
        literal += 1
    return passes, literal + (1 if q < r else 0)


def products(ctx, p, dev):
    """poly_mul at product lengths r of the sweep against the padded product."""
    import torch

    import synth
    from paper_1001_5272_amd import libtft
    print("[bench] products", file=sys.stderr, flush=True)
    prods = []
    for r in SWEEP:
        la = (r + 2) // 2
        lb = r + 1 - la
        A = torch.from_numpy(synth.residues(p, la, 3000 + r)).to(dev)
        B = torch.from_numpy(synth.residues(p, lb, 4000 + r)).to(dev)
        X = torch.empty(r, dtype=torch.uint64, device=dev)
        Y = torch.empty(r, dtype=torch.uint64, device=dev)
        tm = event_time(lambda: libtft.poly_mul(ctx, A, B, X, Y), 5)
        N = 1 << (r - 1).bit_length()
        Ap = torch.empty(N, dtype=torch.uint64, device=dev)
        Bp = torch.empty(N, dtype=torch.uint64, device=dev)
        X2 = torch.empty(r, dtype=torch.uint64, device=dev)
        tpm = event_time(lambda: libtft.poly_mul_padded(ctx, A, B, X2, Ap, Bp), 5)
        same = bool(torch.equal(X, X2))
        X3 = torch.empty(r, dtype=torch.uint64, device=dev)
        trm = event_time(lambda: libtft.poly_mul_restricted(ctx, A, B, X3), 3)
        same_r = bool(torch.equal(X, X3))
        passes, literal = restricted_fold_passes(r)
        prods.append({"r": r, "poly_mul_us": round(tm * 1e3, 1), "padded_mul_us": round(tpm * 1e3, 1),
                      "restricted_mul_us": round(trm * 1e3, 1), "restricted_over_poly_mul": round(trm / tm, 2),
                      "mults_per_s": round(1e3 / tm, 1), "same_as_padded": same, "restricted_same": same_r,
                      "written_words": {"poly_mul": 2 * r, "restricted": r, "padded": 2 * N + r},
                      # every fold pass reads both operands once
                      "restricted_fold_reads": {"passes": passes, "bytes": passes * (la + lb) * 8,
                                                "step_by_step_passes": literal,
                                                "step_by_step_bytes": literal * (la + lb) * 8}})
        del X3
        del Ap, Bp, X2
    return prods


def walk_vs_batch(ctx, p):
    """The paper's Algorithm 1 run literally, one wavefront per instance
    (tft_walk_batch), against the layer-parallel small-instance kernel of the
    batched path, on batches of short instances (kernel time from HIP events;
    both give the same outputs)."""
    import numpy as np
    import torch

    import synth
    from paper_1001_5272_amd import libtft

    print("[bench] walk vs batch", file=sys.stderr, flush=True)
    rows = []
    for lo, hi, count in [(8, 64, 16384), (32, 256, 16384), (256, 1024, 4096)]:
        ns = synth.log_uniform_lengths(lo, hi, count, 6000).astype(np.int64)
        base = torch.from_numpy(synth.residues(p, int(ns.sum()), 6001)).cuda()
        offs = np.concatenate([[0], np.cumsum(ns)[:-1]])
        xs = [base[o:o + n] for o, n in zip(offs, ns)]
        ref = base.clone()
        us = {}
        outs = {}
        for name, fn in [("walk", lambda: libtft.tft_walk_batch(ctx, xs)),
                         ("batch", lambda: libtft.tft_forward_batch(ctx, xs))]:
            base.copy_(ref)
            fn()
            torch.cuda.synchronize()
            outs[name] = base.clone()
            libtft.tft_timing_reset(ctx)
            libtft.tft_timing_enable(ctx, True)
            for _ in range(3):
                base.copy_(ref)
                fn()
            torch.cuda.synchronize()
            t = libtft.tft_timing_read(ctx)
            libtft.tft_timing_enable(ctx, False)
            us[name] = round(t["small_list"][1] * 1e3 / t["small_list"][0], 1)
        base.copy_(ref)
        rows.append({"lengths": f"log-uniform [{lo}, {hi})", "instances": count, "words": int(ns.sum()),
                     "walk_kernel_us": us["walk"], "batch_kernel_us": us["batch"],
                     "walk_over_batch": round(us["walk"] / us["batch"], 2),
                     "same_outputs": bool(torch.equal(outs["walk"], outs["batch"]))})
    return {"workload": "forward TFT of batches of short instances, p=2^64-2^32+1 (seed 6001)", "rows": rows}


def small_c1(dev):
    """Configuration 1: the 998244353 product 1000 x 1500 (launch-bound)."""
    import torch

    import synth
    from paper_1001_5272_amd import libtft
    print("[bench] small product latency", file=sys.stderr, flush=True)
    p1, g1 = synth.P998
    c1 = libtft.Context(p1, g1, 0)
    A = torch.from_numpy(synth.residues_u32(p1, 1000, 1001)).to(dev)
    B = torch.from_numpy(synth.residues_u32(p1, 1500, 1002)).to(dev)
    X = torch.empty(2499, dtype=torch.uint32, device=dev)
    Y = torch.empty(2499, dtype=torch.uint32, device=dev)
    lat = []
    for i in range(110):
        torch.cuda.synchronize()
        s = time.perf_counter()
        libtft.poly_mul(c1, A, B, X, Y)
        torch.cuda.synchronize()
        if i >= 10:
            lat.append((time.perf_counter() - s) * 1e6)
    lat.sort()
    F = torch.from_numpy(synth.residues_u32(p1, 2499, 1)).to(dev)
    rt = event_time(lambda: (libtft.tft_forward(c1, F), libtft.tft_inverse(c1, F)), 21)
    res = {"workload": "998244353, 1000 x 1500 -> r=2499", "poly_mul_p50_us": round(lat[len(lat) // 2], 1),
           "poly_mul_p99_us": round(lat[int(len(lat) * 0.99) - 1], 1),
           "tft_itft_roundtrip_us": round(rt * 1e3, 1)}
    c1.close()
    return res


def length_sweep(ctx, p, per_octave=16, autotune=True):
    """TFT+ITFT time at lengths spread through [2^21, 2^23] (the jump-free
    curve) next to the padded comparator; the summary gives the mean rate,
    the largest time step between adjacent lengths and the lengths where the
    padded comparator is faster."""
    import torch

    import synth
    from paper_1001_5272_amd import libtft
    print("[bench] length sweep", file=sys.stderr, flush=True)
    ns = sorted({int(round(2 ** (21 + i / per_octave))) for i in range(2 * per_octave + 1)} |
                {(1 << 22) - 1, (1 << 22) + 1, (1 << 21) + 1})
    # the library's tuning as a user would apply it: every plan-cache bucket
    # the sweep meets (a quarter octave, or a power of two's own slot) is
    # autotuned once, at the middle one of its sweep lengths; buckets the timed
    # step already tuned keep their plans
    tuned = {}
    if autotune:
        members = {}
        for n in ns:
            members.setdefault(libtft.tft_plan_bucket(n), []).append(n)
        for bk, group in sorted(members.items()):
            if libtft.tft_plan_cache_get(ctx, bk):
                tuned[bk] = "kept"
                continue
            rep = group[len(group) // 2]
            libtft.tft_autotune(ctx, rep)
            tuned[bk] = rep
    pad = torch.empty(1 << 23, dtype=torch.uint64, device="cuda")
    out = []
    for n in ns:
        X = torch.from_numpy(synth.residues(p, n, 7000 + n % 9973)).cuda()
        t = event_time(lambda: (libtft.tft_forward(ctx, X), libtft.tft_inverse(ctx, X)), 5)
        tp = event_time(lambda: (libtft.tft_padded_forward(ctx, X, pad), libtft.tft_padded_inverse(ctx, X, pad)), 5)
        L = 1 << (n - 1).bit_length()
        pad[:n].copy_(X)
        tb = event_time(lambda: (libtft.tft_buffered_forward(ctx, pad[:L], n),
                                 libtft.tft_buffered_inverse(ctx, pad[:L], n)), 5)
        out.append({"n": n, "logW": libtft.tft_plan_info(ctx, n)["logW"],
                    "tft_itft_us": round(t * 1e3, 1), "padded_us": round(tp * 1e3, 1),
                    "buffered_us": round(tb * 1e3, 1), "mem_words": n, "padded_mem_words": n + L,
                    "buffered_mem_words": L,
                    "gbfly_s": round(2 * nominal_butterflies(n) / (t * 1e-3) / 1e9, 1)})
        del X
    steps = [(b["tft_itft_us"] / a["tft_itft_us"], a["n"], b["n"]) for a, b in zip(out, out[1:])]
    worst = max(steps)
    summary = {"points": len(out), "autotuned_quarter_octaves": {str(k): v for k, v in sorted(tuned.items())},
               "mean_gbfly_s": round(sum(d["gbfly_s"] for d in out) / len(out), 1),
               "max_adjacent_step": {"ratio": round(worst[0], 3), "from_n": worst[1], "to_n": worst[2]},
               "slower_than_padded": [d["n"] for d in out if d["tft_itft_us"] > d["padded_us"]]}
    return {"points": out, "summary": summary}


def batched_c3():
    """4096 independent products mod 998244353, operand lengths log-uniform in
    [32, 32768]: one planned batch replayed as a HIP graph, against one plain
    poly_mul launch sequence per instance on the same stream."""
    import numpy as np
    import torch

    import synth
    from paper_1001_5272_amd import libtft
    print("[bench] batched 4096 products (998244353)", file=sys.stderr, flush=True)
    p, g = synth.P998
    ctx = libtft.Context(p, g, 0)
    count = 4096
    la = synth.log_uniform_lengths(32, 32768, count, 3001)
    lb = synth.log_uniform_lengths(32, 32768, count, 3002)
    total = int((la + lb - 1).sum())
    # operands resident in HBM: one flat buffer per role, sliced per instance
    Aall = torch.from_numpy(synth.residues_u32(p, int(la.sum()), 3003)).cuda()
    Ball = torch.from_numpy(synth.residues_u32(p, int(lb.sum()), 3004)).cuda()
    Xall = torch.zeros(total, dtype=torch.uint32, device="cuda")
    Yall = torch.zeros(total, dtype=torch.uint32, device="cuda")
    X2all = torch.zeros(total, dtype=torch.uint32, device="cuda")
    jobs, plain = [], []
    oa = ob = ox = 0
    for i in range(count):
        a, b = int(la[i]), int(lb[i])
        r = a + b - 1
        A, B = Aall[oa:oa + a], Ball[ob:ob + b]
        jobs.append((A, B, Xall[ox:ox + r], Yall[ox:ox + r]))
        plain.append((A, B, X2all[ox:ox + r], Yall[ox:ox + r]))
        oa, ob, ox = oa + a, ob + b, ox + r
    t0 = time.perf_counter()
    batch = libtft.Batch(ctx, jobs)
    plan_ms = (time.perf_counter() - t0) * 1e3
    info = batch.info()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.run()
    graph.replay()
    torch.cuda.synchronize()
    reps = 10
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        graph.replay()
    ev1.record()
    ev1.synchronize()
    t_graph = ev0.elapsed_time(ev1) / reps
    ev0.record()
    for _ in range(3):
        batch.run()
    ev1.record()
    ev1.synchronize()
    t_run = ev0.elapsed_time(ev1) / 3

    def run_plain():
        for A, B, X, Y in plain:
            libtft.poly_mul(ctx, A, B, X, Y)
    run_plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_plain()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) * 1e3
    same = bool(torch.equal(Xall, X2all))
    batch.close()
    # the batch tuner: rows of the two-pass instances at the balanced split, one
    # step wider (the default above) or two steps wider, then the column-list
    # and fused-row workgroup sizes; fastest kept
    Xall.zero_()
    widen = libtft.tft_autotune_batch(ctx, jobs)
    tuning = libtft.tft_batch_tuning_get(ctx)
    tuned_batch = libtft.Batch(ctx, jobs)
    with torch.cuda.stream(s):
        tuned_batch.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph2):
        tuned_batch.run()
    graph2.replay()
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        graph2.replay()
    ev1.record()
    ev1.synchronize()
    t_tuned = ev0.elapsed_time(ev1) / reps
    same_tuned = bool(torch.equal(Xall, X2all))
    tuned_batch.close()
    ctx.close()
    return {"workload": "4096 products mod 998244353, la, lb log-uniform [32, 32768] (seeds 3001, 3002)",
            "total_output_words": total, "batch": info, "plan_ms": round(plan_ms, 1),
            "graph_ms": round(t_graph, 3), "run_ms": round(t_run, 3), "plain_ms": round(t_plain, 3),
            "mults_per_s_graph": round(count / (t_graph * 1e-3), 0), "mults_per_s_plain": round(count / (t_plain * 1e-3), 0),
            "speedup_vs_plain": round(t_plain / t_graph, 2), "batched_equals_plain": same,
            "tuned": {"rows_wider_than_balanced": widen, "list_col_threads": tuning["list_col_threads"],
                      "row_mul_threads": tuning["row_mul_threads"], "graph_ms": round(t_tuned, 3),
                      "mults_per_s_graph": round(count / (t_tuned * 1e-3), 0), "batched_equals_plain": same_tuned},
            # algorithmic bytes of a product: three transforms (each word read
            # and written once) plus the pointwise read of Y: 7 r words
            "hbm": {"alg_bytes": 7 * 4 * total, "achieved_gbs": round(7 * 4 * total / (t_graph * 1e-3) / 1e9, 1),
                    "frac": round(7 * 4 * total / (t_graph * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}


def served_stream(ctx, q, rate, seconds, seed, pool, ring, verify=0):
    """One Poisson stream of products mod 2^64-2^32+1 through the queue: r
    log-uniform in [2^8, 2^22], split la = ceil((r+1)/2), lb = r+1-la; the
    operands of request i are windows of the resident random array `pool` at
    seeded offsets (so every request multiplies its own polynomials) and its
    output a window of the ring buffer `ring`, reused in order once the
    request that held it has completed.  Latency runs from the scheduled
    arrival to the completion seen by the queue's worker.  A submit refused for
    footprint (TFT_EAGAIN) is retried after the oldest outstanding request
    completes.  verify: the last `verify` requests are recomputed with
    poly_mul (GPU, outside the timings) and compared word for word."""
    import numpy as np
    import torch

    import synth
    from paper_1001_5272_amd import libtft
    arrivals = synth.poisson_arrivals(rate, seconds, seed)
    cnt = len(arrivals)
    rs = synth.log_uniform_lengths(1 << 8, 1 << 22, cnt, seed + 1)
    la = (rs + 2) // 2
    lb = rs + 1 - la
    P = pool.numel()
    offa = (synth.uniform01(cnt, seed + 2) * (P - la)).astype(np.int64)
    offb = (synth.uniform01(cnt, seed + 3) * (P - lb)).astype(np.int64)
    R = ring.numel()
    # output windows: consecutive in the ring, wrapping to 0 when one would cross the end
    outs = np.zeros(cnt, dtype=np.int64)
    cur = 0
    for i in range(cnt):
        if cur + rs[i] > R:
            cur = 0
        outs[i] = cur
        cur += int(rs[i])
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()   # the client's collection pauses would delay every arrival in their window
    base = time.monotonic_ns() + 20_000_000
    tickets = [0] * cnt
    t_arr = (base + (arrivals * 1e9).astype(np.int64)).tolist()
    outstanding = []     # (ticket, lo, hi) in submission order
    head = 0
    retries = ring_waits = 0
    for i in range(cnt):
        lo, hi = int(outs[i]), int(outs[i] + rs[i])
        # the ring window must be free: wait for earlier requests whose window overlaps it
        while head < len(outstanding):
            t0, l0, h0 = outstanding[head]
            if h0 <= lo or l0 >= hi:
                if q.poll(t0):
                    head += 1
                    continue
                break
            if not q.poll(t0):
                ring_waits += 1
                q.wait(t0)
            head += 1
        while time.monotonic_ns() < t_arr[i]:
            pass
        A = pool[int(offa[i]):int(offa[i] + la[i])]
        B = pool[int(offb[i]):int(offb[i] + lb[i])]
        X = ring[lo:hi]
        t = q.try_submit(A, B, X)
        while t is None:
            retries += 1
            k = head
            while k < len(outstanding) and q.poll(outstanding[k][0]):
                k += 1
            if k < len(outstanding):
                q.wait(outstanding[k][0])
            t = q.try_submit(A, B, X)
        tickets[i] = t
        outstanding.append((t, lo, hi))
    for t in tickets:
        q.wait(t)
    gc.enable()
    done = np.array([q.completion_ns(t) for t in tickets], dtype=np.int64)
    end = int(done.max())
    lat = (done - np.array(t_arr, dtype=np.int64)) / 1e3
    res = {"rate_offered": rate, "requests": cnt, "duration_s": round((end - base) / 1e9, 3),
           "mults_per_s": round(cnt / ((end - base) / 1e9), 1),
           "p50_us": round(float(np.percentile(lat, 50)), 1), "p99_us": round(float(np.percentile(lat, 99)), 1),
           "mean_r": int(rs.mean()), "footprint_retries": retries, "ring_waits": ring_waits}
    if verify:
        # the last `verify` requests' windows are intact (no later request reused them)
        Y = torch.empty(1 << 22, dtype=torch.uint64, device=ring.device)
        Z = torch.empty(1 << 22, dtype=torch.uint64, device=ring.device)
        same, checked, words = True, 0, 0
        lo_all = None
        for i in range(cnt - 1, -1, -1):
            lo, hi = int(outs[i]), int(outs[i] + rs[i])
            if lo_all is not None and not (hi <= lo_all[0] or lo >= lo_all[1]):
                break        # overwritten by a later request
            r = int(rs[i])
            libtft.poly_mul(ctx, pool[int(offa[i]):int(offa[i] + la[i])], pool[int(offb[i]):int(offb[i] + lb[i])],
                            Z[:r], Y[:r])
            same &= bool(torch.equal(ring[lo:hi], Z[:r]))
            checked += 1
            words += r
            lo_all = (lo, hi) if lo_all is None else (min(lo_all[0], lo), max(lo_all[1], hi))
            if checked >= verify:
                break
        torch.cuda.synchronize()
        res["outputs_checked"] = checked
        res["words_checked"] = words
        res["served_equals_plain"] = same
    return res


def served_c4(ctx, seconds, plain_seconds, capacity=True):
    """Config 4: a Poisson stream (mean 20k requests/s) of products mod
    2^64-2^32+1, r log-uniform in [2^8, 2^22], operands resident in HBM, the
    queue admitting by in-place footprint; then the same stream served one
    request at a time (plain FIFO: poly_mul + wait); then the served capacity:
    the highest offered rate of a short stream that the queue holds at
    p99 < 2 ms, and the throughput it reaches when offered more than it can
    serve."""
    import numpy as np
    import torch

    import synth
    from paper_1001_5272_amd import libtft
    p = synth.GOLDILOCKS[0]
    print(f"[bench] served stream {seconds} s", file=sys.stderr, flush=True)
    pool = torch.from_numpy(synth.residues(p, 1 << 26, 4100)).cuda()   # 512 MiB of operand words
    ring = torch.empty(1 << 27, dtype=torch.uint64, device="cuda")     # 1 GiB of output windows
    q = libtft.Queue(ctx, 1 << 28, 4096)                               # 2 GiB of workspace
    served = served_stream(ctx, q, 20000.0, seconds, 4001, pool, ring, verify=256)
    st = q.stats()
    served.update({"batches": st["batches"], "rejected": st["rejected"], "pool_words": st["pool_words"],
                   "pool_used_max": st["pool_used_max"]})
    cap = None
    if capacity:
        print("[bench] served capacity", file=sys.stderr, flush=True)
        cap = {"criterion": "2 s Poisson streams at increasing offered rates, each after a 1 s warm-up "
                            "stream at the same rate (not counted)", "runs": []}
        held = None
        for rate in (10000.0, 15000.0, 20000.0, 30000.0, 40000.0, 60000.0):
            served_stream(ctx, q, rate, 1.0, 4400 + int(rate) // 1000, pool, ring)
            r = served_stream(ctx, q, rate, 2.0, 4500 + int(rate) // 1000, pool, ring)
            cap["runs"].append({k: r[k] for k in ("rate_offered", "mults_per_s", "p50_us", "p99_us")})
            if r["p99_us"] < 2000.0:
                held = rate
        cap["highest_rate_at_p99_below_2ms"] = held
        cap["saturation_mults_per_s"] = max(x["mults_per_s"] for x in cap["runs"])
    q.close()
    # plain FIFO path on a prefix of the same stream (same operands)
    print(f"[bench] plain FIFO stream {plain_seconds} s", file=sys.stderr, flush=True)
    arrivals = synth.poisson_arrivals(20000.0, seconds, 4001)
    sub = arrivals[arrivals < plain_seconds]
    cnt = len(sub)
    rs = synth.log_uniform_lengths(1 << 8, 1 << 22, len(arrivals), 4002)[:cnt]
    la = (rs + 2) // 2
    lb = rs + 1 - la
    P = pool.numel()
    offa = (synth.uniform01(len(arrivals), 4003)[:cnt] * (P - la)).astype(np.int64)
    offb = (synth.uniform01(len(arrivals), 4004)[:cnt] * (P - lb)).astype(np.int64)
    Y = torch.empty(1 << 22, dtype=torch.uint64, device="cuda")
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    base = time.monotonic_ns() + 20_000_000
    lat_p = []
    for i, ta in enumerate(sub.tolist()):
        r = int(rs[i])
        t_arr = base + int(ta * 1e9)
        while time.monotonic_ns() < t_arr:
            pass
        libtft.poly_mul(ctx, pool[int(offa[i]):int(offa[i] + la[i])], pool[int(offb[i]):int(offb[i] + lb[i])],
                        ring[:r], Y[:r])
        torch.cuda.synchronize()
        lat_p.append((time.monotonic_ns() - t_arr) / 1e3)
    end_p = time.monotonic_ns()
    gc.enable()
    lat_p = np.array(lat_p)
    plain = {"requests": cnt, "duration_s": round((end_p - base) / 1e9, 3),
             "mults_per_s": round(cnt / ((end_p - base) / 1e9), 1),
             "p50_us": round(float(np.percentile(lat_p, 50)), 1), "p99_us": round(float(np.percentile(lat_p, 99)), 1)}
    del pool, ring
    torch.cuda.empty_cache()
    out = {"workload": f"Poisson 20k req/s for {seconds} s, p=2^64-2^32+1, r log-uniform [2^8, 2^22], "
                       "operands: windows of a resident 2^26-word random array at seeded offsets (every request "
                       "its own pair)", "served": served, "plain_fifo": plain}
    if cap is not None:
        out["capacity"] = cap
    return out


def crt_c5():
    """Exact product of two length-(2^24+12345) polynomials with signed 24-bit
    coefficients through the primes 2013265921, 469762049, 1811939329 and CRT
    to int128; timed per prime and for the CRT, with sampled exact checks."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_1001_5272_amd import libtft
    print("[bench] exact integer product via 3 primes", file=sys.stderr, flush=True)
    n = (1 << 24) + 12345
    r = 2 * n - 1
    a = synth.signed24(n, 5001)
    b = synth.signed24(n, 5002)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    ctxs = [libtft.Context(pp, gg) for pp, gg in synth.CRT_PRIMES]
    A = torch.empty(n, dtype=torch.uint32, device="cuda")
    B = torch.empty(n, dtype=torch.uint32, device="cuda")
    Y = torch.empty(r, dtype=torch.uint32, device="cuda")
    Xs = [torch.empty(r, dtype=torch.uint32, device="cuda") for _ in range(3)]
    out = torch.empty(2 * r, dtype=torch.int64, device="cuda")

    def run():
        per = []
        for c, X in zip(ctxs, Xs):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            libtft.tft_from_signed(c, da, A)
            libtft.tft_from_signed(c, db, B)
            libtft.poly_mul(c, A, B, X, Y)
            e1.record()
            per.append((e0, e1))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        libtft.tft_crt3(ctxs, Xs[0], Xs[1], Xs[2], out)
        e1.record()
        e1.synchronize()
        return [s.elapsed_time(e) for s, e in per], e0.elapsed_time(e1)

    run()
    per, tcrt = run()
    got = out.cpu().numpy().view(np.uint64)
    checks = 0
    for s in [0, 1, r // 3, r // 2, r - 2, r - 1]:
        v = (int(got[2 * s + 1]) << 64) | int(got[2 * s])
        if v >= 1 << 127:
            v -= 1 << 128
        assert v == oracle.conv_coeff_i128(a, b, s), s
        checks += 1
    for c in ctxs:
        c.close()
    total = sum(per) + tcrt
    N = 1 << (r - 1).bit_length()
    return {"workload": "signed 24-bit, both lengths 2^24+12345, primes 2013265921, 469762049, 1811939329 "
                        "(1811939329 replaces 998244353, whose 2-adic order 23 is too small for r > 2^23)",
            "r": r, "per_prime_ms": [round(x, 3) for x in per], "crt_ms": round(tcrt, 3), "total_ms": round(total, 3),
            "coeffs_per_s": round(r / (total * 1e-3), 0),
            "inplace_bytes_per_prime": 4 * (2 * n + 2 * r), "padded_bytes_per_prime": 4 * (2 * n + 2 * N),
            "sampled_exact_checks": checks}


def cpu_baseline(p, g, host):
    """CPU timings on this host, beside the GPU numbers (reported baselines,
    not targets):

    - value: the oracle as it stands -- its textbook padded radix-2 FFT and the
      inverse, one thread, at 2^22 and 2^23 (where padded and truncated
      transforms coincide);
    - plain_cpu_tft: the paper's Algorithms 1 and 2 with O(1) auxiliary space
      (oracle.tft_inplace / itft_inplace), one thread, forward + inverse at
      2^22 and 2^22 + 1;
    - c1_product: the 1000 x 1500 product mod 998244353 on one thread, by
      Algorithm 3 (the space-restricted product on Algorithms 1 and 2) and by
      the schoolbook definition;
    - c3_all_cores: the 4096 products of the batched workload by Algorithm 3,
      spread over every core this process may use (threads; the oracle
      releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    import synth
    t_all, bfly, parts = 0.0, 0.0, []
    for n in (SWEEP[0], SWEEP[4]):
        F = host[n]
        print(f"[bench] cpu baseline (oracle, n={n})", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        X = oracle.fft_padded(p, g, F)
        back = oracle.ifft_pow2(p, g, X)
        t1 = time.perf_counter()
        assert (back == F).all()
        t_all += t1 - t0
        bfly += 2 * nominal_butterflies(n)
        parts.append(f"n={n}: {t1 - t0:.2f} s")
    out = {"value": round(bfly / t_all / 1e9, 5), "unit": "Gbutterfly/s", "cores": 1, "kind": "oracle",
           "sample": "forward + inverse (textbook padded radix-2, one thread) at n=2^22 and n=2^23, "
                     "p=2^64-2^32+1; " + ", ".join(parts)}
    # the paper's in-place algorithms, one thread
    plain = {}
    for n in (SWEEP[0], SWEEP[1]):
        print(f"[bench] cpu baseline (Algorithms 1 and 2 in place, n={n})", file=sys.stderr, flush=True)
        F = host[n]
        t0 = time.perf_counter()
        X = oracle.tft_inplace(p, g, F)
        t1 = time.perf_counter()
        back = oracle.itft_inplace(p, g, X)
        t2 = time.perf_counter()
        assert (back == F).all()
        plain[str(n)] = {"fwd_s": round(t1 - t0, 3), "inv_s": round(t2 - t1, 3),
                         "gbfly_s": round(2 * nominal_butterflies(n) / (t2 - t0) / 1e9, 5)}
    out["plain_cpu_tft"] = {"kind": "Algorithms 1 and 2, O(1) auxiliary space", "cores": 1, "unit": "Gbutterfly/s",
                            "p": "2^64-2^32+1", "per_length": plain}
    # config 1 on one thread
    p1, g1 = synth.P998
    A = synth.residues(p1, 1000, 1001)
    B = synth.residues(p1, 1500, 1002)
    t0 = time.perf_counter()
    for _ in range(20):
        C = oracle.mul_restricted(p1, g1, A, B)
    t1 = time.perf_counter()
    C2 = oracle.mul_schoolbook(p1, A, B)
    t2 = time.perf_counter()
    assert (C == C2).all()
    out["c1_product"] = {"cores": 1, "algorithm3_us": round((t1 - t0) / 20 * 1e6, 1),
                         "schoolbook_us": round((t2 - t1) * 1e6, 1), "workload": "998244353, 1000 x 1500 -> r=2499"}
    # config 3 over every usable core
    count = 4096
    la = synth.log_uniform_lengths(32, 32768, count, 3001)
    lb = synth.log_uniform_lengths(32, 32768, count, 3002)
    pairs = [(synth.residues(p1, int(la[i]), 10_000 + 2 * i), synth.residues(p1, int(lb[i]), 10_001 + 2 * i))
             for i in range(count)]
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    print(f"[bench] cpu baseline (4096 products, Algorithm 3, {cores} threads)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        res = list(ex.map(lambda ab: oracle.mul_restricted(p1, g1, ab[0], ab[1]), pairs))
    t1 = time.perf_counter()
    assert len(res) == count
    out["c3_all_cores"] = {"kind": "Algorithm 3 (space-restricted product on Algorithms 1 and 2)", "cores": cores,
                           "products": count, "seconds": round(t1 - t0, 3),
                           "mults_per_s": round(count / (t1 - t0), 1),
                           "cpu_model": _cpu_model()}
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
