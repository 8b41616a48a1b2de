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
- `roofline` for the kernel with the largest share of the timed step, from
  HIP events recorded around each launch during the timed steps;
- `cpu_baseline`: the oracle (textbook padded FFT and its inverse, one core)
  on one length of the sweep.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
"""
from __future__ import annotations

import argparse
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
# VALU: 256 CUs x 4 SIMDs x 16 lanes = 64 lanes/CU/clk at 2.4 GHz
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def nominal_butterflies(n: int) -> float:
    return (n / 2.0) * math.log2(n)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true", help="only the timed step, roofline and baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
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
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
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

    def step():
        for n in SWEEP:
            libtft.tft_forward(ctx, bufs[n])
            libtft.tft_inverse(ctx, bufs[n])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    libtft.tft_timing_reset(ctx)
    libtft.tft_timing_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    libtft.tft_timing_enable(ctx, False)
    kstats = libtft.tft_timing_read(ctx)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    bfly = sum(2 * nominal_butterflies(n) for n in SWEEP)
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
    # every column/row kernel is one HBM pass: it reads and writes each of the
    # words it covers once.  Per timed step the sweep's words are covered once
    # by each pass, so bytes per launch = 2 * 8 * (sum n) / launches per step.
    words_per_step = sum(SWEEP)
    launches_per_step = dcount / args.steps
    alg_bytes = 2 * 8 * words_per_step / launches_per_step
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    roofline = {
        "kernel": dname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
        "avg_launch_us": round(avg_ms * 1e3, 2), "launches": dcount,
        "alg_bytes_per_launch": int(alg_bytes),
    }
    pmc_path = os.path.join(ROOT, "profiles", f"pmc_{dname}_goldilocks_sweep.json")
    if os.path.exists(pmc_path):
        try:
            pm = json.load(open(pmc_path))
            if pm.get("kernel_src_sha") == kernel_source_sha():
                roofline["traffic"] = pm.get("hbm_bytes_per_launch")
        except Exception:
            pass
    per_kernel = {k: {"launches": c, "avg_us": round(ms * 1e3 / c, 2), "share": round(ms / sum(v[1] for v in kstats.values()), 3)}
                  for k, (c, ms) in kstats.items()}

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
        "config": {"workload": "inplace TFT+ITFT sweep, p=2^64-2^32+1, n in {2^22, 2^22+1, 3*2^21, 2^23-1, 2^23}",
                   "prime": p, "generator": g, "lengths": SWEEP, "word_bytes": 8,
                   "algorithmic_hbm_gbs": round(4 * 8 * words_per_step / (ms_per_step * 1e-3) / 1e9, 1)},
        "roofline": roofline,
        "kernels": per_kernel,
    }

    if not args.no_extras:
        result.update(extras(ctx, bufs, host, p))

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(p, g, host)

    print(json.dumps(result), flush=True)
    ctx.close()


def extras(ctx, bufs, host, p):
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
        plan = libtft.tft_plan_info(ctx, n)
        per.append({"n": n, "fwd_us": round(tf * 1e3, 1), "inv_us": round(ti * 1e3, 1),
                    "tft_itft_us": round((tf + ti) * 1e3, 1),
                    "gbfly_s": round(2 * nominal_butterflies(n) / ((tf + ti) * 1e-3) / 1e9, 2),
                    "padded_fwd_us": round(tpf * 1e3, 1), "padded_inv_us": round(tpi * 1e3, 1),
                    "logW": plan["logW"], "a": plan["a"], "b": plan["b"],
                    "mem_bytes": 8 * n, "padded_mem_bytes": 8 * (n + (1 << (n - 1).bit_length()))})
    out["per_length"] = per
    t = {d["n"]: d["tft_itft_us"] for d in per}
    tp = {d["n"]: d["padded_fwd_us"] + d["padded_inv_us"] for d in per}
    out["jump"] = {"tft_ratio_2^22+1_over_2^22": round(t[SWEEP[1]] / t[SWEEP[0]], 3),
                   "padded_ratio_2^22+1_over_2^22": round(tp[SWEEP[1]] / tp[SWEEP[0]], 3)}

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
        prods.append({"r": r, "poly_mul_us": round(tm * 1e3, 1), "padded_mul_us": round(tpm * 1e3, 1),
                      "mults_per_s": round(1e3 / tm, 1), "same_as_padded": same})
        del Ap, Bp, X2
    out["poly_mul"] = prods

    # configuration 1: the small 998244353 product, launch-bound
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
    out["small_c1"] = {"workload": "998244353, 1000 x 1500 -> r=2499", "poly_mul_p50_us": round(lat[len(lat) // 2], 1),
                       "poly_mul_p99_us": round(lat[int(len(lat) * 0.99) - 1], 1),
                       "tft_itft_roundtrip_us": round(rt * 1e3, 1)}
    c1.close()
    return out


def cpu_baseline(p, g, host):
    """The oracle as it stands: its textbook padded radix-2 FFT and the
    inverse, on one core, at the two power-of-two lengths of the sweep
    (2^22 and 2^23), where the padded and truncated transforms coincide."""
    import oracle
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
    return {"value": round(bfly / t_all / 1e9, 5), "unit": "Gbutterfly/s", "cores": 1, "kind": "oracle",
            "sample": "forward + inverse (textbook padded radix-2, one thread) at n=2^22 and n=2^23, "
                      "p=2^64-2^32+1; " + ", ".join(parts)}


if __name__ == "__main__":
    main()
