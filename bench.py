#!/usr/bin/env python3
"""Benchmark: tokens analysed per second by the HIP FindRepeats path.

Workload (default): one window of n = 2^20 uint64 task-hash tokens, a nested
loop stream (outer body 200 tokens with an inner body of 30 tokens repeated
10 times, alphabet 2^16, 1% substitutions, 0.5% insertions), min repeat length
16.  One step = one complete analysis of the window (rank compression, suffix
array, LCP, candidates, sort, greedy selection, output) with the tokens
already resident in device memory.

Prints one JSON line (rank 0).  Runs on one GPU only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per entry of the doubling rounds' LDS sort-and-regroup
# kernel: read key + suffix (8), write the sorted suffix (4), write its new rank
# (4) and its rank snapshot for the LCP stage (4).
LDS_SA_BYTES_PER_ENTRY = 20
LDS_SA_TAG = 1


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="config1", choices=["config0", "config1", "config2"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many steps, no baseline (for profilers)")
    return ap.parse_args()


def workload(name):
    from paper_2406_18111_amd import synth
    if name == "config0":
        t, m = synth.config0()
        desc = "single window n=4096 u64, loop body 50 / alphabet 64, 5% substitutions, min_len 8"
    elif name == "config1":
        t, m = synth.config1()
        desc = ("single window n=2^20 u64, nested loop (outer 200, inner 30 x10), alphabet 2^16, "
                "1% substitutions + 0.5% insertions, min_len 16")
    else:
        t, m = synth.config2()
        desc = "single window n=2^24 u32, first half constant, second half uniform over 4 symbols, min_len 32"
    return t, m, desc


def cpu_baseline(t, m, seconds):
    import oracle
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.find_repeats(t, m)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": reps * len(t) / el, "unit": "tokens/s", "cores": 1, "kind": "oracle",
            "sample": "%d full analyses of the same window by the single-threaded C oracle (%.1f s)" % (reps, el)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only; multi-GPU runs are not part of this build "
              "(see DESIGN.md, 'Sharding').", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2406_18111_amd import Context
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    t, m, desc = workload(args.workload)
    n = len(t)
    dev = torch.from_numpy(t.view(np.int64) if t.dtype == np.uint64 else t.view(np.int32)).cuda()
    ctx = Context(0)
    steps = args.profile_steps or args.steps
    warm = 1 if args.profile_steps else args.warmup
    for _ in range(warm):
        ctx.analyze_dev(dev, m)
    torch.cuda.synchronize()
    stage_tot = None
    kprof = {"launches": 0, "ms": 0.0, "elems": 0}
    ctx.profile_kernel(LDS_SA_TAG)
    t0 = time.perf_counter()
    for _ in range(steps):
        rows, _ = ctx.analyze_dev(dev, m)
        st = ctx.stage_ms()
        stage_tot = st if stage_tot is None else {k: stage_tot[k] + v for k, v in st.items()}
        kp = ctx.kernel_profile()
        for k in kprof:
            kprof[k] += kp[k]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.profile_kernel(0)
    ms = el * 1e3 / steps
    value = n * steps / el
    counters = ctx.counters()
    out = {
        "metric": "tokens analyzed/sec (SA+LCP+repeat mining)",
        "value": value,
        "unit": "tokens/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if t.dtype == np.uint32 else "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": n, "min_len": m,
                   "windows": 1},
        "stage_ms": {k: v / steps for k, v in stage_tot.items()},
        "counters": counters,
        "rows": int(rows.shape[0]),
    }
    if kprof["launches"]:
        avg_ms = kprof["ms"] / kprof["launches"]
        bytes_per_launch = kprof["elems"] * LDS_SA_BYTES_PER_ENTRY / kprof["launches"]
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                           "kernel": "k_lds_sort<MODE_SA> (doubling rounds)",
                           "avg_launch_us": avg_ms * 1e3, "bytes_per_launch": bytes_per_launch,
                           "launches_per_step": kprof["launches"] / steps}
    if not args.profile_steps and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(t, m, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
