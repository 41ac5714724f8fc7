"""Benchmark: sessions/s of fused discrimination + millisecond histogram on one
MI355X, with the HBM roofline of the dominant kernel and the CPU oracle
timed beside it.

One step = one sinet_pipeline call over the whole resident day: clear the
4 x n_bins histogram, then one pass that reads every session's ts/src/dst/
bytes, looks both addresses up in the prefix table, writes the label and
merges (1, bytes) into its (label, 1-ms bin).  Inputs are synthetic (seeded
generator, written straight into HBM) with the paper's day shape.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2|4|5]
                    [--lookup bsearch|trie|pla|mlp|auto] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sessions/sec classify+histogram on 1 GPU, % HBM roofline; learned vs plain lookup"
HBM_PEAK_GBS = 8000.0
BYTES_PER_SESSION = 21   # ts 4 + src 4 + dst 4 + bytes 8 read, label 1 written
BYTES_PER_BIN = 64       # 4 labels x (count 8 + bytes 8) written once


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--n", type=int, default=0, help="override the session count")
    ap.add_argument("--lookup", default="")
    ap.add_argument("--compare", default="", help="comma list of extra lookups to time")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0)
    return ap.parse_args()


def time_calls(torch, fn, steps, warmup):
    """Average device ms per call, HIP events on the stream the library uses
    (torch's current stream), plus the host wall time of the whole loop."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(st)
        fn()
        b.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev = [a.elapsed_time(b) for a, b in evs]
    return sum(dev) / len(dev), min(dev), wall * 1e3 / steps


def cpu_baseline(wl, cols, sinet, sample: int):
    """The C oracle (single thread) on a contiguous sample of the same day."""
    import numpy as np
    import oracle
    n = min(sample, wl.n)
    i0 = (wl.n - n) // 2
    s = {k: (sinet.to_host_u64(v[i0:i0 + n]) if k == "bytes" else sinet.to_host_u32(v[i0:i0 + n]))
         for k, v in cols.items()}
    w = wl.window
    t = time.perf_counter()
    oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"], w.t0, w.width,
                    w.n_bins, mode="hash")
    dt = time.perf_counter() - t
    return {"value": n / dt, "unit": "sessions/s", "cores": 1, "kind": "oracle",
            "sample": f"sessions [{i0}, {i0 + n}) of the same day, per-length-hash LPM, "
                      f"full {w.n_bins}-bin x 4-label histogram cleared and filled; {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_2106_12863_amd as sinet
    import sinetgen
    import sinetgen.gpu as gg

    wl = sinetgen.config(args.config, n=args.n or None)
    lookup = args.lookup or ("pla" if args.config in (4, 5) else "bsearch")
    log(f"config {args.config}: {wl.name} n={wl.n} prefixes={wl.n_prefix} lookup={lookup}")
    cols = gg.alloc_and_fill(wl)
    torch.cuda.synchronize()
    w = wl.window
    label = torch.empty(wl.n, dtype=torch.uint8, device="cuda")
    out = sinet.new_hist(w.n_bins)

    def make_table(kind):
        tab = sinet.Table(wl.pbase, wl.plen, kind=kind)
        rep = tab.train() if kind in ("pla", "mlp") else None
        return tab, rep

    def step_fn(tab, acc=False):
        return lambda: sinet.pipeline(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"],
                                      w.t0, w.width, w.n_bins, label=label, out=out,
                                      accumulate=acc)

    results = {}
    kinds = [lookup] + [k for k in args.compare.split(",") if k and k != lookup]
    for kind in kinds:
        tab, rep = make_table(kind)
        info = tab.info()
        ms, ms_min, wall = time_calls(torch, step_fn(tab), args.steps, args.warmup)
        info = tab.info()
        results[kind] = {"ms_per_step": ms, "ms_min": ms_min, "wall_ms": wall,
                         "sessions_per_s": wl.n / (ms * 1e-3), "m": int(info.m),
                         "max_err": int(info.max_err), "segments": int(info.segments),
                         "fallbacks": int(info.fallbacks),
                         "train_ms": None if rep is None else rep.train_ms}
        log(kind, json.dumps(results[kind]))
        del tab
    r = results[lookup]
    alg_bytes = BYTES_PER_SESSION * wl.n + BYTES_PER_BIN * w.n_bins
    achieved = alg_bytes / (r["ms_per_step"] * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": r["sessions_per_s"], "unit": "sessions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32,u64",
        "data": "synthetic (seeded SINET-shaped day generated in HBM)",
        "config": {"workload": wl.name, "n_sessions": wl.n, "n_prefix": wl.n_prefix,
                   "n_bins": w.n_bins, "bin_ms": w.width, "lookup": lookup,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "sinet_pipeline step: k_stage1 (lookup+label+partition) + "
                               "segment index + k_stage2 (block reduce, one write per bin)",
                     "alg_bytes_per_launch": alg_bytes, "launch_ms": r["ms_per_step"]},
        "lookups": {k: {"sessions_per_s": v["sessions_per_s"], "ms_per_step": v["ms_per_step"],
                        "max_err": v["max_err"], "segments": v["segments"],
                        "fallbacks": v["fallbacks"]}
                    for k, v in results.items()},
    }
    if not args.no_cpu:
        sample = args.cpu_sample or 20_000_000
        line["cpu_baseline"] = cpu_baseline(wl, cols, sinet, sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
