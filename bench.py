"""Benchmark: sessions/s of fused discrimination + millisecond histogram on one
MI355X, with the HBM roofline of the timed step and the CPU oracle timed
beside it.

One step = one pass of the whole hot path over the resident day: every
session's ts/src/dst/bytes read once, both addresses classified against the
prefix table, the label written, and (1, bytes) merged into its (label, 1-ms
bin); the 4 x 86.4 M-bin histogram is fully written (no separate clear).
Inputs are synthetic (seeded generator writing straight into HBM) with the
paper's day shape.

Forms timed on the same resident day (the first is the headline value):
  plain        labels from the table's in/out index (LDS)
  bsearch      plain binary search over the interval boundaries in global memory
  bsearch_lds  binary search with the top levels (sampled boundaries) in LDS
  trie         16-8-8 multibit trie
  pla          learned: error-bounded piecewise-linear model (about 7,700 segments,
               max error 6): one aligned 16-boundary window per address
  pla256       learned: 256 equal-count PLA segments, bounded search in the LDS
               sampled boundaries, then the boundary leaf
  mlp          learned: 1-16-1 ReLU MLP, same bounded search
  (every form but plain runs its own search for every address)
  batched_inout  the day cut into time-ordered streams, one graph launch, labels from
               the in/out index (no model)
  batched_pla  the same streams with the learned PLA answering every lookup
The plain, search and learned forms reduce with the sliding window (a
lookup pass stores the labels, then the window pass bins them); the batched
forms with the two-stage records of the batch plan.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 5|4|2|3]
                    [--forms plain,bsearch,...] [--no-cpu]
    python bench.py --host     the full day from host memory, streamed over PCIe
    python bench.py --rebin    the day's 1-ms histogram summed into one-hour frames
    python bench.py --parse    a 4 GB chunk of session text parsed into columns
    python bench.py --watch    watch-list histograms over the full day
                               (two synthetic lists, 1,177 hosts, 10-min bins)
    python bench.py --crossover  record reduce vs sliding window over session counts
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sessions/sec classify+histogram on 1 GPU, % HBM roofline; learned vs plain lookup"
HBM_PEAK_GBS = 8000.0
BYTES_PER_SESSION = 21   # ts 4 + src 4 + dst 4 + bytes 8 read, label 1 written
BYTES_PER_BIN = 64       # 4 labels x (count 8 + bytes 8) written once
DEFAULT_FORMS = "plain,bsearch,bsearch_lds,trie,pla,pla256,mlp,batched_inout,batched_pla"
# HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counter runs of the
# plain form on the default day, scaled by the counters of a plain copy
# (read x2.000, write x1.000)
COUNTER_TRAFFIC = {
    "k_window": {"workload": "fullday-1.6e9-200kpfx-86.4M1ms",
                 "sources": ("window.hip", "pass_common.h", "sinet_internal.h"),
                 "kernels_sha": "aa00b7ba0d8d2428", "bytes": 26.632e9},
    "k_stage1": {"workload": "fullday-1.6e9-200kpfx-86.4M1ms", "kernels_sha": "7b136c4cdca9f0c5",
                 "bytes": 40.32e9},
    "k_stage2": {"workload": "fullday-1.6e9-200kpfx-86.4M1ms", "kernels_sha": "7b136c4cdca9f0c5",
                 "bytes": 12.98e9},
    "k_watch": {"workload": "watch-fullday-1.6e+09-1177hosts-144x10min",
                "kernels_sha": "99b1e3a42fb8af19", "bytes": 14.77e9},
    "k_rebin_tiles": {"workload": "rebin-4x86.4M1ms-to-24x1h", "sources": ("rebin.hip", "sinet_internal.h"),
                      "kernels_sha": "c72070d268c5ab90", "bytes": 2.766e9},
    # the eight kernels of one batch graph launch together (the last launch of the run)
    "batch_graph": {"workload": "batch-64streams-299999969sessions",
                    "sources": ('batch.hip', 'kernels.hip', 'sinet_internal.h', 'sinet_device.h', 'inout_index.h'),
                    "kernels_sha": "7ec2adec32cac174", "bytes": 28.05e9},
    # the four kernels of one parse call together, summed the same way
    "parse_call": {"workload": "parse-4.0GB-20000000lines", "sources": ("parse.hip", "sinet_internal.h"),
                   "kernels_sha": "2a306051f3f37ac9", "bytes": 12.69e9},
}
KERNEL_SOURCES = ("kernels.hip", "sinet_internal.h", "sinet_device.h", "inout_index.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=5)
    ap.add_argument("--n", type=int, default=0, help="override the session count")
    ap.add_argument("--forms", default="")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0)
    ap.add_argument("--day-streams", type=int, default=24, help="streams of the batched day")
    ap.add_argument("--parse", action="store_true",
                    help="session text (Table 1 lines) parsed into columns, a 4 GB chunk")
    ap.add_argument("--rebin", action="store_true",
                    help="the day's millisecond histogram summed into one-hour frames")
    ap.add_argument("--host", action="store_true",
                    help="the plain pipeline over the full day held in host memory (streamed)")
    ap.add_argument("--watch", action="store_true",
                    help="watch-list histograms over the full day instead of the default forms")
    ap.add_argument("--crossover", action="store_true",
                    help="the record reduce against the sliding window over session counts")
    ap.add_argument("--copy-gb", type=float, default=0.0,
                    help="only run a plain device copy of this many GB (counter calibration)")
    return ap.parse_args()


def time_calls(torch, fn, steps, warmup, sinet=None):
    """Median and minimum device ms per call from HIP events recorded on the
    stream the library launches on (torch's current stream), host wall ms per
    call over the timed loop, (when sinet is given) the library's own
    per-phase event timing summed over the timed calls, and the mean ms."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    if sinet is not None:
        sinet.timing_enable(True)
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(st)
        fn()
        b.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = None
    if sinet is not None:
        phases = sinet.timing_read()
        sinet.timing_enable(False)
    dev = sorted(a.elapsed_time(b) for a, b in evs)
    k = len(dev)
    med = dev[k // 2] if k % 2 else 0.5 * (dev[k // 2 - 1] + dev[k // 2])
    return med, dev[0], wall * 1e3 / steps, phases, sum(dev) / k


def copy_ceiling(torch, gb=4.0, reps=10):
    """Read + write GB/s of a plain device-to-device copy of gb GB (the best
    of reps): the practical bandwidth ceiling the fractions are also reported
    against."""
    n = int(gb * 1e9) // 16
    x = torch.empty(n, 2, dtype=torch.int64, device="cuda")
    y = torch.empty_like(x)
    _, ms, _, _, _ = time_calls(torch, lambda: y.copy_(x), reps, 2)
    del x, y
    return 2 * 16 * n / (ms * 1e-3) / 1e9


def kernel_roofline(phases, n, n_bins, steps, workload):
    """Roofline of the dominant kernel of the step from the library's phase
    events over the timed calls.  Sliding-window reduce: the lookup pass
    (read src/dst, 8 B, write the label, 1 B, per session) or the window pass
    (read ts, bytes and label, 13 B per session, write every bin once, 64 B
    per bin).  Records reduce: stage 1 (21 B per session fused with the
    lookup, else 13 B) or stage 2 (64 B per bin).  Whichever takes longer."""
    if phases is None or phases["stage1_launches"] == 0:
        return None
    launches = phases["stage1_launches"]
    per_step = launches / steps          # launches of each kernel in one step
    cand = []
    if phases.get("window_calls", 0):
        cand.append(("k_window", phases["stage1_ms"] / launches,
                     (13 * n + BYTES_PER_BIN * n_bins) / per_step))
        cand.append(("k_pass (lookup, labels stored)", phases["lookup_ms"] / launches,
                     9 * n / per_step))
    else:
        # the fused stage 1 carries the whole per-session traffic; after a
        # separate lookup pass it reads ts, bytes and the stored label (13 B)
        fused = phases["lookup_ms"] == 0.0
        cand.append(("k_stage1", phases["stage1_ms"] / launches,
                     (BYTES_PER_SESSION if fused else 13) * n / per_step))
        if phases["stage2_ms"] > 0:
            cand.append(("k_stage2", phases["stage2_ms"] / launches, BYTES_PER_BIN * n_bins / per_step))
        if not fused:
            cand.append(("k_pass (lookup, labels stored)", phases["lookup_ms"] / launches,
                         9 * n / per_step))
    name, ms, alg = max(cand, key=lambda c: c[1])
    achieved = alg / (ms * 1e-3) / 1e9
    traffic = measured_traffic(name, workload)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": name,
            "alg_bytes_per_launch": alg, "launch_ms": ms, "launches": launches, "steps": steps}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of the kernel from the FETCH_SIZE / WRITE_SIZE
    counter runs of the default workload, scaled by the same counters of a
    plain copy; null for another workload or when the kernel sources have
    changed since."""
    import hashlib
    rec = COUNTER_TRAFFIC.get(kernel)
    if rec is None:
        return None
    h = hashlib.sha256()
    for name in rec.get("sources", KERNEL_SOURCES):
        with open(os.path.join(ROOT, "paper_2106_12863_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if rec["kernels_sha"] != h.hexdigest()[:16] or rec["workload"] != workload:
        return None
    return rec["bytes"]


def cpu_baseline(wl, cols, sinet, sample: int, gpu=None):
    """The C oracle (per-length hash) as K single-threaded processes, one per
    core this process may use (at most 16), on contiguous shards of a sample
    of the same day; generation and copies excluded from the oracle seconds.
    The shards' bins are added exactly and compared with the GPU's labels and
    bins for the sample (bins only at least the jitter inside the sample's
    time range, which no session outside it can reach)."""
    import shutil
    import tempfile

    import numpy as np

    from oracle import shards
    k = shards.cores()
    n = min(sample * k, wl.n)  # sample: sessions per core
    i0 = (wl.n - n) // 2
    base = "/dev/shm" if os.path.isdir("/dev/shm") else None
    tmp = tempfile.mkdtemp(prefix="sinet_cpu_", dir=base)
    try:
        d = shards.Columns.create(tmp, n)
        step = 1 << 26
        for a in range(0, n, step):
            b = min(n, a + step)
            d.write(a, **{c: (sinet.to_host_u64(cols[c][i0 + a:i0 + b]) if c == "bytes"
                              else sinet.to_host_u32(cols[c][i0 + a:i0 + b]))
                          for c in ("ts", "src", "dst", "bytes")})
        w = wl.window
        res = shards.run(d, wl.pbase, wl.plen, w.t0, w.width, w.n_bins, k=k)
        cpu = shards.cpu_name()
        check = {}
        if gpu is not None:
            import sinetgen
            lab_gpu, cnt_gpu, byt_gpu = gpu
            same_lab = bool(np.array_equal(d.map("label"), lab_gpu[i0:i0 + n].cpu().numpy()))
            # bins no session outside [i0, i0 + n) can reach
            t_lo = int(sinetgen.ts_base(wl, [i0])[0]) + wl.t_origin + wl.jitter + 1
            t_hi = int(sinetgen.ts_base(wl, [i0 + n - 1])[0]) + wl.t_origin - wl.jitter - 1
            b_lo = max(res["b_lo"], (t_lo - w.t0) // w.width + 1)
            b_hi = min(res["b_lo"] + res["count"].shape[1], (t_hi - w.t0) // w.width)
            same_bins = None
            if b_hi > b_lo:
                o = b_lo - res["b_lo"]
                ec = res["count"][:, o:o + b_hi - b_lo]
                eb = res["bytes"][:, o:o + b_hi - b_lo]
                same_bins = bool(np.array_equal(sinet.to_host_u64(cnt_gpu[:, b_lo:b_hi]), ec) and
                                 np.array_equal(sinet.to_host_u64(byt_gpu[:, b_lo:b_hi]), eb))
            check = {"labels_equal_gpu": same_lab, "bins_equal_gpu": same_bins,
                     "bins_checked": int(max(0, b_hi - b_lo)) * 4}
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    value = n / res["shard_s"]
    out = {"value": value, "unit": "sessions/s", "cores": res["k"], "kind": "oracle",
           "per_core": value / res["k"], "cpu": cpu["model"], "cpu_mhz": cpu["mhz"],
           "wall_s": round(res["wall_s"], 2),
           "sample": f"sessions [{i0}, {i0 + n}) of the same day ({n} sessions) in {res['k']} "
                     f"contiguous shards, one oracle process per core (per-length-hash longest-prefix "
                     f"match over {wl.n_prefix} prefixes, each shard's own bins), the slowest shard "
                     f"{res['shard_s']:.1f} s; shard bins added exactly"}
    out.update(check)
    return out


def day_streams(sinet, wl, cols, tab, k, label, out):
    """The day cut into k time-ordered index ranges: every range is its own
    stream with the full-day window, so the batch adds into one histogram
    would double-count; instead each stream gets its own slice of the day's
    bins (its time range, padded by the jitter) and its own output."""
    import torch
    w = wl.window
    per = ((wl.n + k - 1) // k + 2047) // 2048 * 2048   # whole 2048-session chunks
    streams, outs = [], []
    import sinetgen
    for i in range(k):
        lo, hi = i * per, min(wl.n, (i + 1) * per)
        if lo >= hi:
            break
        t_lo = int(sinetgen.ts_base(wl, [lo])[0]) - wl.jitter - 1
        t_hi = int(sinetgen.ts_base(wl, [hi - 1])[0]) + wl.jitter + 1
        t0 = max(w.t0, t_lo)
        nb = min(w.n_bins, t_hi - t0 + 1)
        o = sinet.new_hist(nb)
        outs.append(o)
        streams.append(sinet.BatchStream(tab, cols["ts"][lo:hi], cols["src"][lo:hi],
                                         cols["dst"][lo:hi], cols["bytes"][lo:hi], t0, w.width,
                                         nb, label=label[lo:hi], out=o))
    return streams, outs


def bench_day(args, torch, sinet, sinetgen, gg):
    wl = sinetgen.config(args.config, n=args.n or None)
    forms = (args.forms or (DEFAULT_FORMS if args.config in (4, 5) else
                            "plain,bsearch,bsearch_lds,trie")).split(",")
    log(f"config {args.config}: {wl.name} n={wl.n} prefixes={wl.n_prefix} forms={forms}")
    cols = gg.alloc_and_fill(wl)
    torch.cuda.synchronize()
    w = wl.window
    label = torch.empty(wl.n, dtype=torch.uint8, device="cuda")
    out = sinet.new_hist(w.n_bins)
    results = {}
    for form in forms:
        if form in ("batched_inout", "batched_pla"):
            # batched_inout: labels from the in/out index (no model);
            # batched_pla: labels from the learned PLA lookup itself
            if form == "batched_inout":
                tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch", inout_index=True)
                rep = None
            else:
                tab = sinet.Table(wl.pbase, wl.plen, kind="pla", inout_index=False)
                rep = tab.train()
            streams, outs = day_streams(sinet, wl, cols, tab, args.day_streams, label, out)
            tune = sinet.autotune(streams)
            plan = sinet.BatchPlan(streams, tune=tune)
            fn = plan.run
        else:
            kind = ("bsearch" if form in ("plain", "bsearch_lds") else
                    "pla" if form == "pla256" else form)
            tab = sinet.Table(wl.pbase, wl.plen, kind=kind, inout_index=(form == "plain"),
                              global_bsearch=(form == "bsearch"))
            rep = None
            if kind == "mlp":
                rep = tab.train()
            elif kind == "pla":
                rep = tab.train(segments=256) if form == "pla256" else tab.train()
            fn = (lambda t=tab: sinet.pipeline(t, cols["ts"], cols["src"], cols["dst"],
                                               cols["bytes"], w.t0, w.width, w.n_bins,
                                               label=label, out=out))
        ms, ms_min, wall, phases, ms_mean = time_calls(torch, fn, args.steps, args.warmup,
                                                       None if form.startswith("batched") else sinet)
        info = tab.info()
        results[form] = {"sessions_per_s": wl.n / (ms * 1e-3), "ms_per_step": ms, "ms_min": ms_min,
                         "ms_mean": ms_mean, "wall_ms": wall, "kind": sinet.KIND_NAMES[info.kind],
                         "inout_index": bool(info.inout_index) and form in ("plain", "batched_inout"),
                         "m": int(info.m)}
        if sinet.KIND_NAMES[info.kind] in ("pla", "mlp"):
            e = int(info.max_err)
            results[form].update({
                "max_err": e, "segments": int(info.segments), "fallbacks": int(info.fallbacks),
                # boundaries the bounded search may look at, and its probes (binary search
                # over them; a window of at most 16 is one aligned 16-boundary read)
                "search_window": 2 * e + 1,
                "probes": 1 if 2 * e + 1 <= 16 else math.ceil(math.log2(2 * e + 2)),
                "train_ms": None if rep is None else round(rep.train_ms, 3)})
        if phases is not None:
            results[form]["phases_ms_per_step"] = {
                k[:-3]: phases[k] / args.steps
                for k in ("lookup_ms", "stage1_ms", "index_ms", "stage2_ms", "far_ms")}
            results[form]["_phases"] = phases
        if form.startswith("batched"):
            results[form]["reduce"] = "records (batch plan)"
            results[form]["tune"] = {"block": tune.block, "chunk": tune.chunk, "grid": tune.grid}
            results[form]["streams"] = len(streams)
            del plan, streams, outs
        log(form, json.dumps(results[form]))
        del tab
    if "plain" in results and wl.n < (1 << 32):
        # the label runs (stable partition of the day's indices by label, per-wave
        # ballots and mbcnt ranks) on the plain form's labels; not part of the step
        ridx = torch.empty(wl.n, dtype=torch.int32, device="cuda")
        rtot = torch.empty(4, dtype=torch.int64, device="cuda")
        ms_r, min_r, _, _, _ = time_calls(torch, lambda: sinet.label_runs(label, ridx, rtot),
                                          args.steps, args.warmup)
        rb = 2 * wl.n + 4 * wl.n   # labels read by the count and scatter passes, indices written
        results["plain"]["label_runs"] = {"ms_per_call": ms_r, "ms_min": min_r, "alg_bytes": rb,
                                          "achieved_gbs": rb / (ms_r * 1e-3) / 1e9,
                                          "totals": [int(x) for x in rtot.cpu().tolist()]}
        log("label_runs", json.dumps(results["plain"]["label_runs"]))
        del ridx
    head = forms[0]
    r = results[head]
    alg_bytes = BYTES_PER_SESSION * wl.n + BYTES_PER_BIN * w.n_bins
    roof = kernel_roofline(r.get("_phases"), wl.n, w.n_bins, args.steps, wl.name)
    copy_gbs = copy_ceiling(torch)
    if roof is not None:
        roof["copy_ceiling_gbs"] = copy_gbs
        roof["frac_of_copy"] = roof["achieved"] / copy_gbs
    line = {
        "metric": METRIC, "value": r["sessions_per_s"], "unit": "sessions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32,u64",
        "data": "synthetic (seeded SINET-shaped day generated in HBM)",
        "config": {"workload": wl.name, "n_sessions": wl.n, "n_prefix": wl.n_prefix,
                   "n_bins": w.n_bins, "bin_ms": w.width, "form": head,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "step_roofline": {"alg_bytes": alg_bytes, "ms": r["ms_per_step"],
                          "achieved": alg_bytes / (r["ms_per_step"] * 1e-3) / 1e9,
                          "frac": alg_bytes / (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "frac_of_copy": alg_bytes / (r["ms_per_step"] * 1e-3) / 1e9 / copy_gbs},
        "forms": {k: {kk: vv for kk, vv in v.items() if kk not in ("wall_ms", "_phases")}
                  for k, v in results.items()},
    }
    for k, v in results.items():
        line["forms"][k]["hbm_frac"] = alg_bytes / (v["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS
    if not args.no_cpu:
        # the plain form's labels and bins, for the check
        tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch", inout_index=True)
        sinet.pipeline(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"], w.t0,
                       w.width, w.n_bins, label=label, out=out)
        torch.cuda.synchronize()
        del tab
        sample = args.cpu_sample or 25_000_000
        line["cpu_baseline"] = cpu_baseline(wl, cols, sinet, sample, gpu=(label, out[0], out[1]))
    return line


def bench_batch(args, torch, sinet, sinetgen, gg):
    """Config 3: 64 uneven streams, each with its own table, window and bin
    width: one autotuned graph launch against per-stream pipeline calls."""
    streams_wl = sinetgen.batch_streams()
    log(f"config 3: {len(streams_wl)} streams, {sum(s.n for s in streams_wl)} sessions")
    built = []
    for wl in streams_wl:
        cols = gg.alloc_and_fill(wl)
        tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
        lab = torch.empty(wl.n, dtype=torch.uint8, device="cuda")
        out = sinet.new_hist(wl.window.n_bins)
        built.append((wl, cols, tab, lab, out))
    torch.cuda.synchronize()
    bs = [sinet.BatchStream(tab, c["ts"], c["src"], c["dst"], c["bytes"], wl.window.t0,
                            wl.window.width, wl.window.n_bins, label=lab, out=out)
          for wl, c, tab, lab, out in built]
    tune = sinet.autotune(bs)
    plan = sinet.BatchPlan(bs, tune=tune)

    def per_stream():
        for wl, c, tab, lab, out in built:
            sinet.pipeline(tab, c["ts"], c["src"], c["dst"], c["bytes"], wl.window.t0,
                           wl.window.width, wl.window.n_bins, label=lab, out=out)

    n = sum(wl.n for wl in streams_wl)
    bins = sum(wl.window.n_bins for wl in streams_wl)
    ms_b, min_b, _, _, _ = time_calls(torch, plan.run, args.steps, args.warmup)
    ms_p, min_p, _, _, _ = time_calls(torch, per_stream, args.steps, args.warmup)
    alg_bytes = BYTES_PER_SESSION * n + BYTES_PER_BIN * bins
    achieved = alg_bytes / (ms_b * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": n / (ms_b * 1e-3), "unit": "sessions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_b,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32,u64",
        "data": "synthetic (seeded uneven streams generated in HBM)",
        "config": {"workload": f"batch-{len(streams_wl)}streams-{n}sessions", "n_sessions": n,
                   "n_bins_total": bins, "form": "batched", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("batch_graph",
                                                 f"batch-{len(streams_wl)}streams-{n}sessions"),
                     "kernel": "one batch graph launch", "alg_bytes_per_launch": alg_bytes,
                     "launch_ms": ms_b},
        "forms": {"batched": {"ms_per_step": ms_b, "ms_min": min_b,
                              "tune": {"block": tune.block, "chunk": tune.chunk, "grid": tune.grid}},
                  "per_stream_calls": {"ms_per_step": ms_p, "ms_min": min_p,
                                       "sessions_per_s": n / (ms_p * 1e-3)}},
    }
    if not args.no_cpu:
        # whole streams in order, each in shards over the cores, until about
        # 10 s of oracle time
        tot_n, tot_s, used, k = 0, 0.0, 0, 1
        for wl, c, *_ in built:
            r = cpu_baseline(wl, c, sinet, wl.n)
            k = r["cores"]
            tot_n += wl.n
            tot_s += wl.n / r["value"]
            used += 1
            if tot_s > 10.0:
                break
        line["cpu_baseline"] = {"value": tot_n / tot_s, "unit": "sessions/s", "cores": k,
                                "kind": "oracle", "per_core": tot_n / tot_s / k,
                                "cpu": r["cpu"], "cpu_mhz": r["cpu_mhz"],
                                "sample": f"the first {used} of the {len(built)} streams, whole "
                                          f"({tot_n} sessions, {tot_s:.1f} s of the slowest shards), "
                                          f"each in {k} shards with its own prefix table, window "
                                          "and bins"}
    return line


def bench_parse(args, torch, sinet, sinetgen, gg):
    """A 4 GB chunk of session text (the paper's chunks were 4, 6 and 9 GB of
    PA-7080 records) parsed into columns: 500,000 generated Table 1 lines
    (about 200 bytes each) repeated on the device to 20 million lines."""
    from sinetgen import text as stext
    wl = sinetgen.config(5)
    i0 = wl.n // 2
    unit = 500_000
    buf, _ = stext.session_lines(wl, start=i0, stop=i0 + unit)
    reps = 40
    dev = torch.from_numpy(buf).cuda().repeat(reps)
    n_lines = unit * reps
    cols, bad = sinet.parse_sessions(dev, stext.ORIGIN_DAYS, capacity=n_lines)
    torch.cuda.synchronize()
    assert bad == 0 and cols["ts"].shape[0] == n_lines

    def step():
        sinet.parse_sessions(dev, stext.ORIGIN_DAYS, capacity=n_lines)

    ms, ms_min, wall, _, _ = time_calls(torch, step, args.steps, args.warmup)
    alg = dev.numel() + 20 * n_lines  # the text read once, the columns written once
    achieved = alg / (ms * 1e-3) / 1e9
    workload = f"parse-{dev.numel() / 1e9:.1f}GB-{n_lines}lines"
    line = {
        "metric": "sessions/sec parsed from session text on 1 GPU, % HBM roofline",
        "value": n_lines / (ms * 1e-3), "unit": "sessions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8 text",
        "data": "synthetic (Table 1 lines generated from the full day's sessions, 500,000 lines "
                f"repeated {reps} times)",
        "config": {"workload": workload,
                   "text_bytes": dev.numel(), "lines": n_lines,
                   "bytes_per_line": dev.numel() / n_lines, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("parse_call", workload),
                     "kernel": "the parse call (count, scan, line starts, parse; synchronous)",
                     "alg_bytes_per_launch": alg, "launch_ms": ms},
        "forms": {"parse": {"ms_per_step": ms, "ms_min": ms_min, "wall_ms": wall}},
    }
    if not args.no_cpu:
        import oracle
        tc = time.perf_counter()
        oracle.parse(buf, stext.ORIGIN_DAYS)
        sec = time.perf_counter() - tc
        line["cpu_baseline"] = {"value": unit / sec, "unit": "sessions/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"the {unit} generated lines ({buf.shape[0] / 1e6:.0f} MB, "
                                          f"{sec:.2f} s), parsed once"}
    return line


def bench_rebin(args, torch, sinet, sinetgen, gg):
    """The full day's millisecond histogram (4 x 86.4 M count and byte bins,
    5.53 GB) summed into 24 one-hour frames, as in the paper's Figures 6-7."""
    wl = sinetgen.config(5, n=args.n or None)
    w = wl.window
    cols = gg.alloc_and_fill(wl)
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    _, (c, b, _) = sinet.pipeline(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"], w.t0,
                                  w.width, w.n_bins)
    del cols
    factor = 3_600_000
    oc = sinet.rebin(c, factor)
    ob = sinet.rebin(b, factor)

    def step():
        sinet.rebin(c, factor, out=oc)
        sinet.rebin(b, factor, out=ob)

    ms, ms_min, wall, _, _ = time_calls(torch, step, args.steps, args.warmup)
    alg = 2 * 8 * 4 * w.n_bins  # every millisecond bin read once
    achieved = alg / (ms * 1e-3) / 1e9
    line = {
        "metric": "bins/sec summed into one-hour frames on 1 GPU, % HBM roofline",
        "value": 2 * 4 * w.n_bins / (ms * 1e-3), "unit": "bins/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic (the full synthetic day's histogram, computed in HBM)",
        "config": {"workload": "rebin-4x86.4M1ms-to-24x1h", "n_bins": w.n_bins, "factor": factor,
                   "arrays": 2, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("k_rebin_tiles", "rebin-4x86.4M1ms-to-24x1h"),
                     "kernel": "k_rebin_tiles (two launches per step)",
                     "alg_bytes_per_launch": alg / 2, "launch_ms": ms / 2},
        "forms": {"rebin": {"ms_per_step": ms, "ms_min": ms_min, "wall_ms": wall}},
    }
    if not args.no_cpu:
        import oracle
        hc, hb = sinet.to_host_u64(c), sinet.to_host_u64(b)  # the whole workload, copies excluded
        tc = time.perf_counter()
        oracle.rebin(hc, factor)
        oracle.rebin(hb, factor)
        sec = time.perf_counter() - tc
        line["cpu_baseline"] = {"value": 2 * hc.size / sec, "unit": "bins/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"the whole step: both arrays, {2 * hc.size} bins "
                                          f"({sec:.2f} s)"}
    return line


def bench_host(args, torch, sinet, sinetgen, gg):
    """The plain pipeline over the full synthetic day held in host memory
    (pinned, then pageable), streamed through the device in chunks: the
    rate of the out-of-core path, bound by the host link, never the
    benchmark's headline value."""
    import numpy as np
    wl = sinetgen.config(5, n=args.n or None)
    w = wl.window
    dcols = gg.alloc_and_fill(wl)
    pin = {}
    for c, t in dcols.items():
        pin[c] = torch.empty(wl.n, dtype=t.dtype, pin_memory=True)
        pin[c].copy_(t)
    torch.cuda.synchronize()
    del dcols, t
    torch.cuda.empty_cache()
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    st = sinet.Streamer(chunk=64 << 20)
    out = sinet.new_hist(w.n_bins)
    lab = torch.empty(wl.n, dtype=torch.uint8, pin_memory=True)

    def run(cols, label):
        t = time.perf_counter()
        st.pipeline(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"], w.t0, w.width,
                    w.n_bins, label=label, out=out)
        return (time.perf_counter() - t) * 1e3

    steps = max(1, min(args.steps, 3))
    run(pin, lab)
    ms_pin = min(run(pin, lab) for _ in range(steps))
    # host-to-device ceiling: one pinned 4 GB copy
    x = torch.empty(1 << 30, dtype=torch.int32, pin_memory=True)
    y = torch.empty(1 << 30, dtype=torch.int32, device="cuda")
    y.copy_(x)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        y.copy_(x, non_blocking=True)
    torch.cuda.synchronize()
    h2d = 3 * 4 * (1 << 30) / (time.perf_counter() - t) / 1e9
    del x, y
    page = {c: v.numpy().copy() for c, v in pin.items()}
    lab_np = np.empty(wl.n, np.uint8)
    ms_page = run(page, lab_np)
    moved = 20 * wl.n  # columns in (the labels go the other way on the full-duplex link)
    achieved = moved / (ms_pin * 1e-3) / 1e9
    st.close()
    base = None
    if not args.no_cpu:
        import oracle
        n = min(36_000_000, wl.n)
        i0 = (wl.n - n) // 2
        hs = {k: v[i0:i0 + n].view(np.uint64 if k == "bytes" else np.uint32) for k, v in page.items()}
        tc = time.perf_counter()
        oracle.pipeline(wl.pbase, wl.plen, hs["ts"], hs["src"], hs["dst"], hs["bytes"], w.t0,
                        w.width, w.n_bins, mode="hash")
        dt = time.perf_counter() - tc
        base = {"value": n / dt, "unit": "sessions/s", "cores": 1, "kind": "oracle",
                "sample": f"sessions [{i0}, {i0 + n}) of the same host-resident day ({n} sessions, "
                          f"{dt:.1f} s)"}
    line = {
        "metric": "sessions/sec classify+histogram on 1 GPU from host memory (host link included)",
        "value": wl.n / (ms_pin * 1e-3), "unit": "sessions/s", "n_gpus": 1, "steps": steps,
        "warmup": 1, "ms_per_step": ms_pin, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32,u64",
        "data": "synthetic (seeded SINET-shaped day, generated in HBM, held in pinned host memory)",
        "config": {"workload": wl.name + "-host", "n_sessions": wl.n, "chunk_sessions": 64 << 20,
                   "form": "streamed from host", "parallelism": "single GPU"},
        "roofline": {"bound": "host link", "achieved": achieved, "peak": h2d, "unit": "GB/s",
                     "frac": achieved / h2d, "traffic": None,
                     "kernel": "host-to-device copies of the columns (labels back concurrently)",
                     "peak_note": "measured pinned host-to-device copy rate of this machine"},
        "forms": {"pinned": {"ms_per_step": ms_pin, "sessions_per_s": wl.n / (ms_pin * 1e-3)},
                  "pageable": {"ms_per_step": ms_page,
                               "sessions_per_s": wl.n / (ms_page * 1e-3)}},
    }
    if base is not None:
        line["cpu_baseline"] = base
    return line


def bench_watch(args, torch, sinet, sinetgen, gg):
    """Watch-list histograms (sections "AbuseIPDB" and "GRIZZLY STEPPE") over
    the full synthetic day: the two synthetic lists' 1,177 hosts placed in
    0.2% of the sources and of the destinations, one key per host, 10-minute
    bins, both directions."""
    import numpy as np
    wl = sinetgen.config(5, n=args.n or None)
    wlist = sinetgen.watch_lists()
    log(f"watch: {wl.n} sessions, {wlist.n} listed hosts")
    cols = gg.alloc_and_fill(wl)
    gg.watch_fill(wlist, cols["src"], cols["dst"])
    plen = np.full(wlist.n, 32, np.uint8)
    tab = sinet.Table(wlist.addrs, plen, kind="bsearch")
    t0, width, n_bins, n_keys = 0, 600_000, 144, wlist.n
    out = sinet.new_watch_hist(n_keys, n_bins)

    def step():
        sinet.watch_histogram(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"], t0, width,
                              n_bins, n_keys, out=out)

    ms, ms_min, wall, ph, _ = time_calls(torch, step, args.steps, args.warmup, sinet=sinet)
    addrs = torch.from_numpy(wlist.addrs.view(np.int32)).cuda()
    ls, ld = torch.isin(cols["src"], addrs), torch.isin(cols["dst"], addrs)
    matched = int((ls | ld).sum())
    cells = 2 * n_keys * n_bins
    # what the method must move: both addresses of every session, the time
    # and byte count of the sessions with a listed endpoint, every cell once
    alg = 8 * wl.n + 12 * matched + 16 * cells
    launch_ms = ph["lookup_ms"] / max(1, ph["calls"])
    achieved = alg / (launch_ms * 1e-3) / 1e9
    workload = f"watch-fullday-{wl.n:.2g}-{wlist.n}hosts-{n_bins}x10min"
    line = {
        "metric": "sessions/sec watch-list histograms on 1 GPU, % HBM roofline",
        "value": wl.n / (ms * 1e-3), "unit": "sessions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32,u64",
        "data": "synthetic (seeded SINET-shaped day with synthetic watch lists, generated in HBM)",
        "config": {"workload": workload, "n_sessions": wl.n, "listed_hosts": wlist.n,
                   "lists": [int(x) for x in np.bincount(wlist.lists)], "keys": "per host",
                   "n_bins": n_bins, "bin_ms": width, "listed_share": wlist.frac,
                   "sessions_with_a_listed_end": matched, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("k_watch", workload), "kernel": "k_watch",
                     "alg_bytes_per_launch": alg, "launch_ms": launch_ms,
                     "launches": ph["calls"], "steps": args.steps},
        "forms": {"watch": {"ms_per_step": ms, "ms_min": ms_min, "wall_ms": wall,
                            "cells": cells, "listed_src": int(ls.sum()),
                            "listed_dst": int(ld.sum())}},
    }
    if not args.no_cpu:
        import oracle
        sample = args.cpu_sample or 40_000_000
        n = min(sample, wl.n)
        i0 = (wl.n - n) // 2
        s = {k: (sinet.to_host_u64(v[i0:i0 + n]) if k == "bytes" else sinet.to_host_u32(v[i0:i0 + n]))
             for k, v in cols.items()}
        tc = time.perf_counter()
        oracle.watch(wlist.addrs, plen, s["ts"], s["src"], s["dst"], s["bytes"], t0, width, n_bins,
                     n_keys)
        sec = time.perf_counter() - tc
        line["cpu_baseline"] = {"value": n / sec, "unit": "sessions/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"sessions [{i0}, {i0 + n}) of the same day ({n} sessions, "
                                          f"{sec:.1f} s): per-length-hash match of both ends "
                                          f"against the {wlist.n} hosts, {cells}-cell histogram"}
    return line


def bench_crossover(args, torch, sinet, sinetgen, gg):
    """Median ms per pipeline call of the record reduce and of the sliding
    window on days of the 1e8-session shape (1,024 prefixes) cut to n
    sessions, with 86.4 M and 4 M 1-ms bins, and on 4e8 sessions of the
    200,000-prefix day: where the automatic choice switches."""
    cases = [(2, 4_200_000, 86_400_000), (2, 16_000_000, 86_400_000), (2, 33_000_000, 86_400_000),
             (2, 100_000_000, 86_400_000), (2, 16_000_000, 4_000_000), (5, 400_000_000, 86_400_000)]
    rows = []
    for cfg, n, nb in cases:
        wl = sinetgen.config(cfg, n=n)
        cols = gg.alloc_and_fill(wl)
        tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
        lab = torch.empty(n, dtype=torch.uint8, device="cuda")
        out = sinet.new_hist(nb)
        r = {"config": cfg, "n_sessions": n, "n_bins": nb}
        try:
            for red in ("records", "window"):
                sinet.set_reduce(red)
                ms, _, _, _, _ = time_calls(
                    torch, lambda: sinet.pipeline(tab, cols["ts"], cols["src"], cols["dst"],
                                                  cols["bytes"], 0, 1, nb, label=lab, out=out),
                    args.steps, args.warmup)
                r[red + "_ms"] = ms
        finally:
            sinet.set_reduce("auto")
        log("crossover", json.dumps(r))
        rows.append(r)
        del cols, lab, out, tab
        torch.cuda.empty_cache()
    return {"metric": "ms per pipeline call, record reduce vs sliding window", "unit": "ms",
            "higher_is_better": False, "data": "synthetic", "rows": rows}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if args.copy_gb:
        # a plain copy of known size: the reference that scales the HBM
        # traffic counters (FETCH_SIZE / WRITE_SIZE) of the other kernels
        n = int(args.copy_gb * 1e9) // 16
        x = torch.ones(n, 2, dtype=torch.int64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        ms, _, _, _, _ = time_calls(torch, lambda: y.copy_(x), max(1, args.steps), 1)
        print(json.dumps({"copy_bytes_each_way": 16 * n, "ms": ms,
                          "gbs_read_plus_write": 32 * n / (ms * 1e-3) / 1e9}), flush=True)
        return
    import paper_2106_12863_amd as sinet
    import sinetgen
    import sinetgen.gpu as gg
    if args.crossover:
        line = bench_crossover(args, torch, sinet, sinetgen, gg)
    elif args.watch:
        line = bench_watch(args, torch, sinet, sinetgen, gg)
    elif args.host:
        line = bench_host(args, torch, sinet, sinetgen, gg)
    elif args.rebin:
        line = bench_rebin(args, torch, sinet, sinetgen, gg)
    elif args.parse:
        line = bench_parse(args, torch, sinet, sinetgen, gg)
    elif args.config == 3:
        line = bench_batch(args, torch, sinet, sinetgen, gg)
    else:
        line = bench_day(args, torch, sinet, sinetgen, gg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
