"""The oracle over many processes: contiguous index ranges (shards) of one set
of session columns, each run by its own single-threaded oracle process, the
shards' histograms then added exactly.

TEST INFRASTRUCTURE ONLY: the tests and the benchmark's CPU-baseline leg use
this module; the GPU library never does.  Every shard computes exactly what
the one-process oracle computes for its sessions (labels by the per-length
hash form of the longest-prefix-match definition, one counter per (label,
bin)); the sums over shards are the associative and commutative u64 merge of
the paper's map-reduce sections ("Reduce", "Merge Scatter Pattern with
CPU"), so the result equals the one-process oracle's on the whole input.

A shard's histogram covers only the bins its own sessions reach (its window
starts at its smallest in-window bin), so no process clears or fills the
whole day's histogram; sessions outside the call's window are dropped exactly
as in one process.  Columns and labels live in files (numpy memory maps) that
every process maps; a worker copies its slice before the timed oracle call.

    d = shards.Columns.create(dir, n)      # ts, src, dst, bytes, labels files
    d.write(i0, ts=..., src=..., dst=..., bytes=...)
    res = shards.run(d, pbase, plen, t0, width, n_bins, k=16)
"""
from __future__ import annotations

import json
import os
import subprocess
import sys
import time

import numpy as np

_COLS = (("ts", np.uint32), ("src", np.uint32), ("dst", np.uint32), ("bytes", np.uint64))


class Columns:
    """Session columns (and a label output) as files in one directory."""

    def __init__(self, path: str, n: int):
        self.path, self.n = path, n

    @classmethod
    def create(cls, path: str, n: int) -> "Columns":
        os.makedirs(path, exist_ok=True)
        for name, dt in _COLS + (("label", np.uint8),):
            np.lib.format.open_memmap(os.path.join(path, name + ".npy"), mode="w+", dtype=dt,
                                      shape=(n,))
        with open(os.path.join(path, "meta.json"), "w") as f:
            json.dump({"n": n}, f)
        return cls(path, n)

    @classmethod
    def open(cls, path: str) -> "Columns":
        with open(os.path.join(path, "meta.json")) as f:
            return cls(path, json.load(f)["n"])

    def map(self, name: str, mode: str = "r"):
        return np.load(os.path.join(self.path, name + ".npy"), mmap_mode=mode)

    def write(self, i0: int, **cols):
        for name, a in cols.items():
            m = self.map(name, "r+")
            m[i0:i0 + len(a)] = a
            m.flush()
            del m

    def remove(self):
        for name, _ in _COLS + (("label", np.uint8),):
            p = os.path.join(self.path, name + ".npy")
            if os.path.exists(p):
                os.remove(p)
        for f in os.listdir(self.path):
            if f.startswith("shard") or f in ("meta.json", "table.npz"):
                os.remove(os.path.join(self.path, f))
        try:
            os.rmdir(self.path)
        except OSError:
            pass


def _worker(path: str, k: int, lo: int, hi: int, t0: int, width: int, n_bins: int) -> None:
    import oracle
    cols = Columns.open(path)
    tab = np.load(os.path.join(path, "table.npz"))
    s = {name: np.array(cols.map(name)[lo:hi]) for name, _ in _COLS}  # copied: outside the timing
    ts = s["ts"].astype(np.int64)
    b = (ts - t0) // width
    inw = (ts >= t0) & (b < n_bins)
    b_lo = int(b[inw].min()) if inw.any() else 0
    b_hi = int(b[inw].max()) if inw.any() else 0
    t = time.perf_counter()
    lab, cnt, byt, drp = oracle.pipeline(tab["pbase"], tab["plen"], s["ts"], s["src"], s["dst"],
                                         s["bytes"], t0 + b_lo * width, width, b_hi - b_lo + 1,
                                         mode="hash")
    dt = time.perf_counter() - t
    out = cols.map("label", "r+")
    out[lo:hi] = lab
    out.flush()
    np.savez(os.path.join(path, f"shard{k}.npz"), b_lo=b_lo, count=cnt, bytes=byt, dropped=drp,
             seconds=dt, n=hi - lo)


def cores() -> int:
    """Worker processes to run: the CPUs this process may use, at most 16."""
    try:
        c = len(os.sched_getaffinity(0))
    except AttributeError:
        c = os.cpu_count() or 1
    return max(1, min(16, c))


def cpu_name() -> dict:
    """Model name and clock (MHz) of the host CPU, from /proc/cpuinfo."""
    model, mhz = "unknown", None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model == "unknown":
                    model = line.split(":", 1)[1].strip()
                if line.startswith("cpu MHz") and mhz is None:
                    mhz = float(line.split(":", 1)[1])
    except OSError:
        pass
    return {"model": model, "mhz": mhz}


def run(cols: Columns, pbase, plen, t0: int, width: int, n_bins: int, k: int = 0,
        lo: int = 0, hi: int = -1):
    """Oracle over sessions [lo, hi) of the columns in k processes (k = 0:
    cores()).  Labels go to the columns' label file.  Returns the bins the
    sessions reach, added over the shards: b_lo and count/bytes
    [4][b_hi - b_lo + 1] (u64), dropped [4][2], the wall seconds of the
    parallel oracle calls and the largest single shard's oracle seconds."""
    hi = cols.n if hi < 0 else hi
    k = k or cores()
    np.savez(os.path.join(cols.path, "table.npz"), pbase=np.asarray(pbase, np.uint32),
             plen=np.asarray(plen, np.uint8))
    cuts = [lo + (hi - lo) * j // k for j in range(k + 1)]
    env = dict(os.environ, OMP_NUM_THREADS="1")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    procs = []
    t = time.perf_counter()
    for j in range(k):
        if cuts[j + 1] <= cuts[j]:
            continue
        args = [sys.executable, "-c",
                f"import sys; sys.path.insert(0, {root!r}); from oracle import shards; "
                f"shards._worker({cols.path!r}, {j}, {cuts[j]}, {cuts[j + 1]}, {t0}, {width}, {n_bins})"]
        procs.append((j, subprocess.Popen(args, env=env)))
    bad = [j for j, p in procs if p.wait() != 0]
    wall = time.perf_counter() - t
    if bad:
        raise RuntimeError(f"oracle shards {bad} failed")
    parts = [np.load(os.path.join(cols.path, f"shard{j}.npz")) for j, _ in procs]
    b_lo = min(int(p["b_lo"]) for p in parts if p["count"].shape[1])
    b_hi = max(int(p["b_lo"]) + p["count"].shape[1] - 1 for p in parts)
    cnt = np.zeros((4, b_hi - b_lo + 1), np.uint64)
    byt = np.zeros((4, b_hi - b_lo + 1), np.uint64)
    drp = np.zeros((4, 2), np.uint64)
    longest = 0.0
    for p in parts:
        o = int(p["b_lo"]) - b_lo
        w = p["count"].shape[1]
        cnt[:, o:o + w] += p["count"]
        byt[:, o:o + w] += p["bytes"]
        drp += p["dropped"]
        longest = max(longest, float(p["seconds"]))
    for j, _ in procs:
        os.remove(os.path.join(cols.path, f"shard{j}.npz"))
    return {"b_lo": b_lo, "count": cnt, "bytes": byt, "dropped": drp, "wall_s": wall,
            "shard_s": longest, "k": len(procs), "n": hi - lo}
