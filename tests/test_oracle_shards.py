"""The oracle over many processes (oracle/shards.py) against the one-process
oracle, and Algorithm 1's brute-force scan over all 200,000 prefixes on a
1e5-session sample of the full day against the per-length hash form the
sharded runs use."""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import oracle
import sinetgen
from oracle import shards

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _columns(tmp, s):
    d = shards.Columns.create(os.path.join(tmp, "cols"), len(s["ts"]))
    d.write(0, ts=s["ts"], src=s["src"], dst=s["dst"], bytes=s["bytes"])
    return d


@pytest.mark.parametrize("k,t0,width,n_bins", [(4, 0, 10, 8_640_000), (3, 3_600_000, 7, 2_000_000),
                                               (5, 0, 1000, 86_400)])
def test_shards_equal_one_process(k, t0, width, n_bins):
    """Shards with their own windows, added: the same labels, bins (over the
    bins the shards reach; every other bin is zero in the one-process run)
    and dropped counts, also for a window that drops most sessions."""
    wl = sinetgen.config(2, n=400_000)
    s = sinetgen.sessions(wl)
    with tempfile.TemporaryDirectory() as tmp:
        d = _columns(tmp, s)
        r = shards.run(d, wl.pbase, wl.plen, t0, width, n_bins, k=k)
        lab = np.array(d.map("label"))
    elab, ec, eb, ed = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"],
                                       t0, width, n_bins)
    assert np.array_equal(lab, elab)
    lo, w = r["b_lo"], r["count"].shape[1]
    assert np.array_equal(r["count"], ec[:, lo:lo + w]) and np.array_equal(r["bytes"], eb[:, lo:lo + w])
    assert not ec[:, :lo].any() and not ec[:, lo + w:].any()
    assert np.array_equal(r["dropped"], ed)
    assert r["k"] == k


def test_shards_plant_a_lost_shard():
    """A merge that loses one shard's bins fails the comparison (the check is
    not vacuous)."""
    wl = sinetgen.config(2, n=100_000)
    s = sinetgen.sessions(wl)
    with tempfile.TemporaryDirectory() as tmp:
        d = _columns(tmp, s)
        r = shards.run(d, wl.pbase, wl.plen, 0, 10, 8_640_000, k=2, hi=60_000)   # a shard short
    _, ec, _, _ = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"], 0, 10,
                                  8_640_000)
    lo, w = r["b_lo"], r["count"].shape[1]
    assert not np.array_equal(r["count"], ec[:, lo:lo + w])


def _scan_worker(args):
    lo, hi = args
    code = (f"import sys; sys.path.insert(0, {ROOT!r}); import numpy as np, oracle, sinetgen; "
            f"wl = sinetgen.config(5); s = sinetgen.sessions(wl, idx=np.arange({lo}, {hi}) * 15999); "
            "r1 = oracle.classify(wl.pbase, wl.plen, s['src'], s['dst'], mode='scan'); "
            "r2 = oracle.classify(wl.pbase, wl.plen, s['src'], s['dst'], mode='hash'); "
            "assert all(np.array_equal(x, y) for x, y in zip(r1, r2)); "
            "print(int(np.count_nonzero(r1[0])))")
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)


def test_brute_force_scan_1e5_sessions_200k_prefixes():
    """Algorithm 1 over every one of the 200,000 prefixes (the brute-force
    scan, longest match and institution ids included) equals the per-length
    hash form on 100,000 sessions spread over the full day, in processes
    over the available cores."""
    from concurrent.futures import ThreadPoolExecutor
    n, k = 100_000, max(1, min(8, shards.cores()))
    cuts = [n * j // k for j in range(k + 1)]
    with ThreadPoolExecutor(k) as ex:
        outs = list(ex.map(_scan_worker, zip(cuts[:-1], cuts[1:])))
    for o in outs:
        assert o.returncode == 0, o.stderr[-2000:]
    labelled = sum(int(o.stdout.split()[-1]) for o in outs)
    assert 0 < labelled < n   # both in- and out-of-table sessions
