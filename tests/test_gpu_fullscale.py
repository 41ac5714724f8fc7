"""Every output of the benchmark's workloads against the oracle at full size.

The GPU runs the launch the benchmark times; the oracle runs as one
single-threaded process per host core (at most 16) on contiguous index
ranges, each over its own bins, and the shards' bins are added exactly
(oracle/shards.py: the map-reduce merge of the paper's sections "Reduce" and
"Merge Scatter Pattern with CPU").  Compared bit for bit: every label, every
(label, bin) count and byte sum, the dropped counters.

- The 1e8-session day (1,024 prefixes) and the 1.6e9-session day (200,000
  prefixes), 86.4 M 1-ms bins each: the plain form (in/out index) and, on the
  large day, the error-bounded PLA form.
- The 5e8-session day over the clustered 200,000-prefix table: the learned
  forms (error-bounded PLA, 256-segment PLA, MLP) and the plain form.
- The 64-stream batch (each stream its own table, window and bin width, about
  3e8 sessions): one batch-plan launch, compared stream by stream.

The columns are copied once from the GPU into files that the oracle
processes map (in /dev/shm when it has room, else the temporary directory).
"""
import os
import shutil
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import sinetgen
from oracle import shards

pytestmark = pytest.mark.gpu

STEP = 1 << 26          # sessions per host copy / compare chunk


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sinet():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2106_12863_amd as s
    return s


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _scratch(need: int) -> str:
    """A directory with room for `need` bytes of column files."""
    for base in ("/dev/shm", tempfile.gettempdir()):
        try:
            st = os.statvfs(base)
        except OSError:
            continue
        if st.f_bavail * st.f_frsize > need * 1.2:
            return tempfile.mkdtemp(prefix="sinet_full_", dir=base)
    pytest.fail(f"no host directory with {need / 1e9:.1f} GB free for the oracle's columns")


def _host_columns(sinet, cols, path, n):
    d = shards.Columns.create(path, n)
    for a in range(0, n, STEP):
        b = min(n, a + STEP)
        d.write(a, ts=sinet.to_host_u32(cols["ts"][a:b]), src=sinet.to_host_u32(cols["src"][a:b]),
                dst=sinet.to_host_u32(cols["dst"][a:b]), bytes=sinet.to_host_u64(cols["bytes"][a:b]))
    return d


def _same_labels(sinet, d, lab, n):
    ref = d.map("label")
    for a in range(0, n, STEP):
        b = min(n, a + STEP)
        if not np.array_equal(np.asarray(ref[a:b]), lab[a:b].cpu().numpy()):
            bad = np.flatnonzero(np.asarray(ref[a:b]) != lab[a:b].cpu().numpy())
            return f"labels differ at {a + int(bad[0])} ({bad.shape[0]} in [{a}, {b}))"
    return None


def _same_bins(sinet, res, out):
    """The oracle's bins over [b_lo, b_lo + w) equal the GPU's, every other
    GPU bin is zero, the dropped counters are equal."""
    c, b, dr = out
    lo, w = res["b_lo"], res["count"].shape[1]
    if not np.array_equal(sinet.to_host_u64(c[:, lo:lo + w]), res["count"]):
        return "count bins differ"
    if not np.array_equal(sinet.to_host_u64(b[:, lo:lo + w]), res["bytes"]):
        return "byte bins differ"
    if bool(c[:, :lo].any()) or bool(c[:, lo + w:].any()) or bool(b[:, :lo].any()) \
            or bool(b[:, lo + w:].any()):
        return "bins outside the sessions' range are not zero"
    if not np.array_equal(sinet.to_host_u64(dr), res["dropped"]):
        return "dropped differ"
    return None


DAY_FORMS = {2: ("plain",), 4: ("plain", "pla", "pla256", "mlp"), 5: ("plain", "pla")}


def _table(sinet, wl, form):
    if form == "plain":
        return sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    tab = sinet.Table(wl.pbase, wl.plen, kind="mlp" if form == "mlp" else "pla", inout_index=False)
    if form == "pla256":
        tab.train(segments=256)
    elif form == "mlp":
        tab.train(steps=2000)
    else:
        tab.train()
    return tab


@pytest.mark.timeout(900, method="thread")
@pytest.mark.parametrize("cfg", [2, 4, 5])
def test_day_every_label_and_bin(sinet, torch, cfg):
    import sinetgen.gpu as gg
    wl = sinetgen.config(cfg)
    w = wl.window
    _say("full-size day", cfg, wl.n, "sessions", w.n_bins, "bins")
    cols = gg.alloc_and_fill(wl)
    torch.cuda.synchronize()
    tmp = _scratch(21 * wl.n)
    try:
        d = _host_columns(sinet, cols, os.path.join(tmp, "cols"), wl.n)
        res = shards.run(d, wl.pbase, wl.plen, w.t0, w.width, w.n_bins)
        _say("oracle", res["k"], "shards", round(res["wall_s"], 1), "s")
        assert res["n"] == wl.n
        for form in DAY_FORMS[cfg]:
            tab = _table(sinet, wl, form)
            lab, out = sinet.pipeline(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"],
                                      w.t0, w.width, w.n_bins)
            torch.cuda.synchronize()
            assert _same_labels(sinet, d, lab, wl.n) is None, (cfg, form, _same_labels(sinet, d, lab, wl.n))
            err = _same_bins(sinet, res, out)
            assert err is None, (cfg, form, err)
            if form == "pla":
                assert tab.info().fallbacks == 0
            del lab, out, tab
            torch.cuda.empty_cache()
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


@pytest.mark.timeout(900, method="thread")
def test_batch_64_streams_every_stream(sinet, torch):
    """The benchmark's 64-stream batch, one autotuned plan launch, against the
    oracle stream by stream (each stream's own table, window and width)."""
    import sinetgen.gpu as gg
    streams = sinetgen.batch_streams()
    n_all = sum(s.n for s in streams)
    _say("batch", len(streams), "streams", n_all, "sessions")
    built = []
    for wl in streams:
        cols = gg.alloc_and_fill(wl)
        tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
        lab = torch.empty(wl.n, dtype=torch.uint8, device="cuda")
        built.append((wl, cols, tab, lab, sinet.new_hist(wl.window.n_bins)))
    torch.cuda.synchronize()
    bs = [sinet.BatchStream(tab, c["ts"], c["src"], c["dst"], c["bytes"], wl.window.t0,
                            wl.window.width, wl.window.n_bins, label=lab, out=out)
          for wl, c, tab, lab, out in built]
    plan = sinet.BatchPlan(bs, tune=sinet.autotune(bs))
    plan.run()
    torch.cuda.synchronize()
    tmp = _scratch(21 * n_all)
    try:
        dirs = [_host_columns(sinet, c, os.path.join(tmp, f"s{i}"), wl.n)
                for i, (wl, c, *_) in enumerate(built)]
        k = shards.cores()

        def one(i):
            wl = built[i][0]
            w = wl.window
            return shards.run(dirs[i], wl.pbase, wl.plen, w.t0, w.width, w.n_bins,
                              k=1 if wl.n <= 10_000_000 else 2)
        with ThreadPoolExecutor(max(1, k // 2)) as ex:
            results = list(ex.map(one, range(len(built))))
        for i, ((wl, c, tab, lab, out), res) in enumerate(zip(built, results)):
            assert _same_labels(sinet, dirs[i], lab, wl.n) is None, (i, wl.name)
            err = _same_bins(sinet, res, out)
            assert err is None, (i, wl.name, wl.window, err)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


@pytest.mark.timeout(600, method="thread")
def test_above_2_31_sessions(sinet, torch):
    """A day of 2^31 + 4,099 sessions (the full day's 200,000 prefixes and
    86.4 M bins, 43 GB of columns): the sliding-window reduce over all of it
    equals two calls over ragged halves (the second accumulating), and the
    record reduce, which cuts its input into pieces of at most 2^31 sessions,
    gives the same result; labels and bins are also checked against the
    oracle on sampled sessions (some beyond index 2^31) and sampled bins
    (among them the day's last, where those sessions land), and by
    conservation over every bin."""
    import oracle
    import sinetgen.gpu as gg
    n = (1 << 31) + 4099
    wl = sinetgen.config(5, n=n)
    w = wl.window
    _say("2^31 + 4099 sessions")
    cols = gg.alloc_and_fill(wl)
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    args = (w.t0, w.width, w.n_bins)
    lab, out = sinet.pipeline(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"], *args)
    torch.cuda.synchronize()
    h = (1 << 30) + 1237
    lab2 = torch.empty_like(lab)
    out2 = sinet.new_hist(w.n_bins)
    sinet.pipeline(tab, cols["ts"][:h], cols["src"][:h], cols["dst"][:h], cols["bytes"][:h], *args,
                   label=lab2[:h], out=out2)
    sinet.pipeline(tab, cols["ts"][h:], cols["src"][h:], cols["dst"][h:], cols["bytes"][h:], *args,
                   label=lab2[h:], out=out2, accumulate=True)
    torch.cuda.synchronize()
    assert torch.equal(lab2, lab)
    assert all(torch.equal(x, y) for x, y in zip(out2, out))
    del out2
    try:
        sinet.set_reduce("records")
        lab3, out3 = sinet.pipeline(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"], *args)
        torch.cuda.synchronize()
    finally:
        sinet.set_reduce("auto")
    assert torch.equal(lab3, lab)
    assert all(torch.equal(x, y) for x, y in zip(out3, out))
    del lab2, lab3, out3
    c, b, d = out
    # conservation over every bin
    per_label = torch.bincount(lab.long(), minlength=4)
    assert torch.equal(c.sum(dim=1) + d[:, 0], per_label) and int(per_label.sum()) == n
    assert (int(b.sum()) + int(d[:, 1].sum()) - int(cols["bytes"].sum())) % (1 << 64) == 0
    # sampled labels, the last sessions among them
    rng = np.random.default_rng(31)
    idx = np.unique(np.concatenate([rng.integers(0, n, 20_000), np.arange(n - 4099 - 8, n)]))
    s = sinetgen.sessions(wl, idx=idx)
    elab = oracle.classify(wl.pbase, wl.plen, s["src"], s["dst"], want_inst=False)
    assert np.array_equal(lab[torch.from_numpy(idx).cuda()].cpu().numpy(), elab)
    # sampled bins: every session within the jitter of the bin's time, recomputed
    for tb in list(rng.integers(0, w.n_bins, 3)) + [w.n_bins // 2, w.n_bins - 2, w.n_bins - 1]:
        tb = int(tb)
        lo_t = max(0, tb - wl.jitter - 1)
        hi_t = min(w.n_bins - 1, tb + wl.jitter + 1)
        i0, i1 = sinetgen.index_range_for_time(wl, lo_t, hi_t)
        if tb < wl.jitter + 1:
            i0 = 0
        if tb > w.n_bins - wl.jitter - 2:
            i1 = wl.n
        ss = sinetgen.sessions(wl, start=i0, stop=i1)
        sel = ss["ts"] == tb
        sl = oracle.classify(wl.pbase, wl.plen, ss["src"][sel], ss["dst"][sel], want_inst=False)
        ec, eb, _ = oracle.histogram(ss["ts"][sel] - np.uint32(tb), ss["bytes"][sel], sl, 0, 1, 1)
        assert np.array_equal(sinet.to_host_u64(c[:, tb]), ec[:, 0]), tb
        assert np.array_equal(sinet.to_host_u64(b[:, tb]), eb[:, 0]), tb
