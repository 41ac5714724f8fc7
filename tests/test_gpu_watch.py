"""GPU parity of the watch-list histograms (sections "AbuseIPDB" and
"GRIZZLY STEPPE") through the C ABI against the CPU oracle: every bin,
key and direction bit-identical, on small cases of every lookup kind and on
whole 10-minute bins of the full synthetic day."""
import sys

import numpy as np
import pytest

import oracle
import sinetgen

pytestmark = pytest.mark.gpu


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


def _up(sinet, s):
    return (sinet.to_device_u32(s["ts"]), sinet.to_device_u32(s["src"]),
            sinet.to_device_u32(s["dst"]), sinet.to_device_u64(s["bytes"]))


def _cmp(sinet, out, exp, n_keys, n_bins):
    c, b, d = out
    ec, eb, ed = exp
    assert np.array_equal(sinet.to_host_u64(c).reshape(2, n_keys, n_bins), ec), "count cells differ"
    assert np.array_equal(sinet.to_host_u64(b).reshape(2, n_keys, n_bins), eb), "byte cells differ"
    assert np.array_equal(sinet.to_host_u64(d).reshape(2, 2), ed), "dropped differ"


def _list_with_networks(wlist):
    """The list's /32 hosts plus a few /24 and /28 networks around some of
    them (nested rows: the longest match decides the key)."""
    nets = [(int(a) & 0xFFFFFF00, 24) for a in wlist.addrs[:6]] + \
           [(int(a) & 0xFFFFFFF0, 28) for a in wlist.addrs[3:9]]
    base = np.concatenate([wlist.addrs, np.array([a for a, _ in nets], np.uint32)])
    plen = np.concatenate([np.full(wlist.n, 32, np.uint8), np.array([z for _, z in nets], np.uint8)])
    return base, plen


@pytest.mark.parametrize("kind", ["scan", "bsearch", "trie", "pla"])
@pytest.mark.parametrize("per", ["host", "list"])
def test_watch_small_all_kinds(sinet, torch, kind, per):
    wl = sinetgen.config(1, n=400_009, seed=7)
    wlist = sinetgen.watch_lists(seed=7, sizes=(20, 37), frac=0.03)
    base, plen = _list_with_networks(wlist)
    if kind == "scan":
        base, plen = base[:60], plen[:60]
    rows = base.shape[0]
    if per == "host":
        keys, n_keys = np.arange(rows, dtype=np.uint32), rows
    else:
        keys = np.concatenate([wlist.lists, np.full(rows - wlist.n, 2, np.uint32)])[:rows]
        n_keys = 3
    _say("watch small", kind, per, rows)
    s = sinetgen.sessions(wl, watch=wlist)
    ts, src, dst, nb = _up(sinet, s)
    tab = sinet.Table(base, plen, inst=keys, kind=kind, inout_index=False)
    if kind == "pla":
        tab.train()
    # window cut on both ends, so both directions drop sessions
    for t0, width, n_bins in ((1_000, 1_000, 57), (2_500, 7, 5_000)):
        out = sinet.watch_histogram(tab, ts, src, dst, nb, t0, width, n_bins, n_keys)
        torch.cuda.synchronize()
        exp = oracle.watch(base, plen, s["ts"], s["src"], s["dst"], s["bytes"], t0, width, n_bins,
                           n_keys, inst=keys)
        _cmp(sinet, out, exp, n_keys, n_bins)
        assert exp[0].sum() > 0 and exp[2].sum() > 0


def test_watch_accumulate_unaligned_chunks(sinet, torch):
    """Chunks cut at arbitrary sessions (columns off 16-byte alignment run
    the one-session path) added into one histogram equal the whole."""
    wl = sinetgen.config(2, n=700_001)
    wlist = sinetgen.watch_lists(seed=3, sizes=(40, 60), frac=0.02)
    s = sinetgen.sessions(wl, watch=wlist)
    ts, src, dst, nb = _up(sinet, s)
    plen = np.full(wlist.n, 32, np.uint8)
    tab = sinet.Table(wlist.addrs, plen, kind="bsearch")
    t0, width, n_bins, n_keys = 0, 600_000, 144, wlist.n
    exp = oracle.watch(wlist.addrs, plen, s["ts"], s["src"], s["dst"], s["bytes"], t0, width,
                       n_bins, n_keys)
    acc = sinet.new_watch_hist(n_keys, n_bins)
    cuts = [0, 1, 6, 4_099, 350_003, wl.n]
    for a, b in zip(cuts[:-1], cuts[1:]):
        sinet.watch_histogram(tab, ts[a:b], src[a:b], dst[a:b], nb[a:b], t0, width, n_bins, n_keys,
                              out=acc, accumulate=a > 0)
    torch.cuda.synchronize()
    _cmp(sinet, acc, exp, n_keys, n_bins)


def test_watch_empty_input_and_bad_calls(sinet, torch):
    plen = np.full(3, 32, np.uint8)
    base = np.array([1, 2, 3], np.uint32)
    tab = sinet.Table(base, plen, kind="bsearch")
    e32 = torch.empty(0, dtype=torch.int32, device="cuda")
    e64 = torch.empty(0, dtype=torch.int64, device="cuda")
    out = sinet.new_watch_hist(3, 10)
    for t in out:
        t.fill_(5)
    sinet.watch_histogram(tab, e32, e32, e32, e64, 0, 1, 10, 3, out=out, accumulate=True)
    torch.cuda.synchronize()
    assert all(bool((t == 5).all()) for t in out)
    sinet.watch_histogram(tab, e32, e32, e32, e64, 0, 1, 10, 3, out=out)
    torch.cuda.synchronize()
    assert all(bool((t == 0).all()) for t in out)
    with pytest.raises(sinet.SinetError):   # row index 2 is not below n_keys = 2
        sinet.watch_histogram(tab, e32, e32, e32, e64, 0, 1, 10, 2)
    with pytest.raises(sinet.SinetError):
        sinet.watch_histogram(tab, e32, e32, e32, e64, 0, 0, 10, 3)
    mlp = sinet.Table(base, plen, kind="mlp")
    with pytest.raises(sinet.SinetError):   # learned table before training
        sinet.watch_histogram(mlp, e32, e32, e32, e64, 0, 1, 10, 3)


def test_device_watch_overlay_equals_host(sinet, torch):
    import sinetgen.gpu as gg
    wl = sinetgen.config(2, n=2_000_003)
    wlist = sinetgen.watch_lists()
    n, i0 = 300_007, 1_500_000
    src = torch.empty(n, dtype=torch.int32, device="cuda")
    dst = torch.empty(n, dtype=torch.int32, device="cuda")
    gg.fill(wl, None, src, dst, None, i0=i0, n=n)
    gg.watch_fill(wlist, src, dst, i0=i0)
    torch.cuda.synchronize()
    host = sinetgen.sessions(wl, start=i0, stop=i0 + n, watch=wlist)
    assert np.array_equal(sinet.to_host_u32(src), host["src"])
    assert np.array_equal(sinet.to_host_u32(dst), host["dst"])


def test_watch_full_day_whole_bins(sinet, torch):
    """The benchmark's watch workload: the 1.6e9-session day with the two
    lists' 1,177 hosts in 0.2% of the sources and destinations, one key per
    host, 10-minute bins.  Three whole bins (every key, both directions) are
    recomputed by the oracle from the index range that can reach them;
    counts are conserved over every cell."""
    import sinetgen.gpu as gg
    wl = sinetgen.config(5)
    wlist = sinetgen.watch_lists()
    _say("watch full day", wl.n, wlist.n)
    cols = gg.alloc_and_fill(wl)
    gg.watch_fill(wlist, cols["src"], cols["dst"])
    plen = np.full(wlist.n, 32, np.uint8)
    tab = sinet.Table(wlist.addrs, plen, kind="bsearch")
    t0, width, n_bins, n_keys = 0, 600_000, 144, wlist.n
    c, b, d = sinet.watch_histogram(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"], t0,
                                    width, n_bins, n_keys)
    torch.cuda.synchronize()
    addrs = torch.from_numpy(wlist.addrs.view(np.int32)).cuda()
    for dr, col in ((0, "src"), (1, "dst")):
        listed = int(torch.isin(cols[col], addrs).sum())
        assert int(c[dr].sum()) + int(d[dr, 0]) == listed
    assert int(d.sum()) == 0  # the day lies inside the window
    for tb in (0, 71, 143):
        lo_t = max(0, tb * width - wl.jitter - 1)
        hi_t = min(86_400_000 - 1, (tb + 1) * width + wl.jitter)
        i0, i1 = sinetgen.index_range_for_time(wl, lo_t, hi_t)
        if tb == 0:
            i0 = 0
        if tb == n_bins - 1:
            i1 = wl.n
        _say("watch bin", tb, i0, i1)
        ss = sinetgen.sessions(wl, start=i0, stop=i1, watch=wlist)
        ec, eb, _ = oracle.watch(wlist.addrs, plen, ss["ts"], ss["src"], ss["dst"], ss["bytes"],
                                 t0, width, n_bins, n_keys)
        got_c = sinet.to_host_u64(c[:, :, tb].contiguous())
        got_b = sinet.to_host_u64(b[:, :, tb].contiguous())
        assert np.array_equal(got_c, ec[:, :, tb]), tb
        assert np.array_equal(got_b, eb[:, :, tb]), tb
        assert ec[:, :, tb].sum() > 1000
