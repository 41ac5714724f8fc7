"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer outputs (labels, institution ids, interval indices, histogram bins,
dropped counters) must be bit-identical.  Sizes span many tiles plus ragged
tails; the full-day configuration is checked on sampled sessions and bins
that the oracle recomputes one by one, and by invariants over all bins.
"""
import sys

import numpy as np
import pytest

import oracle
import sinetgen
from oracle import learned

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


def _up(sinet, s, dev="cuda"):
    return (sinet.to_device_u32(s["ts"], dev), sinet.to_device_u32(s["src"], dev),
            sinet.to_device_u32(s["dst"], dev), sinet.to_device_u64(s["bytes"], dev))


def _cmp_hist(sinet, out, exp):
    c, b, d = out
    ec, eb, ed = exp
    assert np.array_equal(sinet.to_host_u64(c), ec), "count bins differ"
    assert np.array_equal(sinet.to_host_u64(b), eb), "byte bins differ"
    assert np.array_equal(sinet.to_host_u64(d), ed), "dropped differ"


# --------------------------------------------------------------- generator
def test_device_generator_equals_host(sinet, torch):
    import sinetgen.gpu as gg
    cases = [sinetgen.config(1, n=200_003), sinetgen.config(2, n=1_000_001),
             sinetgen.config(4, n=300_007), sinetgen.batch_streams()[5]]
    for wl in cases:
        _say("generator", wl.name, wl.n)
        n = min(wl.n, 300_007)
        dev = {c: torch.empty(n, dtype=torch.int64 if c == "bytes" else torch.int32, device="cuda")
               for c in ("ts", "src", "dst", "bytes")}
        i0 = wl.n - n
        gg.fill(wl, dev["ts"], dev["src"], dev["dst"], dev["bytes"], i0=i0, n=n)
        torch.cuda.synchronize()
        host = sinetgen.sessions(wl, start=i0, stop=wl.n)
        for c in ("ts", "src", "dst"):
            assert np.array_equal(sinet.to_host_u32(dev[c]), host[c]), (wl.name, c)
        assert np.array_equal(sinet.to_host_u64(dev["bytes"]), host["bytes"]), wl.name


# ---------------------------------------------------------- fused pipeline
@pytest.mark.parametrize("kind,inout", [("scan", False), ("bsearch", True), ("bsearch", False),
                                        ("trie", True), ("trie", False), ("auto", True)])
def test_pipeline_tiny_config_all_kinds(sinet, torch, kind, inout):
    wl = sinetgen.config(1)
    _say("pipeline tiny", kind, inout, wl.n)
    s = sinetgen.sessions(wl)
    ts, src, dst, nb = _up(sinet, s)
    w = wl.window
    tab = sinet.Table(wl.pbase, wl.plen, kind=kind, inout_index=inout)
    assert tab.info().inout_index == (1 if inout and kind != "auto" else 0) or kind == "auto"
    lab, out = sinet.pipeline(tab, ts, src, dst, nb, w.t0, w.width, w.n_bins)
    torch.cuda.synchronize()
    elab, ec, eb, ed = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"],
                                       w.t0, w.width, w.n_bins)
    assert np.array_equal(lab.cpu().numpy(), elab)
    _cmp_hist(sinet, out, (ec, eb, ed))


@pytest.mark.parametrize("t0,width,n_bins", [(1000, 1, 50_000), (777, 7, 5_000),
                                              (0, 1000, 50), (59_000, 3, 1), (0, 86_400_000, 1)])
def test_pipeline_windows_drop_and_divide(sinet, torch, t0, width, n_bins):
    wl = sinetgen.config(1, n=300_001)
    _say("window", t0, width, n_bins)
    s = sinetgen.sessions(wl)
    ts, src, dst, nb = _up(sinet, s)
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    lab, out = sinet.pipeline(tab, ts, src, dst, nb, t0, width, n_bins)
    torch.cuda.synchronize()
    elab, ec, eb, ed = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"],
                                       t0, width, n_bins)
    assert np.array_equal(lab.cpu().numpy(), elab)
    _cmp_hist(sinet, out, (ec, eb, ed))


def test_pipeline_day_shape_full_bins(sinet, torch):
    """Config-2 table and time shape, 3e6 sessions, all 86.4 M 1-ms bins."""
    wl = sinetgen.config(2, n=3_000_000)
    _say("day shape", wl.n)
    s = sinetgen.sessions(wl)
    ts, src, dst, nb = _up(sinet, s)
    w = wl.window
    for kind, inout in (("bsearch", True), ("bsearch", False), ("trie", False), ("pla", False)):
        tab = sinet.Table(wl.pbase, wl.plen, kind=kind, inout_index=inout)
        if kind == "pla":
            tab.train()
        assert tab.info().inout_index == int(inout)
        lab, out = sinet.pipeline(tab, ts, src, dst, nb, w.t0, w.width, w.n_bins)
        torch.cuda.synchronize()
        if kind == "bsearch" and inout:
            elab, ec, eb, ed = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"],
                                               s["bytes"], w.t0, w.width, w.n_bins)
        assert np.array_equal(lab.cpu().numpy(), elab), kind
        _cmp_hist(sinet, out, (ec, eb, ed))
        del out


def test_phase_timing_counts_calls_and_keeps_results(sinet, torch):
    """Timed calls record their phases and compute the same histogram."""
    wl = sinetgen.config(2, n=1_000_003)
    s = sinetgen.sessions(wl)
    ts, src, dst, nb = _up(sinet, s)
    w = wl.window
    elab, ec, eb, ed = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"],
                                       w.t0, w.width, w.n_bins)
    tab = sinet.Table(wl.pbase, wl.plen, kind="trie", inout_index=False)  # separate lookup pass
    sinet.timing_enable(True)
    try:
        for _ in range(2):
            lab, out = sinet.pipeline(tab, ts, src, dst, nb, w.t0, w.width, w.n_bins)
            assert np.array_equal(lab.cpu().numpy(), elab)
            _cmp_hist(sinet, out, (ec, eb, ed))
            del out
        # a small window takes the private-histogram pass (stage-1 phase only)
        sinet.pipeline(tab, ts, src, dst, nb, w.t0, 60_000, 1441)
        t = sinet.timing_read()
    finally:
        sinet.timing_enable(False)
    _say("timing", t)
    assert t["calls"] == 3 and t["stage1_launches"] == 3
    for k in ("lookup_ms", "stage1_ms", "index_ms", "stage2_ms"):
        assert t[k] > 0.0, k
    sinet.pipeline(tab, ts, src, dst, nb, w.t0, w.width, w.n_bins)
    sinet.timing_enable(True)
    t2 = sinet.timing_read()
    sinet.timing_enable(False)
    assert t2["calls"] == 0 and t2["stage1_ms"] == 0.0


# ------------------------------------------------------------ discrimination
@pytest.mark.parametrize("kind", ["scan", "bsearch", "trie"])
def test_discriminate_institutions(sinet, torch, kind):
    wl = sinetgen.config(2, n=500_003)
    _say("discriminate", kind)
    s = sinetgen.sessions(wl, start=0, stop=wl.n)
    inst = (np.arange(wl.n_prefix, dtype=np.uint32) * 2654435761) & 0x7FFFFFFF
    tab = sinet.Table(wl.pbase, wl.plen, inst=inst, kind=kind)
    src, dst = sinet.to_device_u32(s["src"]), sinet.to_device_u32(s["dst"])
    lab, si, di = sinet.discriminate(tab, src, dst, label=True, src_inst=True, dst_inst=True)
    torch.cuda.synchronize()
    elab, esi, edi = oracle.classify(wl.pbase, wl.plen, s["src"], s["dst"], inst=inst)
    assert np.array_equal(lab.cpu().numpy(), elab)
    assert np.array_equal(sinet.to_host_u32(si), esi)
    assert np.array_equal(sinet.to_host_u32(di), edi)
    # institution only (no label buffer)
    _, si2, _ = sinet.discriminate(tab, src, dst, label=False, src_inst=True)
    torch.cuda.synchronize()
    assert np.array_equal(sinet.to_host_u32(si2), esi)


def test_histogram_entry_and_accumulate(sinet, torch):
    wl = sinetgen.config(1, n=400_009)
    _say("histogram entry")
    s = sinetgen.sessions(wl)
    lab = oracle.classify(wl.pbase, wl.plen, s["src"], s["dst"], want_inst=False)
    ts, _, _, nb = _up(sinet, s)
    lt = torch.from_numpy(lab).cuda()
    t0, w, n_bins = 500, 3, 19_000
    out = sinet.histogram(ts, nb, lt, t0, w, n_bins)
    torch.cuda.synchronize()
    exp = oracle.histogram(s["ts"], s["bytes"], lab, t0, w, n_bins)
    _cmp_hist(sinet, out, exp)
    # the paper's two-stage merge: chunks added into one histogram
    acc = sinet.new_hist(n_bins)
    cuts = [0, 1, 5, 4099, 100_000, 250_001, wl.n]
    for a, b in zip(cuts[:-1], cuts[1:]):
        sinet.histogram(ts[a:b], nb[a:b], lt[a:b], t0, w, n_bins, out=acc, accumulate=a > 0)
    torch.cuda.synchronize()
    _cmp_hist(sinet, acc, exp)


@pytest.mark.parametrize("n_bins,co,bo", [(5_122, 0, 2), (5_122, 6, 14), (4_104, 4, 10),
                                          (3_073, 0, 1), (5_122, 9, 3)])
def test_histogram_rows_off_line_boundaries(sinet, torch, n_bins, co, bo):
    """Output rows that start anywhere relative to 128-byte lines (the row
    stride n_bins * 8 and the buffers' own offsets), with 16- and 8-byte
    stores: every bin is written once, nothing outside the rows is touched."""
    wl = sinetgen.config(1, n=300_007)
    _say("histogram rows", n_bins, co, bo)
    s = sinetgen.sessions(wl)
    lab = oracle.classify(wl.pbase, wl.plen, s["src"], s["dst"], want_inst=False)
    ts, _, _, nb = _up(sinet, s)
    lt = torch.from_numpy(lab).cuda()
    t0, w = 100, 1
    exp = oracle.histogram(s["ts"], s["bytes"], lab, t0, w, n_bins)
    guard = -7
    bc = torch.full((co + 4 * n_bins + 5,), guard, dtype=torch.int64, device="cuda")
    bb = torch.full((bo + 4 * n_bins + 5,), guard, dtype=torch.int64, device="cuda")
    out = (bc[co:co + 4 * n_bins].view(4, n_bins), bb[bo:bo + 4 * n_bins].view(4, n_bins),
           torch.empty((4, 2), dtype=torch.int64, device="cuda"))
    sinet.histogram(ts, nb, lt, t0, w, n_bins, out=out)
    torch.cuda.synchronize()
    _cmp_hist(sinet, out, exp)
    # accumulate onto earlier contents
    base_c = torch.arange(4 * n_bins, dtype=torch.int64, device="cuda").view(4, n_bins) * 3
    base_b = torch.arange(4 * n_bins, dtype=torch.int64, device="cuda").view(4, n_bins) * 5 + 11
    out[0].copy_(base_c)
    out[1].copy_(base_b)
    out[2].zero_()
    sinet.histogram(ts, nb, lt, t0, w, n_bins, out=out, accumulate=True)
    torch.cuda.synchronize()
    ec, eb, ed = exp
    _cmp_hist(sinet, out, (ec + sinet.to_host_u64(base_c), eb + sinet.to_host_u64(base_b), ed))
    for buf, off in ((bc, co), (bb, bo)):
        h = buf.cpu().numpy()
        assert (h[:off] == guard).all() and (h[off + 4 * n_bins:] == guard).all(), \
            "a write outside the histogram rows"


def test_pipeline_chunked_accumulate_equals_whole(sinet, torch):
    wl = sinetgen.config(2, n=1_000_000)
    _say("chunked accumulate")
    s = sinetgen.sessions(wl)
    ts, src, dst, nb = _up(sinet, s)
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    t0, w, n_bins = 0, 10, 8_640_000
    lab, whole = sinet.pipeline(tab, ts, src, dst, nb, t0, w, n_bins)
    acc = sinet.new_hist(n_bins)
    labs = torch.empty_like(lab)
    cuts = [0, 3, 333_333, 333_337, 999_999, wl.n]
    for a, b in zip(cuts[:-1], cuts[1:]):
        sinet.pipeline(tab, ts[a:b], src[a:b], dst[a:b], nb[a:b], t0, w, n_bins, label=labs[a:b],
                       out=acc, accumulate=a > 0)
    torch.cuda.synchronize()
    assert torch.equal(lab, labs)
    for x, y in zip(whole, acc):
        assert torch.equal(x, y)


# ------------------------------------------------------------- edge cases
def _edge_table():
    # /0 default route, /32 host, duplicates, nested, adjacent blocks, top of space
    rows = [(0x00000000, 0), (0xCB007105, 32), (0xAC100000, 12), (0xAC100000, 12),
            (0xAC100500, 24), (0xC0000200, 24), (0xC0000300, 24), (0xFFFFFFFF, 32),
            (0xFFFFFF00, 24), (0x0A000000, 8), (0x0A010000, 16)]
    b = np.array([r[0] for r in rows], np.uint32)
    l = np.array([r[1] for r in rows], np.uint8)
    return b, l


@pytest.mark.parametrize("kind", ["scan", "bsearch", "trie"])
def test_edge_tables_and_ragged_sizes(sinet, torch, kind):
    b, l = _edge_table()
    _say("edge", kind)
    rng = np.random.default_rng(5)
    special = np.array([0, 1, 0xCB007104, 0xCB007105, 0xCB007106, 0xAC0FFFFF, 0xAC100000,
                        0xAC1004FF, 0xAC100500, 0xAC1005FF, 0xAC100600, 0xAC1FFFFF, 0xAC200000,
                        0xC00001FF, 0xC0000200, 0xC00003FF, 0xC0000400, 0xFFFFFEFF, 0xFFFFFF00,
                        0xFFFFFFFE, 0xFFFFFFFF, 0x0A000000, 0x0A00FFFF, 0x0A010000, 0x0A01FFFF,
                        0x0A020000, 0x0AFFFFFF, 0x0B000000], np.uint32)
    for n in (1, 2, 3, 5, 63, 64, 65, 1023, 4097, 65_537):
        src = np.concatenate([special, rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)])[:n]
        dst = np.roll(src, 1)
        ts = rng.integers(0, 2000, n).astype(np.uint32)
        by = rng.integers(0, 1 << 63, n, dtype=np.uint64) | np.uint64(1 << 63)  # wraps mod 2^64
        s = {"ts": ts, "src": src, "dst": dst, "bytes": by}
        for off in (0, 1):  # off = 1: unaligned device pointers (scalar path)
            T, S, D, B = _up(sinet, {k: np.concatenate([v[:1], v]) if off else v for k, v in s.items()})
            T, S, D, B = T[off:], S[off:], D[off:], B[off:]
            tab = sinet.Table(b, l, kind=kind)
            lab, out = sinet.pipeline(tab, T, S, D, B, 100, 1, 1500)
            _, si, di = sinet.discriminate(tab, S, D, label=False, src_inst=True, dst_inst=True)
            torch.cuda.synchronize()
            elab, ec, eb, ed = oracle.pipeline(b, l, ts, src, dst, by, 100, 1, 1500)
            _, esi, edi = oracle.classify(b, l, src, dst)
            assert np.array_equal(lab.cpu().numpy(), elab), (n, off)
            _cmp_hist(sinet, out, (ec, eb, ed))
            assert np.array_equal(sinet.to_host_u32(si), esi)
            assert np.array_equal(sinet.to_host_u32(di), edi)


def _dense_tables():
    """Tables whose union cuts /16 blocks many times: /24s and /28s packed in
    two blocks (more than four boundaries per block), single hosts at block
    offsets 5, 9 and 0xFFFF, and 3000 random hosts."""
    rng = np.random.default_rng(11)
    b = ([0x0A000000 + (i << 8) for i in range(0, 200, 3)] +
         [0x0A010000 + (i << 4) for i in range(0, 4000, 7)] +
         [0x0A020005, 0x0A020009, 0x0A02FFFF, 0x0A030000, 0x0A04FFFF])
    l = [24] * 67 + [28] * len(range(0, 4000, 7)) + [32, 32, 32, 32, 32]
    hosts = rng.integers(0, 1 << 32, 3000, dtype=np.uint64).astype(np.uint32)
    return [(np.array(b, np.uint32), np.array(l, np.uint8)),
            (hosts, np.full(3000, 32, np.uint8))]


def test_inout_index_dense_blocks(sinet, torch):
    """Label-only lookups through the in/out index at every union boundary
    and its neighbours, at block edges and at random addresses."""
    rng = np.random.default_rng(12)
    for b, l in _dense_tables():
        B, own = oracle.endpoints(b, l)
        inn = (own != 0).astype(np.int8)
        U = B[np.concatenate([[inn[0] == 1], inn[1:] != inn[:-1]])].astype(np.int64)
        near = (U[:, None] + np.arange(-2, 3)[None, :]).ravel() % (1 << 32)
        blocks = np.unique(U >> 16)
        edges = np.concatenate([blocks << 16, (blocks << 16) | 0xFFFF, (blocks << 16) | 0x7FFF])
        rand = rng.integers(0, 1 << 32, 200_003, dtype=np.uint64)
        src = np.concatenate([near, edges, rand]).astype(np.uint32)
        dst = rng.permutation(src)
        tab = sinet.Table(b, l, kind="bsearch")
        assert tab.info().inout_index == 1
        S, D = sinet.to_device_u32(src), sinet.to_device_u32(dst)
        lab, _, _ = sinet.discriminate(tab, S, D)
        torch.cuda.synchronize()
        elab, _, _ = oracle.classify(b, l, src, dst)
        assert np.array_equal(lab.cpu().numpy(), elab)


@pytest.mark.parametrize("kind", ["bsearch", "trie"])
def test_byte_magnitudes_and_record_overflow(sinet, torch, kind):
    """Byte counts of every magnitude (one to four 17-bit part records, and
    the far path from 2^52 on), sorted and shuffled time order, and chunks
    whose large counts exceed the extra record slots."""
    wl = sinetgen.config(1)
    rng = np.random.default_rng(21)
    n = 3 * 2048 * 7 + 123
    k = rng.integers(0, 64, n)
    by = (np.uint64(1) << k.astype(np.uint64)) + rng.integers(0, 1 << 16, n).astype(np.uint64)
    by[: 2048 * 3] = (np.uint64(1) << np.uint64(40)) + rng.integers(0, 1 << 30, 2048 * 3).astype(np.uint64)
    ts = np.sort(rng.integers(0, 3_000_000, n)).astype(np.uint32)
    s = sinetgen.sessions(wl, start=0, stop=n)
    for order in ("sorted", "shuffled"):
        t = ts if order == "sorted" else rng.permutation(ts)
        T, S, D, B = _up(sinet, {"ts": t, "src": s["src"], "dst": s["dst"], "bytes": by})
        tab = sinet.Table(wl.pbase, wl.plen, kind=kind)
        lab, out = sinet.pipeline(tab, T, S, D, B, 0, 1, 3_000_000)
        torch.cuda.synchronize()
        elab, ec, eb, ed = oracle.pipeline(wl.pbase, wl.plen, t, s["src"], s["dst"], by, 0, 1,
                                           3_000_000)
        assert np.array_equal(lab.cpu().numpy(), elab), order
        _cmp_hist(sinet, out, (ec, eb, ed))


def test_empty_input_clears_or_keeps(sinet, torch):
    b, l = _edge_table()
    tab = sinet.Table(b, l, kind="bsearch")
    e32 = torch.empty(0, dtype=torch.int32, device="cuda")
    e64 = torch.empty(0, dtype=torch.int64, device="cuda")
    out = sinet.new_hist(77)
    for t in out:
        t.fill_(5)
    sinet.pipeline(tab, e32, e32, e32, e64, 0, 1, 77, out=out, accumulate=True)
    torch.cuda.synchronize()
    assert all(int(t.min()) == 5 and int(t.max()) == 5 for t in out)
    sinet.pipeline(tab, e32, e32, e32, e64, 0, 1, 77, out=out, accumulate=False)
    torch.cuda.synchronize()
    assert all(int(t.abs().max()) == 0 for t in out)


def test_unsupported_and_bad_calls_raise(sinet, torch):
    b, l = _edge_table()
    tab = sinet.Table(b, l, kind="pla")
    x = torch.zeros(8, dtype=torch.int32, device="cuda")
    with pytest.raises(sinet.SinetError):
        sinet.discriminate(tab, x, x)           # learned table before training
    tab2 = sinet.Table(b, l, kind="bsearch")
    with pytest.raises(sinet.SinetError):
        sinet.pipeline(tab2, x, x, x, x.long(), 0, 0, 10)   # width 0
    # sizes the kernels would read or write past: refused before any launch
    short = torch.zeros(7, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        sinet.pipeline(tab2, x, short, x, x.long(), 0, 1, 10)
    with pytest.raises(ValueError):
        sinet.pipeline(tab2, x, x, x, x, 0, 1, 10)         # 4-byte byte counts
    with pytest.raises(ValueError):
        sinet.pipeline(tab2, x, x, x, x.long(), 0, 1, 10, out=sinet.new_hist(9))
    with pytest.raises(ValueError):
        sinet.pipeline(tab2, x, x, x, x.long(), 0, 1, 10,
                       label=torch.zeros(7, dtype=torch.uint8, device="cuda"))
    with pytest.raises(ValueError):
        sinet.discriminate(tab2, x, short)
    with pytest.raises(ValueError):
        sinet.histogram(x, x.long(), short.to(torch.uint8), 0, 1, 10)
    with pytest.raises(ValueError):
        sinet.BatchStream(tab2, x, x, x, x.long(), 0, 1, 10, out=sinet.new_hist(5))


# ------------------------------------------------------ intervals/positions
@pytest.mark.parametrize("cfg", [1, 2, 4])
def test_intervals_and_positions(sinet, torch, cfg):
    wl = sinetgen.config(cfg, n=10)
    _say("positions cfg", cfg)
    B, own = oracle.endpoints(wl.pbase, wl.plen)
    rng = np.random.default_rng(cfg)
    hi = np.concatenate([B[1:] - 1, [0xFFFFFFFF]]).astype(np.uint32)
    q = np.concatenate([B, hi, rng.integers(0, 1 << 32, 200_001, dtype=np.uint64).astype(np.uint32)])
    expect = learned.positions(B, q)
    qd = sinet.to_device_u32(q)
    kinds = ["bsearch", "bsearch_global", "trie", "pla", "mlp"] + (["scan"] if wl.n_prefix <= 1024 else [])
    for kind in kinds:
        tab = sinet.Table(wl.pbase, wl.plen, kind=kind.replace("_global", ""),
                          global_bsearch=kind.endswith("_global"))
        gB, gown = tab.intervals()
        assert np.array_equal(gB, B) and np.array_equal(gown, own), kind
        modes = [{}]
        if kind == "mlp":
            modes = [{"steps": 300}]
        if kind == "pla":   # error-bounded segmentation, and 256 least-squares segments
            modes = [{}, {"target_err": 2}, {"segments": 256}]
        for mode in modes:
            if kind in ("pla", "mlp"):
                tab.train(**mode)
            pos = tab.position(qd)
            torch.cuda.synchronize()
            assert np.array_equal(sinet.to_host_u32(pos).astype(np.int64), expect), (kind, mode)
            if kind == "pla":
                assert tab.info().fallbacks == 0, mode


# ---------------------------------------------------------- full-size day
@pytest.mark.parametrize("cfg", [2, 5])
def test_full_day_sampled_and_invariants(sinet, torch, cfg):
    """The 1e8-session day (1,024 prefixes) and the 1.6e9-session day
    (200,000 prefixes), both with 86.4 M 1-ms bins, in the launch the
    benchmark times: sampled labels and bins recomputed by the oracle,
    conservation over every bin; on the large day the learned PLA form must
    give the same labels and bins as the plain form."""
    import sinetgen.gpu as gg
    wl = sinetgen.config(cfg)
    _say("full day", cfg, wl.n)
    cols = gg.alloc_and_fill(wl)
    w = wl.window
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    lab, (c, b, d) = sinet.pipeline(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"],
                                    w.t0, w.width, w.n_bins)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    idx = np.unique(np.concatenate([rng.integers(0, wl.n, 20_000), [0, 1, wl.n - 1]]))
    s = sinetgen.sessions(wl, idx=idx)
    elab = oracle.classify(wl.pbase, wl.plen, s["src"], s["dst"], want_inst=False)
    assert np.array_equal(lab[torch.from_numpy(idx).cuda()].cpu().numpy(), elab)
    # conservation: every session lands in exactly one (label, bin) or dropped
    per_label = torch.bincount(lab.long(), minlength=4)
    assert torch.equal(c.sum(dim=1) + d[:, 0], per_label)
    assert int(per_label.sum()) == wl.n
    tot_bytes = int(cols["bytes"].sum())  # sum of the input column (int64 wraps like u64)
    assert (int(b.sum()) + int(d[:, 1].sum()) - tot_bytes) % (1 << 64) == 0
    # sampled bins: every session whose un-jittered time is within the jitter
    for tb in list(rng.integers(0, w.n_bins, 6)) + [0, 1, 4999, w.n_bins - 1]:
        tb = int(tb)
        lo_t = max(0, tb - wl.jitter - 1)
        hi_t = min(w.n_bins - 1, tb + wl.jitter + 1)
        i0, i1 = sinetgen.index_range_for_time(wl, lo_t, hi_t)
        if tb < wl.jitter + 1:  # reflected at the day's start
            i0 = 0
        if tb > w.n_bins - wl.jitter - 2:
            i1 = wl.n
        ss = sinetgen.sessions(wl, start=i0, stop=i1)
        sel = ss["ts"] == tb
        sl = oracle.classify(wl.pbase, wl.plen, ss["src"][sel], ss["dst"][sel], want_inst=False)
        ec, eb, _ = oracle.histogram(ss["ts"][sel] - np.uint32(tb), ss["bytes"][sel], sl, 0, 1, 1)
        got_c = sinet.to_host_u64(c[:, tb])
        got_b = sinet.to_host_u64(b[:, tb])
        assert np.array_equal(got_c, ec[:, 0]), tb
        assert np.array_equal(got_b, eb[:, 0]), tb
    if cfg == 5:
        pla = sinet.Table(wl.pbase, wl.plen, kind="pla", inout_index=False)
        pla.train()
        lab2, (c2, b2, d2) = sinet.pipeline(pla, cols["ts"], cols["src"], cols["dst"],
                                            cols["bytes"], w.t0, w.width, w.n_bins)
        torch.cuda.synchronize()
        assert pla.info().pla_window == 1 and pla.info().fallbacks == 0
        assert torch.equal(lab2, lab)
        assert torch.equal(c2, c) and torch.equal(b2, b) and torch.equal(d2, d)


# ---------------------------------------------------------------- learned
def test_mlp_gradients_vs_oracle(sinet, torch):
    wl = sinetgen.config(4, n=10)
    B, _ = oracle.endpoints(wl.pbase, wl.plen)
    x, y = learned.training_set(B)
    rng = np.random.default_rng(4)
    for trial in range(3):
        p = learned.mlp_init_hinges() + rng.normal(0, 0.2, learned.N_PARAMS)
        p32 = p.astype(np.float32)
        x32 = (B.astype(np.float32) * np.float32(2.0 ** -32)).astype(np.float32)
        y32 = (np.arange(len(B)) / len(B)).astype(np.float32)
        loss, g = sinet.mlp_loss_grad(torch.from_numpy(p32).cuda(), torch.from_numpy(x32).cuda(),
                                      torch.from_numpy(y32).cuda())
        torch.cuda.synchronize()
        eloss, eg = learned.mlp_loss_grad(p32.astype(np.float64), x32.astype(np.float64),
                                          y32.astype(np.float64))
        scale = learned.mlp_grad_abs_sum(p32.astype(np.float64), x32.astype(np.float64),
                                         y32.astype(np.float64))
        gg_ = g.cpu().numpy().astype(np.float64)
        tol = 1e-5 * (scale + np.abs(eg)) + 1e-12
        assert np.all(np.abs(gg_ - eg) <= tol), (trial, np.max(np.abs(gg_ - eg) / tol))
        assert abs(float(loss.item()) - eloss) <= 1e-5 * eloss + 1e-12


@pytest.mark.parametrize("kind,inout", [("pla", False), ("mlp", False), ("pla", True),
                                        ("pla256", False), ("bsearch", False),
                                        ("bsearch_global", False), ("trie", False)])
def test_learned_lookup_exact_and_trained_beats_untrained(sinet, torch, kind, inout):
    """The 200,000-prefix clustered table: labels and histograms of every
    kind, with the kind's own search (in/out index off) and with the index."""
    wl = sinetgen.config(4, n=2_000_000)
    _say("large table", kind, inout)
    s = sinetgen.sessions(wl, start=0, stop=wl.n)
    ts, src, dst, nb = _up(sinet, s)
    tab = sinet.Table(wl.pbase, wl.plen, kind=kind.replace("_global", "").replace("256", ""),
                      inout_index=inout, global_bsearch=kind.endswith("_global"))
    assert tab.info().inout_index == int(inout)
    if kind not in ("pla", "pla256", "mlp"):
        w = wl.window
        lab, out = sinet.pipeline(tab, ts, src, dst, nb, w.t0, w.width, w.n_bins)
        torch.cuda.synchronize()
        elab, ec, eb, ed = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"],
                                           s["bytes"], w.t0, w.width, w.n_bins)
        assert np.array_equal(lab.cpu().numpy(), elab)
        _cmp_hist(sinet, out, (ec, eb, ed))
        return
    # the 256-segment PLA's bound is too wide for one window: its leaves are
    # read by quads of lanes in the lookup pass's queue
    rep = tab.train(segments=256) if kind == "pla256" else tab.train(steps=1500)
    info = tab.info()
    assert info.trained == 1 and info.max_err == rep.max_err
    if kind == "mlp":
        assert rep.loss_last < rep.loss_first
        assert rep.max_err < rep.max_err_untrained
    w = wl.window
    lab, out = sinet.pipeline(tab, ts, src, dst, nb, w.t0, w.width, w.n_bins)
    torch.cuda.synchronize()
    elab, ec, eb, ed = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"],
                                       w.t0, w.width, w.n_bins)
    assert np.array_equal(lab.cpu().numpy(), elab)
    _cmp_hist(sinet, out, (ec, eb, ed))
    if kind == "pla":
        assert tab.info().fallbacks == 0
        # the bound is small enough for one 16-boundary window per lookup
        assert tab.info().pla_window == 1 and tab.info().max_err <= 6
    if kind == "pla256":
        assert tab.info().fallbacks == 0 and tab.info().pla_window == 0 and tab.info().segments == 256


def test_learned_forced_fallback_stays_exact(sinet, torch):
    """A model whose bound is wrong (weights replaced from the host) must
    still give exact positions through the bracket check, and count its
    fallbacks."""
    wl = sinetgen.config(4, n=10)
    B, _ = oracle.endpoints(wl.pbase, wl.plen)
    rng = np.random.default_rng(1)
    q = rng.integers(0, 1 << 32, 100_000, dtype=np.uint64).astype(np.uint32)
    qd = sinet.to_device_u32(q)
    for kind in ("mlp", "pla"):
        tab = sinet.Table(wl.pbase, wl.plen, kind=kind)
        tab.train(steps=200)
        k, model, err = tab.get_model()
        assert k == kind and err == tab.info().max_err
        if kind == "mlp":
            tab.set_model(params=model, max_err=0)            # bound forced too small
        else:
            tab.set_model(pla=model, max_err=0)
        pos = tab.position(qd)
        torch.cuda.synchronize()
        assert np.array_equal(sinet.to_host_u32(pos).astype(np.int64), learned.positions(B, q))
        assert tab.info().fallbacks > 0
        # labels only, with the same wrong bound, at every boundary and the
        # address below it, and a ragged tail of unqueued waves: the lookup
        # pass's queued search (the PLA's window, or the MLP's leaf found
        # through the full search over the sample), read by quads of lanes
        tl = sinet.Table(wl.pbase, wl.plen, kind=kind, inout_index=False)
        if kind == "pla":
            tl.set_model(pla=model, max_err=0)
            assert tl.info().pla_window == 1
        else:
            tl.set_model(params=model, max_err=0)
        src = np.concatenate([B, B - 1, q[:7]]).astype(np.uint32)
        dst = rng.permutation(src)
        lab, _, _ = sinet.discriminate(tl, sinet.to_device_u32(src), sinet.to_device_u32(dst))
        torch.cuda.synchronize()
        elab, _, _ = oracle.classify(wl.pbase, wl.plen, src, dst)
        assert np.array_equal(lab.cpu().numpy(), elab)
        assert tl.info().fallbacks > 0
        # reloading with a measured bound restores exact, fallback-free PLA lookups
        if kind == "pla":
            tab2 = sinet.Table(wl.pbase, wl.plen, kind=kind)
            tab2.set_model(pla=model)
            assert tab2.info().max_err == err
            pos2 = tab2.position(qd)
            torch.cuda.synchronize()
            assert np.array_equal(sinet.to_host_u32(pos2).astype(np.int64), learned.positions(B, q))
            assert tab2.info().fallbacks == 0


def test_leaf_sizes_of_a_larger_table(sinet, torch):
    """150,000 random host routes (about 300,000 interval boundaries): the
    sampled binary search keeps leaves of 32 boundaries in global memory (read
    by quads of lanes, two 16-byte loads per lane), the learned kinds leaves of
    64 (the queue's drain of two searches per lane).  Labels of 1,000,003
    sessions, half of their endpoints on or next to a listed host, against
    the oracle."""
    rng = np.random.default_rng(31)
    hosts = np.unique(rng.integers(0, 1 << 32, 150_000, dtype=np.uint64)).astype(np.uint32)
    plen = np.full(hosts.shape[0], 32, np.uint8)
    n = 1_000_003
    near = rng.choice(hosts, n // 2) + rng.integers(0, 2, n // 2, dtype=np.uint32)
    src = np.concatenate([near, rng.integers(0, 1 << 32, n - n // 2, dtype=np.uint64)]).astype(np.uint32)
    dst = rng.permutation(src)
    elab = oracle.classify(hosts, plen, src, dst, want_inst=False)
    S, D = sinet.to_device_u32(src), sinet.to_device_u32(dst)
    for kind in ("bsearch", "mlp", "pla"):
        _say("larger table", kind)
        tab = sinet.Table(hosts, plen, kind=kind, inout_index=False)
        assert tab.info().m > 262_144
        if kind == "mlp":
            tab.train(steps=300)
        elif kind == "pla":
            tab.train(segments=256)
        lab, _, _ = sinet.discriminate(tab, S, D)
        torch.cuda.synchronize()
        assert np.array_equal(lab.cpu().numpy(), elab), kind
        if kind != "bsearch":
            assert tab.info().fallbacks == 0, kind


# ------------------------------------------------------------------ batching
def _batch_setup(sinet, torch, n_streams=10, total=2_000_000, inout=True):
    import sinetgen.gpu as gg
    streams = sinetgen.batch_streams(seed=33, n_streams=n_streams, total=total, hist_cap=3 << 30)
    # two coarse streams whose histograms fit in LDS (the private path)
    # (the tail beyond their last bin is dropped)
    streams[0].window = sinetgen.Window(streams[0].t_origin, 1000, 500)
    streams[1].window = sinetgen.Window(streams[1].t_origin + 123, 997, 1000)
    built = []
    for k, wl in enumerate(streams):
        cols = gg.alloc_and_fill(wl)
        if k == 3:  # columns one element off 16-byte alignment: this stream's scalar path
            for key in list(cols):
                big = torch.empty(wl.n + 1, dtype=cols[key].dtype, device="cuda")
                big[1:].copy_(cols[key])
                cols[key] = big[1:]
        # stream 2 uses the table's own search (a second kernel kind in the batch)
        tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch", inout_index=inout and k != 2)
        lab = torch.empty(wl.n, dtype=torch.uint8, device="cuda")
        out = sinet.new_hist(wl.window.n_bins)
        built.append((wl, cols, tab, lab, out))
    torch.cuda.synchronize()
    return built


def _bstreams(sinet, built):
    return [sinet.BatchStream(tab, c["ts"], c["src"], c["dst"], c["bytes"], wl.window.t0,
                              wl.window.width, wl.window.n_bins, label=lab, out=out)
            for wl, c, tab, lab, out in built]


def test_batch_equals_per_stream_and_oracle(sinet, torch):
    built = _batch_setup(sinet, torch)
    _say("batch", [wl.n for wl, *_ in built])
    plan = sinet.BatchPlan(_bstreams(sinet, built))
    ref = []
    for wl, c, tab, lab, out in built:
        l2, o2 = sinet.pipeline(tab, c["ts"], c["src"], c["dst"], c["bytes"], wl.window.t0,
                                wl.window.width, wl.window.n_bins)
        ref.append((l2, o2))
    for rep in range(3):   # graph replays, with eager work in between
        for _, _, _, lab, out in built:
            lab.fill_(7)
            for t in out:
                t.fill_(-1)
        plan.run()
        torch.cuda.synchronize()
        for (wl, c, tab, lab, out), (l2, o2) in zip(built, ref):
            assert torch.equal(lab, l2), (rep, wl.name)
            for x, y in zip(out, o2):
                assert torch.equal(x, y), (rep, wl.name)
        _ = torch.randn(1000, device="cuda").sum()
    # oracle on four streams (host regeneration), the unaligned one included
    for wl, c, tab, lab, out in built[:4]:
        s = sinetgen.sessions(wl)
        w = wl.window
        elab, ec, eb, ed = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"],
                                           w.t0, w.width, w.n_bins)
        assert np.array_equal(lab.cpu().numpy(), elab), wl.name
        _cmp_hist(sinet, out, (ec, eb, ed))


def test_batch_with_separate_lookup_pass(sinet, torch):
    """Streams whose lookups walk global memory (trie, learned PLA and MLP,
    in/out index off) run a batched lookup pass that stores the labels, then
    stage 1 on stored labels: outputs equal per-stream calls and the oracle,
    also for a stream without label output (plan-owned buffer) and one whose
    label output is off 4-byte alignment."""
    import sinetgen.gpu as gg
    streams = sinetgen.batch_streams(seed=41, n_streams=6, total=1_500_000, hist_cap=2 << 30)
    kinds = ["trie", "pla", "mlp", "pla", "trie", "bsearch"]
    built = []
    for k, wl in enumerate(streams):
        cols = gg.alloc_and_fill(wl)
        tab = sinet.Table(wl.pbase, wl.plen, kind=kinds[k], inout_index=False)
        if kinds[k] in ("pla", "mlp"):
            tab.train(steps=300)
        if k == 1:
            lab = None
        elif k == 4:
            lab = torch.empty(wl.n + 1, dtype=torch.uint8, device="cuda")[1:]
        else:
            lab = torch.empty(wl.n, dtype=torch.uint8, device="cuda")
        out = sinet.new_hist(wl.window.n_bins)
        built.append((wl, cols, tab, lab, out))
    torch.cuda.synchronize()
    plan = sinet.BatchPlan(_bstreams(sinet, built))
    ref = [sinet.pipeline(tab, c["ts"], c["src"], c["dst"], c["bytes"], wl.window.t0,
                          wl.window.width, wl.window.n_bins)
           for wl, c, tab, lab, out in built]
    for rep in range(2):
        for _, _, _, lab, out in built:
            if lab is not None:
                lab.fill_(7)
            for t in out:
                t.fill_(-1)
        plan.run()
        torch.cuda.synchronize()
        for (wl, c, tab, lab, out), (l2, o2) in zip(built, ref):
            if lab is not None:
                assert torch.equal(lab, l2), (rep, wl.name)
            for x, y in zip(out, o2):
                assert torch.equal(x, y), (rep, wl.name)
    for wl, c, tab, lab, out in built[:3]:
        s = sinetgen.sessions(wl)
        w = wl.window
        elab, ec, eb, ed = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"],
                                           w.t0, w.width, w.n_bins)
        if lab is not None:
            assert np.array_equal(lab.cpu().numpy(), elab), wl.name
        _cmp_hist(sinet, out, (ec, eb, ed))


def test_autotune_candidates_identical(sinet, torch, tmp_path):
    built = _batch_setup(sinet, torch, n_streams=6, total=600_000)
    bs = _bstreams(sinet, built)
    cache = str(tmp_path / "tune.json")
    t = sinet.autotune(bs, cache_path=cache)
    assert t.chunk >= 2048 and t.block in (512, 1024)
    t2 = sinet.autotune(bs, cache_path=cache)   # from the cache
    assert (t2.chunk, t2.grid) == (t.chunk, t.grid)
    outs = []
    for chunk, grid in ((4096, 0), (65536, 0), (16384, 64), (t.chunk, t.grid)):
        tune = sinet.Tune(1024, chunk, grid, 0)
        plan = sinet.BatchPlan(bs, tune=tune)
        plan.run()
        torch.cuda.synchronize()
        outs.append([(lab.clone(), [o.clone() for o in out]) for _, _, _, lab, out in built])
        plan.close()
    for o in outs[1:]:
        for (l1, h1), (l2, h2) in zip(outs[0], o):
            assert torch.equal(l1, l2)
            for x, y in zip(h1, h2):
                assert torch.equal(x, y)
