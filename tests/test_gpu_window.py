"""GPU parity of the sliding-window reduce (the histogram pass that keeps the
bins a piece of nearly time-sorted sessions touches in LDS), through the C
ABI against the CPU oracle, bit for bit.

Every test forces the window reduce, also at sizes where the default picks
the records reduce, and covers what the pass must get right on any input:
pieces with one or a few steps, bins that spill across piece boundaries,
sessions late for the window (shuffled time order), byte counts of every
magnitude (the far path from 2^22, carries of the 27-bit byte field), more
than 32 sessions in one bin (wraps of the 5-bit count field), windows that
drop and divide, accumulation, given labels, and unaligned slices.
"""
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
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a ROCm device"
    return t


@pytest.fixture(scope="module")
def sinet(torch):
    import paper_2106_12863_amd as s
    s.set_reduce("window")
    yield s
    s.set_reduce("auto")


def _up(sinet, s):
    return (sinet.to_device_u32(s["ts"]), sinet.to_device_u32(s["src"]),
            sinet.to_device_u32(s["dst"]), sinet.to_device_u64(s["bytes"]))


def _cmp(sinet, lab, out, exp, what=""):
    elab, ec, eb, ed = exp
    if lab is not None:
        assert np.array_equal(lab.cpu().numpy(), elab), f"labels differ {what}"
    c, b, d = out
    assert np.array_equal(sinet.to_host_u64(c), ec), f"count bins differ {what}"
    assert np.array_equal(sinet.to_host_u64(b), eb), f"byte bins differ {what}"
    assert np.array_equal(sinet.to_host_u64(d), ed), f"dropped differ {what}"


def _run(sinet, torch, wl, s, kind="bsearch", inout=True, t0=None, width=None, n_bins=None):
    w = wl.window
    t0 = w.t0 if t0 is None else t0
    width = w.width if width is None else width
    n_bins = w.n_bins if n_bins is None else n_bins
    ts, src, dst, nb = _up(sinet, s)
    tab = sinet.Table(wl.pbase, wl.plen, kind=kind, inout_index=inout)
    if kind in ("pla", "mlp"):
        tab.train()
    lab, out = sinet.pipeline(tab, ts, src, dst, nb, t0, width, n_bins)
    torch.cuda.synchronize()
    exp = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"], t0, width,
                          n_bins)
    return lab, out, exp


def test_day_shape_all_bins(sinet, torch):
    """Config-2 table and time shape (diurnal, +-5 s jitter), 3e6 sessions,
    every one of the 4 x 86.4 M bins, in/out index and two search kinds."""
    wl = sinetgen.config(2, n=3_000_000)
    s = sinetgen.sessions(wl)
    for kind, inout in (("bsearch", True), ("trie", False)):
        _say("window day", kind, inout)
        lab, out, exp = _run(sinet, torch, wl, s, kind, inout)
        _cmp(sinet, lab, out, exp, kind)
        del out


def test_full_day_rate_slice(sinet, torch):
    """Sessions at the 1.6e9-per-day rate (about 18.5 per ms on average), a
    2-minute slice at the diurnal trough and one at the peak, all bins."""
    wl = sinetgen.config(5)
    for t_lo in (0, 43_200_000 - 60_000):
        lo, hi = sinetgen.index_range_for_time(wl, t_lo, t_lo + 120_000)
        _say("window full-day rate", t_lo, hi - lo)
        s = sinetgen.sessions(wl, start=lo, stop=hi)
        w = wl.window
        lab, out, exp = _run(sinet, torch, wl, s, "bsearch", True)
        _cmp(sinet, lab, out, exp, str(t_lo))
        del out


@pytest.mark.parametrize("n", [1, 2, 1023, 1024, 1025, 4097, 65_537, 262_143, 1_000_003])
def test_ragged_sizes_and_few_pieces(sinet, torch, n):
    """From one session to a million: pieces of one step, a partial last step,
    fewer steps than workgroups."""
    wl = sinetgen.config(2, n=max(n, 2))
    s = sinetgen.sessions(wl, start=0, stop=n)
    _say("window ragged", n)
    lab, out, exp = _run(sinet, torch, wl, s, width=100, n_bins=864_000)
    _cmp(sinet, lab, out, exp, str(n))


def test_tiny_config_unsorted_minute(sinet, torch):
    """Config 1: timestamps uniform over one minute in random order, so most
    sessions fall outside their piece's window and take the far path."""
    wl = sinetgen.config(1)
    s = sinetgen.sessions(wl)
    _say("window tiny", wl.n)
    for kind in ("scan", "bsearch"):
        lab, out, exp = _run(sinet, torch, wl, s, kind, kind == "bsearch")
        _cmp(sinet, lab, out, exp, kind)


def test_shuffled_day_is_exact(sinet, torch):
    """The day shape in random order: nearly every session is late or outside
    its piece's reach."""
    wl = sinetgen.config(2, n=2_000_000)
    s = sinetgen.sessions(wl)
    perm = np.random.default_rng(3).permutation(wl.n)
    s = {k: v[perm] for k, v in s.items()}
    _say("window shuffled")
    lab, out, exp = _run(sinet, torch, wl, s)
    _cmp(sinet, lab, out, exp)


@pytest.mark.parametrize("t0,width,n_bins", [(1000, 1, 50_000), (777, 7, 5_000),
                                              (0, 1000, 86_400), (3_600_000, 1, 7_200_000),
                                              (0, 10, 8_640_000), (86_000_000, 1, 2_049)])
def test_windows_drop_and_divide(sinet, torch, t0, width, n_bins):
    wl = sinetgen.config(2, n=1_500_001)
    s = sinetgen.sessions(wl)
    _say("window drop/divide", t0, width, n_bins)
    lab, out, exp = _run(sinet, torch, wl, s, t0=t0, width=width, n_bins=n_bins)
    _cmp(sinet, lab, out, exp)


def test_byte_magnitudes(sinet, torch):
    """Byte counts 2^k + noise for every k < 64 (the far path from 2^22 on,
    sums wrapping modulo 2^64), on the day's time shape."""
    wl = sinetgen.config(2, n=700_001)
    s = sinetgen.sessions(wl)
    rng = np.random.default_rng(8)
    k = rng.integers(0, 64, wl.n).astype(np.uint64)
    s["bytes"] = (np.uint64(1) << k) + rng.integers(0, 1 << 16, wl.n).astype(np.uint64)
    _say("window byte magnitudes")
    lab, out, exp = _run(sinet, torch, wl, s)
    _cmp(sinet, lab, out, exp)


@pytest.mark.parametrize("shape", ["one_bin", "40_sorted_bins", "3_random_bins"])
def test_crowded_bins_wrap_and_carry(sinet, torch, shape):
    """600,000 sessions in a few bins with byte counts just under 2^22: the
    5-bit count field wraps every 32 sessions and the 27-bit byte field
    carries; the recorded events must restore both exactly."""
    rng = np.random.default_rng(len(shape))
    n = 600_000
    wl = sinetgen.config(1, n=n)
    s = sinetgen.sessions(wl)
    if shape == "one_bin":
        s["ts"] = np.full(n, 5_000, np.uint32)
    elif shape == "40_sorted_bins":
        s["ts"] = (5_000 + (np.arange(n) * 40) // n + rng.integers(0, 2, n)).astype(np.uint32)
    else:
        s["ts"] = (5_000 + rng.integers(0, 3, n)).astype(np.uint32)
    s["bytes"] = ((1 << 22) - 1 - rng.integers(0, 64, n)).astype(np.uint64)
    _say("window crowded", shape)
    lab, out, exp = _run(sinet, torch, wl, s, t0=0, width=1, n_bins=10_000_000)
    _cmp(sinet, lab, out, exp, shape)


def test_histogram_entry_accumulate_and_slices(sinet, torch):
    """sinet_histogram with given labels: whole, as accumulated pieces with
    cuts at unaligned session offsets, and onto earlier contents."""
    wl = sinetgen.config(2, n=1_200_007)
    s = sinetgen.sessions(wl)
    lab = oracle.classify(wl.pbase, wl.plen, s["src"], s["dst"], want_inst=False)
    ts, _, _, nb = _up(sinet, s)
    lt = torch.from_numpy(lab).cuda()
    t0, w, n_bins = 100, 1, 86_400_000
    out = sinet.histogram(ts, nb, lt, t0, w, n_bins)
    torch.cuda.synchronize()
    exp = oracle.histogram(s["ts"], s["bytes"], lab, t0, w, n_bins)
    _cmp(sinet, None, out, (None,) + tuple(exp))
    del out
    acc = sinet.new_hist(n_bins)
    cuts = [0, 1, 5, 4099, 500_001, 500_002, 1_100_000, wl.n]
    for a, b in zip(cuts[:-1], cuts[1:]):
        sinet.histogram(ts[a:b], nb[a:b], lt[a:b], t0, w, n_bins, out=acc, accumulate=a > 0)
    torch.cuda.synchronize()
    _cmp(sinet, None, acc, (None,) + tuple(exp), "pieces")
    base_c = torch.arange(4 * n_bins, dtype=torch.int64, device="cuda").view(4, n_bins) % 1000
    acc[0].copy_(base_c)
    acc[1].copy_(base_c * 7 + 1)
    acc[2].zero_()
    sinet.histogram(ts, nb, lt, t0, w, n_bins, out=acc, accumulate=True)
    torch.cuda.synchronize()
    ec, eb, ed = exp
    hc = sinet.to_host_u64(base_c)
    _cmp(sinet, None, acc, (None, ec + hc, eb + hc * np.uint64(7) + np.uint64(1), ed), "onto")


def test_pipeline_unaligned_slices(sinet, torch):
    """Columns that start 1, 2 or 3 sessions past 16-byte alignment."""
    wl = sinetgen.config(2, n=900_003)
    s = sinetgen.sessions(wl)
    ts, src, dst, nb = _up(sinet, s)
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    w = wl.window
    for h in (1, 2, 3):
        _say("window unaligned", h)
        lab, out = sinet.pipeline(tab, ts[h:], src[h:], dst[h:], nb[h:], w.t0, w.width, w.n_bins)
        torch.cuda.synchronize()
        exp = oracle.pipeline(wl.pbase, wl.plen, s["ts"][h:], s["src"][h:], s["dst"][h:],
                              s["bytes"][h:], w.t0, w.width, w.n_bins)
        _cmp(sinet, lab, out, exp, str(h))
        del out


def test_window_equals_records(sinet, torch):
    """The two reduces give identical histograms on the same day."""
    wl = sinetgen.config(2, n=4_000_000)
    s = sinetgen.sessions(wl)
    ts, src, dst, nb = _up(sinet, s)
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    w = wl.window
    _say("window vs records")
    lab_w, out_w = sinet.pipeline(tab, ts, src, dst, nb, w.t0, w.width, w.n_bins)
    sinet.set_reduce("records")
    try:
        lab_r, out_r = sinet.pipeline(tab, ts, src, dst, nb, w.t0, w.width, w.n_bins)
    finally:
        sinet.set_reduce("window")
    torch.cuda.synchronize()
    assert torch.equal(lab_w, lab_r)
    for x, y in zip(out_w, out_r):
        assert torch.equal(x, y)
