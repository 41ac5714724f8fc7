"""sinet_pipeline_noalloc (the pipeline with the library's static device
workspace) against sinet_pipeline, through the C ABI: bit-identical labels
and histograms on two calls in a row, the second with a smaller input (the
array keeps the first call's contents), with and without stored labels, with
accumulation, and at the 2^25-session limit; more sessions are refused."""
import sys

import numpy as np
import pytest

import sinetgen

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2106_12863_amd as sinet
    return sinet, torch


def _cols(sinet, wl, start, stop):
    s = sinetgen.sessions(wl, start=start, stop=stop)
    return (sinet.to_device_u32(s["ts"]), sinet.to_device_u32(s["src"]),
            sinet.to_device_u32(s["dst"]), sinet.to_device_u64(s["bytes"]))


def _same(torch, a, b):
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_noalloc_equals_pipeline_two_calls(env):
    sinet, torch = env
    wl = sinetgen.config(2, n=30_000_000)
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    w = wl.window
    for n, lab_on in ((12_000_003, True), (5_000_001, False)):
        _say("noalloc", n, lab_on)
        ts, src, dst, nb = _cols(sinet, wl, 1_000_000, 1_000_000 + n)
        lab_ref, ref = sinet.pipeline(tab, ts, src, dst, nb, w.t0, w.width, w.n_bins)
        lab = torch.empty(n, dtype=torch.uint8, device="cuda") if lab_on else None
        out = sinet.new_hist(w.n_bins)
        sinet.pipeline_noalloc(tab, ts, src, dst, nb, w.t0, w.width, w.n_bins, lab, out)
        torch.cuda.synchronize()
        if lab_on:
            assert torch.equal(lab, lab_ref)
        _same(torch, out, ref)
        del out, ref


def test_noalloc_accumulate_and_small_window(env):
    """Two halves accumulated equal the whole; a 2,000-bin window (the
    private pass) and a one-minute table (config 1)."""
    sinet, torch = env
    wl = sinetgen.config(1, n=3_000_017)
    tab = sinet.Table(wl.pbase, wl.plen, kind="scan")
    ts, src, dst, nb = _cols(sinet, wl, 0, wl.n)
    for t0, width, n_bins in ((0, 1, 60_000), (500, 30, 2_000)):
        _say("noalloc acc", n_bins)
        lab_ref, ref = sinet.pipeline(tab, ts, src, dst, nb, t0, width, n_bins)
        lab = torch.empty(wl.n, dtype=torch.uint8, device="cuda")
        out = sinet.new_hist(n_bins)
        h = 1_234_567
        sinet.pipeline_noalloc(tab, ts[:h], src[:h], dst[:h], nb[:h], t0, width, n_bins, lab[:h], out)
        sinet.pipeline_noalloc(tab, ts[h:], src[h:], dst[h:], nb[h:], t0, width, n_bins, lab[h:], out,
                               accumulate=True)
        torch.cuda.synchronize()
        assert torch.equal(lab, lab_ref)
        _same(torch, out, ref)


def test_noalloc_limit(env):
    """Exactly 2^25 sessions run (the day's shape, no labels stored);
    one more is refused before anything is enqueued."""
    sinet, torch = env
    n = 1 << 25
    wl = sinetgen.config(5, n=n * 48)
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    w = wl.window
    import sinetgen.gpu as gg
    cols = {c: torch.empty(n + 1, dtype=torch.int64 if c == "bytes" else torch.int32, device="cuda")
            for c in ("ts", "src", "dst", "bytes")}
    gg.fill(wl, cols["ts"], cols["src"], cols["dst"], cols["bytes"], i0=20 * n, n=n + 1)
    ts, src, dst, nb = (cols[c][:n] for c in ("ts", "src", "dst", "bytes"))
    _say("noalloc limit")
    _, ref = sinet.pipeline(tab, ts, src, dst, nb, w.t0, w.width, w.n_bins, label=False)
    out = sinet.new_hist(w.n_bins)
    sinet.pipeline_noalloc(tab, ts, src, dst, nb, w.t0, w.width, w.n_bins, None, out)
    torch.cuda.synchronize()
    _same(torch, out, ref)
    del ref
    with pytest.raises(sinet.SinetError):
        sinet.pipeline_noalloc(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"], w.t0, w.width,
                               w.n_bins, None, out)
