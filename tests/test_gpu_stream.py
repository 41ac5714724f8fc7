"""GPU parity of the out-of-core pipeline: host-resident columns streamed in
chunks through the device give the same labels and histogram as one
pipeline call over the same sessions resident on the device, and as the CPU
oracle."""
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


def _resident(sinet, tab, s, t0, w, nb):
    cols = (sinet.to_device_u32(s["ts"]), sinet.to_device_u32(s["src"]),
            sinet.to_device_u32(s["dst"]), sinet.to_device_u64(s["bytes"]))
    return sinet.pipeline(tab, *cols, t0, w, nb)


@pytest.mark.parametrize("pinned", [False, True])
def test_streamed_equals_resident_and_oracle(sinet, torch, pinned):
    wl = sinetgen.config(2, n=3_000_017)
    _say("streamed", pinned)
    s = sinetgen.sessions(wl)
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    t0, w, nb = 2_000_000, 7, 3_000_000
    lab_r, hist_r = _resident(sinet, tab, s, t0, w, nb)
    cols = [s["ts"], s["src"], s["dst"], s["bytes"]]
    if pinned:
        pin = []
        for a in cols:
            t = torch.empty(a.shape[0], dtype=torch.int64 if a.itemsize == 8 else torch.int32,
                            pin_memory=True)
            t.copy_(torch.from_numpy(a.view(np.int64 if a.itemsize == 8 else np.int32)))
            pin.append(t)
        cols = pin
    st = sinet.Streamer(chunk=1_000_003)       # three chunks, the last one ragged
    lab, hist = st.pipeline(tab, *cols, t0, w, nb)
    torch.cuda.synchronize()
    assert np.array_equal(lab, lab_r.cpu().numpy())
    for x, y in zip(hist, hist_r):
        assert torch.equal(x, y)
    elab, ec, eb, ed = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"],
                                       t0, w, nb)
    assert np.array_equal(lab, elab)
    assert np.array_equal(sinet.to_host_u64(hist[0]), ec)
    assert np.array_equal(sinet.to_host_u64(hist[1]), eb)
    assert np.array_equal(sinet.to_host_u64(hist[2]), ed)
    # the same streamer again: a smaller input, no labels, added onto the result
    lab2, hist2 = st.pipeline(tab, s["ts"][:12_345], s["src"][:12_345], s["dst"][:12_345],
                              s["bytes"][:12_345], t0, w, nb, label=None, out=hist,
                              accumulate=True)
    torch.cuda.synchronize()
    assert lab2 is None
    _, e2c, e2b, e2d = oracle.pipeline(wl.pbase, wl.plen, s["ts"][:12_345], s["src"][:12_345],
                                       s["dst"][:12_345], s["bytes"][:12_345], t0, w, nb)
    assert np.array_equal(sinet.to_host_u64(hist2[0]), ec + e2c)
    assert np.array_equal(sinet.to_host_u64(hist2[2]), ed + e2d)
    st.close()


def test_streamer_small_chunks_and_edges(sinet, torch):
    """Chunks of 4,099 sessions (not a multiple of the device chunk), a day
    window with many bins, empty input and bad arguments."""
    wl = sinetgen.config(1, n=50_021)
    s = sinetgen.sessions(wl)
    tab = sinet.Table(wl.pbase, wl.plen)
    t0, w, nb = 0, 1, 60_000
    lab_r, hist_r = _resident(sinet, tab, s, t0, w, nb)
    st = sinet.Streamer(chunk=4_099)
    lab, hist = st.pipeline(tab, s["ts"], s["src"], s["dst"], s["bytes"], t0, w, nb)
    torch.cuda.synchronize()
    assert np.array_equal(lab, lab_r.cpu().numpy())
    for x, y in zip(hist, hist_r):
        assert torch.equal(x, y)
    e32, e64 = np.zeros(0, np.uint32), np.zeros(0, np.uint64)
    for t in hist:
        t.fill_(3)
    st.pipeline(tab, e32, e32, e32, e64, t0, w, nb, out=hist)
    torch.cuda.synchronize()
    assert all(bool((t == 0).all()) for t in hist)
    with pytest.raises(sinet.SinetError):
        sinet.Streamer(chunk=0)
    with pytest.raises(ValueError):
        st.pipeline(tab, s["ts"], s["src"][:10], s["dst"], s["bytes"], t0, w, nb)
    st.close()


@pytest.mark.parametrize("kind", ["trie", "pla"])
def test_streamed_with_separate_lookup_pass(sinet, torch, kind):
    """Tables whose lookups run as their own pass (trie, learned) stream the
    same way: equal to the resident call, with and without host labels."""
    wl = sinetgen.config(4, n=1_000_003)
    s = sinetgen.sessions(wl)
    tab = sinet.Table(wl.pbase, wl.plen, kind=kind, inout_index=False)
    if kind == "pla":
        tab.train()
    w = wl.window
    lab_r, hist_r = _resident(sinet, tab, s, w.t0, w.width, w.n_bins)
    st = sinet.Streamer(chunk=300_007)
    for label in (True, None):
        lab, hist = st.pipeline(tab, s["ts"], s["src"], s["dst"], s["bytes"], w.t0, w.width, w.n_bins,
                                label=label)
        torch.cuda.synchronize()
        if label is True:
            assert np.array_equal(lab, lab_r.cpu().numpy())
        for x, y in zip(hist, hist_r):
            assert torch.equal(x, y)
    st.close()


def test_streamed_full_day_equals_resident(sinet, torch):
    """The out-of-core benchmark's day and launch: the full synthetic day
    (1.6e9 sessions) generated in HBM, held in pinned host memory and streamed
    in 64 Mi-session chunks with labels into pinned memory; labels and
    histogram equal one resident pipeline call over the same day."""
    from sinetgen import gpu as gg
    wl = sinetgen.config(5)
    w = wl.window
    _say("streamed full day", wl.n)
    dcols = gg.alloc_and_fill(wl)
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    lab_r, hist_r = sinet.pipeline(tab, dcols["ts"], dcols["src"], dcols["dst"], dcols["bytes"],
                                   w.t0, w.width, w.n_bins)
    pin = {}
    for c, t in dcols.items():
        pin[c] = torch.empty(wl.n, dtype=t.dtype, pin_memory=True)
        pin[c].copy_(t)
    torch.cuda.synchronize()
    del dcols
    lab = torch.empty(wl.n, dtype=torch.uint8, pin_memory=True)
    st = sinet.Streamer(chunk=64 << 20)
    _, hist = st.pipeline(tab, pin["ts"], pin["src"], pin["dst"], pin["bytes"], w.t0, w.width,
                          w.n_bins, label=lab)
    torch.cuda.synchronize()
    st.close()
    assert torch.equal(lab.to("cuda"), lab_r)
    for x, y in zip(hist, hist_r):
        assert torch.equal(x, y)
