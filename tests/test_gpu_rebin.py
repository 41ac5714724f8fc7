"""GPU parity of the coarser time frames (sinet_rebin) against the CPU
oracle: random 64-bit bins (sums wrap modulo 2^64), small and large factors,
ragged last frames, and the full day's millisecond histogram in hours."""
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


@pytest.mark.parametrize("rows,n_bins", [(4, 100_003), (2354, 144), (1, 8_192 * 3 + 5)])
def test_rebin_random_bins(sinet, torch, rows, n_bins):
    rng = np.random.default_rng(rows + n_bins)
    a = rng.integers(-(1 << 63), 1 << 63, (rows, n_bins), dtype=np.int64)
    d = torch.from_numpy(a).cuda()
    for f in (1, 2, 7, 32, 33, 100, 1_000, 8_191, 8_192, 8_193, 50_000, n_bins, n_bins + 9):
        _say("rebin", rows, n_bins, f)
        got = sinet.rebin(d, f)
        torch.cuda.synchronize()
        exp = oracle.rebin(a.view(np.uint64), f)
        assert np.array_equal(got.cpu().numpy().view(np.uint64), exp), f


def test_rebin_full_day_to_hours(sinet, torch):
    """The 1.6e9-session day's 86.4 M millisecond bins as 24 one-hour frames:
    equal to the oracle's frames of the same bins and, per label, to the
    sessions counted in the window."""
    import sinetgen.gpu as gg
    wl = sinetgen.config(5)
    cols = gg.alloc_and_fill(wl)
    w = wl.window
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    lab, (c, b, d) = sinet.pipeline(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"],
                                    w.t0, w.width, w.n_bins)
    del cols
    hc = sinet.rebin(c, 3_600_000)
    hb = sinet.rebin(b, 3_600_000)
    torch.cuda.synchronize()
    assert tuple(hc.shape) == (4, 24)
    ec = oracle.rebin(sinet.to_host_u64(c), 3_600_000)
    eb = oracle.rebin(sinet.to_host_u64(b), 3_600_000)
    assert np.array_equal(sinet.to_host_u64(hc), ec)
    assert np.array_equal(sinet.to_host_u64(hb), eb)
    per_label = torch.bincount(lab.long(), minlength=4)
    assert torch.equal(hc.sum(dim=1) + d[:, 0], per_label)
