"""Label runs on the GPU (per-wave ballots and mbcnt ranks, class totals)
against the oracle's stable partition, through the C ABI: every index and
every total, bit for bit, over ragged sizes around the tile (4,096) and
workgroup-range (65,536) sizes and their multiples, unaligned label pointers, label bytes with
high bits set, single-label inputs and the labels of a full-size day."""
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


def _check(sinet, lab_host, lab_dev):
    idx, tot = sinet.label_runs(lab_dev)
    eidx, etot = oracle.label_runs(lab_host)
    assert np.array_equal(sinet.to_host_u64(tot), etot)
    assert np.array_equal(sinet.to_host_u32(idx), eidx)


@pytest.mark.parametrize("n", [1, 3, 15, 16, 17, 4095, 4096, 4097, 16_383, 16_384, 16_385,
                               65_535, 65_536, 65_537, 262_143, 262_144, 262_145, 1_000_003,
                               9_000_001])
def test_random_labels_ragged(sinet, n):
    import torch
    _say("runs n", n)
    rng = np.random.default_rng(n)
    lab = rng.integers(0, 256, n).astype(np.uint8)
    _check(sinet, lab, torch.from_numpy(lab).cuda())


def test_unaligned_and_single_label(sinet):
    import torch
    rng = np.random.default_rng(9)
    base = rng.integers(0, 4, 1_000_010).astype(np.uint8)
    dev = torch.from_numpy(base).cuda()
    for off in (1, 2, 3, 4, 8, 15):   # label pointers off 16-byte alignment
        _check(sinet, base[off:], dev[off:])
    for L in range(4):
        one = np.full(300_001, L, np.uint8)
        _check(sinet, one, torch.from_numpy(one).cuda())


def test_empty_zeroes_totals(sinet):
    import torch
    tot = torch.full((4,), 7, dtype=torch.int64, device="cuda")
    sinet.label_runs(torch.empty(0, dtype=torch.uint8, device="cuda"),
                     idx=torch.empty(0, dtype=torch.int32, device="cuda"), totals=tot)
    assert tot.cpu().tolist() == [0, 0, 0, 0]


def test_day_labels(sinet):
    """The labels of the 1e8-session day (1,024 prefixes) from the GPU's own
    discrimination, partitioned; the totals also equal the per-label sums of
    the day's histogram plus its dropped sessions."""
    import torch
    import sinetgen.gpu as gg
    wl = sinetgen.config(2)
    cols = gg.alloc_and_fill(wl, columns=("ts", "src", "dst", "bytes"))
    tab = sinet.Table(wl.pbase, wl.plen, kind="bsearch")
    w = wl.window
    lab, (c, b, d) = sinet.pipeline(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"],
                                    w.t0, w.width, w.n_bins)
    torch.cuda.synchronize()
    idx, tot = sinet.label_runs(lab)
    torch.cuda.synchronize()
    eidx, etot = oracle.label_runs(lab.cpu().numpy())
    assert np.array_equal(sinet.to_host_u64(tot), etot)
    assert np.array_equal(sinet.to_host_u32(idx), eidx)
    assert np.array_equal(sinet.to_host_u64(c.sum(dim=1) + d[:, 0]), etot)
