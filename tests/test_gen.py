"""Host generator: determinism, index-addressability and workload shape."""
import numpy as np

import sinetgen as g


def test_splitmix64_reference_values():
    # SplitMix64 seeded with 0 (Steele, Lea and Flood, 2014): its published
    # first outputs, as given with the reference implementation by Vigna.
    st = 0
    outs = []
    for _ in range(3):
        st = (st + g.GOLDEN) & g.M64
        outs.append(g.mix64_int(st))
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert g.draw(0, np.arange(3)).tolist() == outs


def test_sessions_are_index_addressable():
    wl = g.config(2, n=1_000_000)
    full = g.sessions(wl, start=0, stop=20_000)
    idx = np.array([0, 1, 19_999, 5_000, 123])
    part = g.sessions(wl, idx=idx)
    for k in full:
        assert np.array_equal(full[k][idx], part[k])


def test_diurnal_shape_and_near_sortedness():
    wl = g.config(2, n=2_000_000)
    s = g.sessions(wl, idx=np.arange(0, wl.n, 7))
    ts = s["ts"].astype(np.int64)
    assert ts.min() >= 0 and ts.max() < g.DAY_MS
    # nearly sorted: a later index is never more than 2 J earlier in time
    run_min = np.minimum.accumulate(ts[::-1])[::-1]
    assert np.all(ts - run_min <= 2 * 5000 + 1)
    h, _ = np.histogram(ts, bins=24, range=(0, g.DAY_MS))
    assert 2.4 < h.max() / h.min() < 3.6   # peak/trough 3 (hourly bins blur it)


def test_bytes_lognormal_shape():
    wl = g.config(1, n=400_000)
    b = g.sessions(wl)["bytes"].astype(np.float64)
    lb = np.log(np.maximum(b, 1))
    assert abs(np.median(lb) - 8.0) < 0.05
    assert abs(np.std(lb) - 2.0) < 0.1


def test_tables():
    w1 = g.config(1)
    assert w1.n_prefix == 64 and w1.plen.min() >= 16 and w1.plen.max() <= 24
    w2 = g.config(2)
    assert w2.n_prefix == 1024 and w2.plen.min() >= 12 and w2.plen.max() <= 28
    w4 = g.config(4)
    assert w4.n_prefix == 200_000 and w4.plen.min() >= 8 and w4.plen.max() <= 32
    assert g.coverage(w4.pbase, w4.plen) < 0.5
    st = g.batch_streams()
    assert len(st) == 64 and abs(sum(s.n for s in st) - 3e8) < 1e6
    assert sum(s.hist_bytes() for s in st) <= 32 << 30
    assert all(64 <= s.n_prefix <= 4096 for s in st)
