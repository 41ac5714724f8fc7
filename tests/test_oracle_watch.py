"""Pins of the oracle's watch-list histograms (sections "AbuseIPDB" and
"GRIZZLY STEPPE"): hand-worked cases, the special case that reduces to the
pinned main histogram, a brute force with the standard library's ipaddress,
and the invariants of the definition (per-list = sum of its hosts, order and
chunking do not matter)."""
import ipaddress
import os
from collections import defaultdict

import numpy as np
import pytest

import oracle
import sinetgen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "watch_examples.txt")


def _ip(s):
    return int(ipaddress.IPv4Address(s))


def _load_golden():
    rows, sess, hist, drop, win = [], [], [], [], None
    with open(GOLDEN) as f:
        for line in f:
            t = line.split("#", 1)[0].split()
            if not t:
                continue
            if t[0] == "wrow":
                a, z = t[1].split("/")
                rows.append((_ip(a), int(z), int(t[2])))
            elif t[0] == "wwin":
                win = tuple(int(x) for x in t[1:5])
            elif t[0] == "wsess":
                sess.append((int(t[1]), _ip(t[2]), _ip(t[3]), int(t[4])))
            elif t[0] == "whist":
                hist.append(tuple(int(x) for x in t[1:6]))
            elif t[0] == "wdrop":
                drop.append(tuple(int(x) for x in t[1:4]))
            else:
                raise ValueError(line)
    return rows, win, sess, hist, drop


@pytest.mark.parametrize("mode", ["scan", "hash"])
def test_watch_hand_examples(mode):
    rows, (t0, width, n_bins, n_keys), sess, hist, drop = _load_golden()
    base = np.array([r[0] for r in rows], np.uint32)
    plen = np.array([r[1] for r in rows], np.uint8)
    keys = np.array([r[2] for r in rows], np.uint32)
    ts, src, dst, nb = (np.array([s[k] for s in sess], dt) for k, dt in
                        ((0, np.uint32), (1, np.uint32), (2, np.uint32), (3, np.uint64)))
    c, b, d = oracle.watch(base, plen, ts, src, dst, nb, t0, width, n_bins, n_keys, inst=keys,
                           mode=mode)
    ec = np.zeros((2, n_keys, n_bins), np.uint64)
    eb = np.zeros((2, n_keys, n_bins), np.uint64)
    for dr, k, bn, cnt, by in hist:
        ec[dr, k, bn] = cnt
        eb[dr, k, bn] = by
    ed = np.zeros((2, 2), np.uint64)
    for dr, cnt, by in drop:
        ed[dr] = (cnt, by)
    assert np.array_equal(c, ec)
    assert np.array_equal(b, eb)
    assert np.array_equal(d, ed)


def test_watch_with_the_backbone_table_and_one_key_is_the_label_histogram():
    """List = the backbone table, every row key 0: direction 0 counts the
    sessions whose source is in the table (labels 1 and 3), direction 1 those
    whose destination is (labels 2 and 3), bin for bin."""
    wl = sinetgen.config(2, n=200_003)
    s = sinetgen.sessions(wl)
    t0, w, n_bins = 3_000_000, 60_000, 1_300
    lab, c4, b4, d4 = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"],
                                      t0, w, n_bins)
    keys = np.zeros(wl.n_prefix, np.uint32)
    c, b, d = oracle.watch(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"], t0, w,
                           n_bins, 1, inst=keys)
    assert np.array_equal(c[0, 0], c4[1] + c4[3]) and np.array_equal(b[0, 0], b4[1] + b4[3])
    assert np.array_equal(c[1, 0], c4[2] + c4[3]) and np.array_equal(b[1, 0], b4[2] + b4[3])
    assert np.array_equal(d[0], d4[1] + d4[3]) and np.array_equal(d[1], d4[2] + d4[3])
    assert c[0, 0].sum() > 0 and c[1, 0].sum() > 0


def _watch_case(n=150_001, seed=5):
    wl = sinetgen.config(1, n=n, seed=seed)
    wlist = sinetgen.watch_lists(seed=seed, sizes=(30, 70), frac=0.05)
    s = sinetgen.sessions(wl, watch=wlist)
    return wl, wlist, s


def test_watch_equals_institution_lookup_then_bincount():
    """Per-host keys: the same counts follow from the pinned institution
    lookup (classify) and numpy's unbuffered add."""
    wl, wlist, s = _watch_case()
    keys = np.arange(wlist.n, dtype=np.uint32)
    plen = np.full(wlist.n, 32, np.uint8)
    t0, w, n_bins = 5_000, 1_000, 50
    c, b, d = oracle.watch(wlist.addrs, plen, s["ts"], s["src"], s["dst"], s["bytes"], t0, w,
                           n_bins, wlist.n, inst=keys)
    _, si, di = oracle.classify(wlist.addrs, plen, s["src"], s["dst"], inst=keys)
    ts = s["ts"].astype(np.int64)
    inw = (ts >= t0) & ((ts - t0) // w < n_bins)
    bn = (ts - t0) // w
    for dr, k in ((0, si), (1, di)):
        hit = k != oracle.NO_INST
        ec = np.zeros((wlist.n, n_bins), np.uint64)
        eb = np.zeros((wlist.n, n_bins), np.uint64)
        m = hit & inw
        np.add.at(ec, (k[m].astype(np.int64), bn[m]), np.uint64(1))
        np.add.at(eb, (k[m].astype(np.int64), bn[m]), s["bytes"][m])
        assert np.array_equal(c[dr], ec) and np.array_equal(b[dr], eb)
        mo = hit & ~inw
        assert int(d[dr, 0]) == int(mo.sum())
        assert int(d[dr, 1]) == int(s["bytes"][mo].sum(dtype=np.uint64))
    assert c.sum() > 1000


def test_watch_brute_force_with_ipaddress():
    """Nested /24-/32 list rows with duplicates, matched by ipaddress
    membership, longest network first, lowest row on ties."""
    rng = np.random.default_rng(11)
    nets = []
    for _ in range(12):
        a = int(rng.integers(0, 1 << 32))
        z = int(rng.choice([24, 28, 32]))
        nets.append((a & (0xFFFFFFFF << (32 - z)) & 0xFFFFFFFF, z))
    nets.append((nets[0][0] | 5, 32) if nets[0][1] < 32 else (nets[0][0], 32))  # nested / duplicate
    nets.append(nets[3])                                                        # exact duplicate
    base = np.array([a for a, _ in nets], np.uint32)
    plen = np.array([z for _, z in nets], np.uint8)
    keys = rng.integers(0, 5, len(nets)).astype(np.uint32)
    n = 3_000
    pick = lambda: np.array([int(nets[int(rng.integers(0, len(nets)))][0]) |
                             int(rng.integers(0, 1 << (32 - 24))) if rng.random() < 0.6 else
                             int(rng.integers(0, 1 << 32)) for _ in range(n)], np.uint64
                            ).astype(np.uint32)
    src, dst = pick(), pick()
    ts = rng.integers(0, 40, n).astype(np.uint32)
    nb = rng.integers(0, 1 << 40, n).astype(np.uint64)
    t0, w, n_bins, n_keys = 3, 7, 5, 5
    net_objs = [ipaddress.ip_network((int(a), z)) for a, z in nets]

    def key_of(a):
        best, bz = None, -1
        addr = ipaddress.ip_address(int(a))
        for r, nt in enumerate(net_objs):
            if addr in nt and nt.prefixlen > bz:
                best, bz = r, nt.prefixlen
        return None if best is None else int(keys[best])

    ec = defaultdict(lambda: [0, 0])
    ed = [[0, 0], [0, 0]]
    for i in range(n):
        for dr, a in ((0, src[i]), (1, dst[i])):
            k = key_of(a)
            if k is None:
                continue
            if ts[i] >= t0 and (int(ts[i]) - t0) // w < n_bins:
                cell = ec[(dr, k, (int(ts[i]) - t0) // w)]
            else:
                cell = ed[dr]
            cell[0] += 1
            cell[1] = (cell[1] + int(nb[i])) % (1 << 64)
    c, b, d = oracle.watch(base, plen, ts, src, dst, nb, t0, w, n_bins, n_keys, inst=keys)
    got = {(dr, k, bn): [int(c[dr, k, bn]), int(b[dr, k, bn])]
           for dr, k, bn in zip(*np.nonzero(c))}
    assert got == dict(ec)
    assert [[int(x) for x in row] for row in d] == ed
    assert len(got) > 10


def test_watch_per_list_is_the_sum_of_its_hosts():
    wl, wlist, s = _watch_case()
    plen = np.full(wlist.n, 32, np.uint8)
    t0, w, n_bins = 0, 600, 120
    ch, bh, dh = oracle.watch(wlist.addrs, plen, s["ts"], s["src"], s["dst"], s["bytes"], t0, w,
                              n_bins, wlist.n, inst=np.arange(wlist.n, dtype=np.uint32))
    cl, bl, dl = oracle.watch(wlist.addrs, plen, s["ts"], s["src"], s["dst"], s["bytes"], t0, w,
                              n_bins, 2, inst=wlist.lists)
    for j in (0, 1):
        m = wlist.lists == j
        assert np.array_equal(cl[:, j], ch[:, m].sum(axis=1, dtype=np.uint64))
        assert np.array_equal(bl[:, j], bh[:, m].sum(axis=1, dtype=np.uint64))
    assert np.array_equal(dl, dh)


def test_watch_order_and_chunks_do_not_matter():
    wl, wlist, s = _watch_case(n=60_007)
    plen = np.full(wlist.n, 32, np.uint8)
    keys = np.arange(wlist.n, dtype=np.uint32)
    args = (1_000, 250, 200, wlist.n)
    whole = oracle.watch(wlist.addrs, plen, s["ts"], s["src"], s["dst"], s["bytes"], *args,
                         inst=keys)
    perm = np.random.default_rng(2).permutation(wl.n)
    shuf = oracle.watch(wlist.addrs, plen, s["ts"][perm], s["src"][perm], s["dst"][perm],
                        s["bytes"][perm], *args, inst=keys)
    out = None
    for a, b in ((0, 1), (1, 20_000), (20_000, wl.n)):
        part = oracle.watch(wlist.addrs, plen, s["ts"][a:b], s["src"][a:b], s["dst"][a:b],
                            s["bytes"][a:b], *args, inst=keys, out=out)
        out = part
    for x, y, z in zip(whole, shuf, out):
        assert np.array_equal(x, y) and np.array_equal(x, z)


def test_watch_rejects_keys_outside_n_keys():
    with pytest.raises(ValueError):
        oracle.watch(np.array([1], np.uint32), np.array([32], np.uint8), np.zeros(1, np.uint32),
                     np.zeros(1, np.uint32), np.zeros(1, np.uint32), np.zeros(1, np.uint64),
                     0, 1, 1, 1, inst=np.array([1], np.uint32))


def test_watch_overlay_rate_and_skew():
    """The generator's overlay: about frac of the sources (and of the
    destinations) become listed hosts, the first hosts most often."""
    wl = sinetgen.config(2, n=400_000)
    wlist = sinetgen.watch_lists(frac=0.01)
    s0 = sinetgen.sessions(wl)
    s = sinetgen.sessions(wl, watch=wlist)
    pos = {int(a): i for i, a in enumerate(wlist.addrs)}
    for col in ("src", "dst"):
        hit = np.isin(s[col], wlist.addrs) & (s[col] != s0[col])
        assert abs(hit.mean() - 0.01) < 0.001
        idx = np.array([pos[int(a)] for a in s[col][hit]])
        # floor(K u^2): P(index < K/4) = P(u < 1/2) = 1/2
        assert abs((idx < wlist.n / 4).mean() - 0.5) < 0.03
    assert np.array_equal(s["ts"], s0["ts"]) and np.array_equal(s["bytes"], s0["bytes"])


# ------------------------------------------------------------ coarser frames
def test_rebin_equals_the_histogram_at_the_coarser_width():
    """Figures 6-7 group the day into one-hour frames: summing every group of
    f bins of width w gives the histogram of width w * f (floor((t - t0) / w)
    // f == floor((t - t0) / (w * f))), with a short last frame holding only
    the sessions of the fine window."""
    wl = sinetgen.config(2, n=300_007)
    s = sinetgen.sessions(wl)
    lab = oracle.classify(wl.pbase, wl.plen, s["src"], s["dst"], want_inst=False)
    t0, w = 40_000, 3
    for n_bins, f in ((9_000, 1_000), (9_001, 1_000), (9_000, 7), (9_000, 1), (9_000, 9_000),
                      (9_000, 50_000)):
        fine_c, fine_b, _ = oracle.histogram(s["ts"], s["bytes"], lab, t0, w, n_bins)
        n_out = -(-n_bins // f)
        # the coarse histogram of exactly the sessions inside the fine window
        keep = s["ts"].astype(np.int64) < t0 + w * n_bins
        cc, cb, _ = oracle.histogram(s["ts"][keep], s["bytes"][keep], lab[keep], t0, w * f, n_out)
        assert np.array_equal(oracle.rebin(fine_c, f), cc), (n_bins, f)
        assert np.array_equal(oracle.rebin(fine_b, f), cb), (n_bins, f)


def test_rebin_special_cases_and_wraparound():
    rng = np.random.default_rng(4)
    a = rng.integers(0, 1 << 63, (3, 101), dtype=np.int64).astype(np.uint64) * np.uint64(3)
    assert np.array_equal(oracle.rebin(a, 1), a)
    total = oracle.rebin(a, 500)
    assert total.shape == (3, 1)
    for r in range(3):
        assert int(total[r, 0]) == sum(int(x) for x in a[r]) % (1 << 64)
    got = oracle.rebin(a, 10)
    for r in range(3):
        for k in range(11):
            assert int(got[r, k]) == sum(int(x) for x in a[r, 10 * k:10 * k + 10]) % (1 << 64)
