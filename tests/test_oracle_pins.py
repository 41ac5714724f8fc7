"""Pins of the CPU oracle against things other than itself: hand-worked
cases, Python's ipaddress module, brute force over small universes, numpy's
bincount / add.at, and the invariants the paper's map-reduce implies."""
import ipaddress

import numpy as np
import pytest

import oracle
from _golden import load

G, TABLES = load()


def _tab(name):
    b, z, inst = TABLES[name]
    return (np.array(b, np.uint32), np.array(z, np.uint8), np.array(inst, np.uint32))


# ---------------------------------------------------------------- hand cases
@pytest.mark.parametrize("z,expect", G["mask"])
def test_hand_mask(z, expect):
    assert oracle.bitmask(0xFFFFFFFF, z) == expect


@pytest.mark.parametrize("a,b,z,result,m", G["match"])
def test_hand_match(a, b, z, result, m):
    # result of Algorithm 1's subtraction, worked by hand
    assert (oracle.bitmask(a, z) - oracle.bitmask(b, z)) & 0xFFFFFFFF == result
    assert oracle.match(a, b, z) == bool(m)


@pytest.mark.parametrize("mode", ["scan", "hash"])
def test_hand_lpm(mode):
    for name, a, inst in G["lpm"]:
        b, z, ids = _tab(name)
        lab, si, di = oracle.classify(b, z, [a], [a], inst=ids, mode=mode)
        assert si[0] == (oracle.NO_INST if inst is None else inst), (name, a)
        assert lab[0] == (0 if inst is None else 3)


@pytest.mark.parametrize("mode", ["scan", "hash"])
def test_hand_labels(mode):
    for name, s, d, lab in G["label"]:
        b, z, ids = _tab(name)
        got = oracle.classify(b, z, [s], [d], inst=ids, mode=mode, want_inst=False)
        assert got[0] == lab, (name, s, d)


def test_hand_endpoints_and_positions():
    from oracle import learned
    for name, B, own in G["ends"]:
        b, z, _ = _tab(name)
        gb, go = oracle.endpoints(b, z)
        assert gb.tolist() == B
        assert go.tolist() == own
    for name, a, p in G["pos"]:
        b, z, _ = _tab(name)
        gb, _ = oracle.endpoints(b, z)
        assert learned.positions(gb, [a])[0] == p


def test_hand_bins():
    for ts, t0, w, nb, expect in G["bin"]:
        c, by, dr = oracle.histogram([ts], [1], [0], t0, w, nb)
        if expect is None:
            assert c.sum() == 0 and dr[0, 0] == 1
        else:
            assert c[0, expect] == 1 and dr.sum() == 0


def test_hand_histogram():
    ts, lab, byt = zip(*G["sess"])
    for t0, w, nb, l, b, cnt, bb in G["hist"]:
        c, by, dr = oracle.histogram(ts, byt, lab, t0, w, nb)
        assert c[l, b] == cnt and by[l, b] == bb
    exp_nz = {(l, b) for (_, _, _, l, b, _, _) in G["hist"]}
    assert {tuple(x) for x in np.argwhere(c)} == exp_nz
    for l, cnt, bb in G["drop"]:
        assert dr[l, 0] == cnt and dr[l, 1] == bb
    assert dr.sum() == sum(cnt + bb for _, cnt, bb in G["drop"])


# -------------------------------------------------------- ipaddress library
def test_match_vs_ipaddress():
    rng = np.random.default_rng(11)
    for _ in range(3000):
        z = int(rng.integers(0, 33))
        base = int(rng.integers(0, 1 << 32))
        net = ipaddress.ip_network((base, z), strict=False)
        if rng.random() < 0.5:
            a = int(net.network_address) + int(rng.integers(0, net.num_addresses))
        else:
            a = int(rng.integers(0, 1 << 32))
        assert oracle.match(a, base, z) == (ipaddress.ip_address(a) in net)


def test_lpm_vs_ipaddress():
    rng = np.random.default_rng(12)
    base = rng.integers(0, 1 << 32, 40, dtype=np.uint64).astype(np.uint32)
    plen = rng.integers(0, 33, 40).astype(np.uint8)
    base[5] = base[4]
    plen[5] = plen[4]                     # a duplicate
    nets = [ipaddress.ip_network((int(b), int(z)), strict=False) for b, z in zip(base, plen)]
    addrs = []
    for n in nets:
        addrs.append(int(n.network_address))
        addrs.append(int(n.broadcast_address))
    addrs += rng.integers(0, 1 << 32, 200).tolist()
    addrs = np.array(addrs, np.uint32)
    for mode in ("scan", "hash"):
        lab, si, _ = oracle.classify(base, plen, addrs, addrs, mode=mode)
        for a, s, l in zip(addrs.tolist(), si.tolist(), lab.tolist()):
            hits = [i for i, n in enumerate(nets) if ipaddress.ip_address(a) in n]
            if not hits:
                assert s == oracle.NO_INST and l == 0
            else:
                best = max(hits, key=lambda i: (nets[i].prefixlen, -i))
                assert s == best and l == 3


# ----------------------------------------------------------------- brute force
def _random_table(rng, n, lmin, lmax, universe=None):
    base = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    plen = rng.integers(lmin, lmax + 1, n).astype(np.uint8)
    if universe is not None:
        base = (np.uint32(universe) | (base & np.uint32(0xFFFF))).astype(np.uint32)
    # some nested and duplicated rows
    for i in range(n // 4):
        j = int(rng.integers(0, n))
        k = int(rng.integers(0, n))
        base[k] = base[j]
        plen[k] = min(32, int(plen[j]) + int(rng.integers(0, 4)))
    return base, plen


def test_scan_equals_hash_random_tables():
    rng = np.random.default_rng(13)
    for t in range(20):
        base, plen = _random_table(rng, int(rng.integers(1, 60)), 0 if t % 5 == 0 else 4, 32)
        a = rng.integers(0, 1 << 32, 3000, dtype=np.uint64).astype(np.uint32)
        a[:len(base)] = base
        r1 = oracle.classify(base, plen, a, a[::-1].copy(), mode="scan")
        r2 = oracle.classify(base, plen, a, a[::-1].copy(), mode="hash")
        for x, y in zip(r1, r2):
            assert np.array_equal(x, y)


def test_exhaustive_slash16_universe():
    """Every address of a /16, a table of prefixes inside it: the scan, the
    per-length hash and the interval search (sorted boundaries + owner) agree
    everywhere, and each /Z prefix covers exactly 2^(32-Z) addresses."""
    rng = np.random.default_rng(14)
    uni = 0xC6330000  # 198.51.0.0/16
    base, plen = _random_table(rng, 48, 16, 32, universe=uni)
    a = (np.uint32(uni) + np.arange(1 << 16, dtype=np.uint32)).astype(np.uint32)
    l1, s1, _ = oracle.classify(base, plen, a, a, mode="scan")
    l2, s2, _ = oracle.classify(base, plen, a, a, mode="hash")
    assert np.array_equal(l1, l2) and np.array_equal(s1, s2)
    from oracle import learned
    B, own = oracle.endpoints(base, plen)
    pos = learned.positions(B, a)
    via_int = np.where(own[pos] == 0, np.uint32(oracle.NO_INST), own[pos] - 1).astype(np.uint32)
    assert np.array_equal(via_int, s1)
    # closed form: a /Z prefix inside the universe covers exactly 2^(32-Z) of it
    for p in range(len(base)):
        lab = oracle.classify(base[p:p + 1], plen[p:p + 1], a, a, want_inst=False)
        assert int(np.count_nonzero(lab & 1)) == 1 << (32 - int(plen[p]))


# ------------------------------------------------------------- histogram pins
def test_histogram_vs_numpy():
    rng = np.random.default_rng(15)
    n, nb, t0, w = 200_000, 5000, 777, 7
    ts = rng.integers(0, t0 + nb * w + 3000, n).astype(np.uint32)
    lab = rng.integers(0, 4, n).astype(np.uint8)
    byt = rng.integers(0, 1 << 62, n, dtype=np.uint64)
    byt[:10] = np.uint64(0xFFFFFFFFFFFFFFFF)   # exercises wraparound mod 2^64
    c, by, dr = oracle.histogram(ts, byt, lab, t0, w, nb)
    ok = (ts >= t0) & ((ts.astype(np.int64) - t0) // w < nb)
    b = (ts.astype(np.int64) - t0) // w
    key = lab.astype(np.int64) * nb + b
    ec = np.bincount(key[ok], minlength=4 * nb).reshape(4, nb).astype(np.uint64)
    eb = np.zeros(4 * nb, np.uint64)
    np.add.at(eb, key[ok], byt[ok])
    assert np.array_equal(c, ec)
    assert np.array_equal(by, eb.reshape(4, nb))
    for l in range(4):
        sel = (~ok) & (lab == l)
        assert dr[l, 0] == sel.sum()
        assert dr[l, 1] == np.add.reduce(byt[sel], dtype=np.uint64)


def test_histogram_invariants_shuffle_chunk_accumulate():
    """Merge by addition is associative and commutative (section "Merge
    Scatter Pattern with CPU"): any order and any chunking give the same
    bins, and bins plus dropped equal the per-label totals."""
    import sinetgen
    wl = sinetgen.config(1, n=60_000)
    s = sinetgen.sessions(wl)
    win = wl.window
    lab = oracle.classify(wl.pbase, wl.plen, s["src"], s["dst"], want_inst=False)
    c, by, dr = oracle.histogram(s["ts"], s["bytes"], lab, 1000, 1, 50_000)
    for l in range(4):
        sel = lab == l
        assert int(c[l].sum()) + int(dr[l, 0]) == int(sel.sum())
        assert int(by[l].sum(dtype=np.uint64)) + int(dr[l, 1]) == int(
            np.add.reduce(s["bytes"][sel], dtype=np.uint64))
    assert int(c.sum() + dr[:, 0].sum()) == wl.n
    perm = np.random.default_rng(1).permutation(wl.n)
    c2, by2, dr2 = oracle.histogram(s["ts"][perm], s["bytes"][perm], lab[perm], 1000, 1, 50_000)
    assert np.array_equal(c, c2) and np.array_equal(by, by2) and np.array_equal(dr, dr2)
    acc = (np.zeros((4, 50_000), np.uint64), np.zeros((4, 50_000), np.uint64),
           np.zeros((4, 2), np.uint64))
    for lo in range(0, wl.n, 7001):
        hi = min(wl.n, lo + 7001)
        oracle.histogram(s["ts"][lo:hi], s["bytes"][lo:hi], lab[lo:hi], 1000, 1, 50_000, out=acc)
    assert np.array_equal(acc[0], c) and np.array_equal(acc[1], by) and np.array_equal(acc[2], dr)
    assert win.n_bins == 60_000


def test_two_way_projection_matches_algorithm1():
    """The paper's two-way mark (Algorithm 1 on the source address) is bit 0
    of the label: outgoing iff the source matches some CIDR block."""
    import sinetgen
    wl = sinetgen.config(1, n=20_000)
    s = sinetgen.sessions(wl)
    lab = oracle.classify(wl.pbase, wl.plen, s["src"], s["dst"], want_inst=False)
    for i in range(0, 20_000, 97):
        a = int(s["src"][i])
        outgoing = any((((a & m) - (int(b) & m)) & 0xFFFFFFFF) == 0
                       for b, z in zip(wl.pbase.tolist(), wl.plen.tolist())
                       for m in [(0xFFFFFFFF << (32 - z)) & 0xFFFFFFFF if z else 0])
        assert bool(lab[i] & 1) == outgoing
    # exactly one label per session, and in-table share near the generator's 30%
    assert set(np.unique(lab).tolist()) <= {0, 1, 2, 3}
    share = np.mean(lab & 1)
    assert 0.27 < share < 0.33


def test_pipeline_equals_classify_then_histogram():
    import sinetgen
    wl = sinetgen.config(2, n=50_000)
    s = sinetgen.sessions(wl, start=0, stop=50_000)
    lab, c, by, dr = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"],
                                     0, 1, 86_400_000 // 1000)
    lab2 = oracle.classify(wl.pbase, wl.plen, s["src"], s["dst"], mode="scan", want_inst=False)
    assert np.array_equal(lab, lab2)
    c2, by2, dr2 = oracle.histogram(s["ts"], s["bytes"], lab2, 0, 1, 86_400_000 // 1000)
    assert np.array_equal(c, c2) and np.array_equal(by, by2) and np.array_equal(dr, dr2)


def test_label_bits_equal_institution_presence():
    """Bit 0 of the label is set exactly when the source has a longest match
    (an institution id), bit 1 likewise for the destination."""
    import sinetgen
    wl = sinetgen.config(2, n=30_000)
    s = sinetgen.sessions(wl, start=0, stop=30_000)
    lab, si, di = oracle.classify(wl.pbase, wl.plen, s["src"], s["dst"])
    assert np.array_equal((lab & 1) == 1, si != np.uint32(oracle.NO_INST))
    assert np.array_equal((lab >> 1) == 1, di != np.uint32(oracle.NO_INST))


def test_dense_bins_equal_the_papers_sparse_maps():
    """The paper's outputs are <timestamp,count> and <timestamp,bytes> maps
    per direction; built here with plain dictionaries, they are exactly the
    non-zero bins of the dense label-major histogram."""
    import sinetgen
    wl = sinetgen.config(1, n=5_000)
    s = sinetgen.sessions(wl)
    t0, width, n_bins = 500, 7, 8_000
    lab, c, by, dr = oracle.pipeline(wl.pbase, wl.plen, s["ts"], s["src"], s["dst"], s["bytes"],
                                     t0, width, n_bins)
    count_map = [dict() for _ in range(4)]
    bytes_map = [dict() for _ in range(4)]
    for i in range(wl.n):
        t = int(s["ts"][i])
        if t < t0 or (t - t0) // width >= n_bins:
            continue
        key = (t - t0) // width
        l = int(lab[i])
        count_map[l][key] = count_map[l].get(key, 0) + 1
        bytes_map[l][key] = (bytes_map[l].get(key, 0) + int(s["bytes"][i])) % (1 << 64)
    for l in range(4):
        nz = np.nonzero(c[l])[0]
        assert sorted(count_map[l]) == nz.tolist()
        assert all(count_map[l][k] == int(c[l][k]) for k in nz)
        assert all(bytes_map[l][k] == int(by[l][k]) for k in nz)


def test_scan_equals_hash_on_the_200k_table_sample():
    """The per-length hash mode (used to time and check the large tables)
    equals Algorithm 1's scan over all 200,000 prefixes on a sample of the
    large day's addresses, institutions included."""
    import sinetgen
    wl = sinetgen.config(4, n=4_000)
    s = sinetgen.sessions(wl, start=0, stop=wl.n)
    r1 = oracle.classify(wl.pbase, wl.plen, s["src"], s["dst"], mode="scan")
    r2 = oracle.classify(wl.pbase, wl.plen, s["src"], s["dst"], mode="hash")
    for x, y in zip(r1, r2):
        assert np.array_equal(x, y)
    assert 0 < int(np.count_nonzero(r1[0])) < wl.n   # both in- and out-of-table addresses
