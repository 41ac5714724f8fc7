"""Seeded synthetic session workloads shaped like the paper's SINET data.

This module is the only code shared by the CPU oracle and the GPU library's
tests and benchmark.  It holds no part of the method (no prefix matching,
no labelling, no binning): it only produces inputs.

Every session column value is a pure function of (workload, session index),
built from the SplitMix64 output function (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014) used as a counter
based generator, plus integer-only table interpolation.  The same integer
arithmetic is implemented for the GPU in ``gen.hip``; because no floating
point is evaluated per session, the two produce identical bytes, so any
sample of a multi-billion-session day can be regenerated on the host one
index at a time.

Shapes follow the paper's workload (section "Experimental Result"): a session
carries a millisecond capture time, source and destination IPv4 addresses and
a byte total (Table 1 items 1, 5, 8 and 21); a day holds 1.2-1.6 billion
sessions (Table 2) with a diurnal weekday pattern (Figures 6-7).  The SINET
prefix list and session logs are not public; every table and column here is
synthetic.
"""
from __future__ import annotations

import bisect
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

U64 = np.uint64
GOLDEN = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
KEYMUL = 0x632BE59BD9B4E019
M64 = (1 << 64) - 1

DAY_MS = 86_400_000
QTAB_K = 65536          # knots of the diurnal inverse-CDF table
QTAB_FRAC_BITS = 8      # the diurnal table holds ms * 256
LTAB_K = 65536          # knots of the lognormal quantile table

# column stream ids (one independent SplitMix64 stream each)
COL_TS, COL_SRC, COL_SRCP, COL_DST, COL_DSTP, COL_BYTES = 1, 2, 3, 4, 5, 6
COL_WSRC, COL_WDST = 7, 8   # watch-list overlay of sources / destinations

TS_UNIFORM, TS_DIURNAL, TS_STRATIFIED = 0, 1, 2


# ----------------------------------------------------------------------------
# SplitMix64 counter-based generator
# ----------------------------------------------------------------------------
def mix64_int(z: int) -> int:
    """SplitMix64 output function on a Python int (mod 2**64)."""
    z &= M64
    z = ((z ^ (z >> 30)) * MIX1) & M64
    z = ((z ^ (z >> 27)) * MIX2) & M64
    return z ^ (z >> 31)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wraps mod 2**64)."""
    z = z.astype(U64, copy=True)
    z ^= z >> U64(30)
    z *= U64(MIX1)
    z ^= z >> U64(27)
    z *= U64(MIX2)
    z ^= z >> U64(31)
    return z


def stream_key(seed: int, col: int) -> int:
    """Key of one column stream: mix64((seed << 16) ^ (col * KEYMUL))."""
    return mix64_int(((seed << 16) ^ (col * KEYMUL)) & M64)


def draw(key: int, idx: np.ndarray) -> np.ndarray:
    """Value number ``idx`` of the SplitMix64 sequence started at state ``key``.

    SplitMix64 advances its state by the golden gamma before mixing, so value
    i is mix64(key + (i + 1) * GOLDEN).
    """
    idx = np.asarray(idx, dtype=U64)
    st = (idx + U64(1)) * U64(GOLDEN) + U64(key)
    return mix64(st)


def _mulhi32(x32: np.ndarray, n: int) -> np.ndarray:
    """floor(x32 * n / 2**32) for 32-bit x32 and n <= 2**32 (exact in u64)."""
    return (x32.astype(U64) * U64(n)) >> U64(32)


# ----------------------------------------------------------------------------
# Integer interpolation tables (computed once on the host, shared with the GPU)
# ----------------------------------------------------------------------------
_LTAB_CACHE = {}
_QTAB_CACHE = {}


def lognormal_table(mu: float = 8.0, sigma: float = 2.0) -> np.ndarray:
    """Quantiles of lognormal(mu, sigma) at probabilities (k+0.5)/(K+1), k=0..K,
    rounded to integers.  A session's byte count interpolates this table
    linearly in integer arithmetic, so the distribution is lognormal up to a
    truncation of the tails at about 4.3 sigma."""
    key = (mu, sigma)
    if key not in _LTAB_CACHE:
        from scipy.special import ndtri
        p = (np.arange(LTAB_K + 1, dtype=np.float64) + 0.5) / (LTAB_K + 1)
        _LTAB_CACHE[key] = np.rint(np.exp(mu + sigma * ndtri(p))).astype(U64)
    return _LTAB_CACHE[key]


def diurnal_table(T: int = DAY_MS) -> np.ndarray:
    """Inverse CDF of the diurnal session rate, in ms * 256 at K+1 knots.

    The rate is proportional to 1 - 0.5 cos(2 pi t / T) on [0, T): peak over
    trough is 3, with the trough at t = 0.  Its CDF is
    F(t) = t/T - sin(2 pi t/T) / (4 pi); the knots solve F(t) = k/K by Newton
    in float64."""
    if T not in _QTAB_CACHE:
        u = np.arange(QTAB_K + 1, dtype=np.float64) / QTAB_K
        t = u * T
        w = 2.0 * math.pi / T
        for _ in range(60):
            F = t / T - np.sin(w * t) / (4.0 * math.pi)
            f = (1.0 - 0.5 * np.cos(w * t)) / T
            t = np.clip(t - (F - u) / f, 0.0, float(T))
        t[0] = 0.0
        t[-1] = float(T)
        q = np.rint(t * (1 << QTAB_FRAC_BITS)).astype(U64)
        q = np.maximum.accumulate(q)
        _QTAB_CACHE[T] = q
    return _QTAB_CACHE[T]


# ----------------------------------------------------------------------------
# Workload description
# ----------------------------------------------------------------------------
@dataclass
class Window:
    t0: int
    width: int
    n_bins: int


@dataclass
class Workload:
    """One stream of sessions and the prefix table it is classified against."""
    name: str
    n: int
    seed: int
    ts_mode: int                 # TS_UNIFORM / TS_DIURNAL / TS_STRATIFIED
    ts_span: int                 # uniform: ts range; diurnal: T; stratified: window W
    jitter: int = 0              # +-J ms reflected jitter (diurnal / stratified)
    t_origin: int = 0            # added to every ts
    in_frac: float = 0.3         # share of src (and of dst) drawn inside a table prefix
    pbase: np.ndarray = field(default_factory=lambda: np.zeros(0, np.uint32))
    plen: np.ndarray = field(default_factory=lambda: np.zeros(0, np.uint8))
    pinst: Optional[np.ndarray] = None
    window: Window = field(default_factory=lambda: Window(0, 1, 1))

    @property
    def n_prefix(self) -> int:
        return int(self.pbase.shape[0])

    @property
    def in_thr(self) -> int:
        return min(int(self.in_frac * 2.0 ** 32), 2 ** 32 - 1) if self.n_prefix else 0

    def keys(self):
        return [stream_key(self.seed, c) for c in
                (COL_TS, COL_SRC, COL_SRCP, COL_DST, COL_DSTP, COL_BYTES)]

    def hist_bytes(self) -> int:
        return 4 * self.window.n_bins * 16


# ----------------------------------------------------------------------------
# Session columns for arbitrary index sets (host)
# ----------------------------------------------------------------------------
def ts_base(wl: Workload, idx: np.ndarray) -> np.ndarray:
    """Un-jittered time of session i (non-decreasing in i), before the origin
    offset: the diurnal inverse CDF at (i + 1/2)/n, or a uniform rate."""
    i = np.asarray(idx).astype(np.int64)
    if wl.ts_mode == TS_DIURNAL:
        q = diurnal_table(wl.ts_span)
        num = (2 * i + 1) * QTAB_K
        den = 2 * wl.n
        k = num // den
        frac = num % den
        qk = q[k].astype(np.int64)
        dq = q[k + 1].astype(np.int64) - qk
        return (qk + (dq * frac) // den) >> QTAB_FRAC_BITS
    return ((2 * i + 1) * wl.ts_span) // (2 * wl.n)   # TS_STRATIFIED: uniform rate


def index_range_for_time(wl: Workload, t_lo: int, t_hi: int):
    """Smallest index range [i0, i1) holding every session whose un-jittered
    time lies in [t_lo, t_hi] (bisection on the monotone base)."""
    def first_at_least(t):
        lo, hi = 0, wl.n
        while lo < hi:
            mid = (lo + hi) // 2
            if int(ts_base(wl, np.array([mid]))[0]) >= t:
                hi = mid
            else:
                lo = mid + 1
        return lo
    return first_at_least(t_lo), first_at_least(t_hi + 1)


def _ts(wl: Workload, idx: np.ndarray) -> np.ndarray:
    r = draw(wl.keys()[0], idx) >> U64(32)
    if wl.ts_mode == TS_UNIFORM:
        t = _mulhi32(r, wl.ts_span).astype(np.int64)
        return (t + wl.t_origin).astype(np.uint32)
    base = ts_base(wl, idx)
    J = wl.jitter
    j = _mulhi32(r, 2 * J + 1).astype(np.int64) - J
    x = base + j
    T = wl.ts_span
    x = np.where(x < 0, -x - 1, x)
    x = np.where(x >= T, 2 * T - 1 - x, x)
    return (x + wl.t_origin).astype(np.uint32)


def _addr(wl: Workload, idx: np.ndarray, kcol: int, kpick: int) -> np.ndarray:
    r = draw(kcol, idx)
    host = (r >> U64(32)).astype(U64)
    if wl.n_prefix == 0:
        return host.astype(np.uint32)
    inside = (r & U64(0xFFFFFFFF)) < U64(wl.in_thr)
    p = _mulhi32(draw(kpick, idx) >> U64(32), wl.n_prefix).astype(np.int64)
    b = wl.pbase.astype(U64)[p]
    span = (U64(1) << (U64(32) - wl.plen.astype(U64)[p])) - U64(1)
    a = np.where(inside, b | (host & span), host)
    return a.astype(np.uint32)


def _bytes(wl: Workload, idx: np.ndarray) -> np.ndarray:
    L = lognormal_table()
    u = draw(wl.keys()[5], idx) >> U64(32)
    k = (u >> U64(16)).astype(np.int64)
    f = u & U64(0xFFFF)
    lo = L[k]
    d = L[k + 1] - lo
    return lo + ((d * f) >> U64(16))


def sessions(wl: Workload, idx=None, start: int = 0, stop: Optional[int] = None,
             watch: Optional["WatchList"] = None):
    """Columns ts/src/dst (uint32) and bytes (uint64) for the given indices
    (or the range [start, stop)); with ``watch``, the list's hosts are
    placed in (``watch_overlay``)."""
    if idx is None:
        stop = wl.n if stop is None else stop
        idx = np.arange(start, stop, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    k = wl.keys()
    src = _addr(wl, idx, k[1], k[2])
    dst = _addr(wl, idx, k[3], k[4])
    if watch is not None:
        src, dst = watch_overlay(watch, idx, src, dst)
    return {
        "ts": _ts(wl, idx),
        "src": src,
        "dst": dst,
        "bytes": _bytes(wl, idx),
    }


# ----------------------------------------------------------------------------
# Watch lists (sections "AbuseIPDB" and "GRIZZLY STEPPE": per-host session
# counts of published lists of malicious addresses)
# ----------------------------------------------------------------------------
@dataclass
class WatchList:
    """Listed hosts and how often sessions involve them.

    addrs: distinct /32 host addresses; lists: the list each host belongs to.
    With ``watch_overlay``, a share ``frac`` of the sessions has its source
    replaced by a listed host, and independently a share ``frac`` its
    destination; the host is drawn as floor(K * u^2) for u uniform in [0, 1),
    so a few hosts carry most of the listed sessions."""
    name: str
    addrs: np.ndarray
    lists: np.ndarray
    seed: int
    frac: float = 0.002

    @property
    def n(self) -> int:
        return int(self.addrs.shape[0])

    @property
    def thr(self) -> int:
        return min(int(self.frac * 2.0 ** 32), 2 ** 32 - 1)

    def keys(self):
        return stream_key(self.seed, COL_WSRC), stream_key(self.seed, COL_WDST)


def watch_lists(seed: int = 6, sizes=(300, 877), frac: float = 0.002) -> WatchList:
    """Two synthetic lists of distinct random /32 hosts, sized like the
    paper's AbuseIPDB sample (300 addresses) and the GRIZZLY STEPPE report
    (877 addresses).  The real lists are not used."""
    rng = np.random.Generator(np.random.PCG64(seed * 7919 + 6))
    need = int(sum(sizes))
    seen, addrs = set(), []
    while len(addrs) < need:
        a = int(rng.integers(0, 1 << 32))
        if a not in seen:
            seen.add(a)
            addrs.append(a)
    lists = np.concatenate([np.full(k, j, np.uint32) for j, k in enumerate(sizes)])
    return WatchList(f"watch-{'+'.join(str(k) for k in sizes)}hosts", np.asarray(addrs, np.uint32),
                     lists, seed, frac)


def watch_overlay(wlist: WatchList, idx: np.ndarray, src: np.ndarray, dst: np.ndarray):
    """Sources and destinations of sessions ``idx`` with the list's hosts
    placed in (new arrays)."""
    idx = np.asarray(idx, dtype=np.int64)
    out = []
    for key, col in zip(wlist.keys(), (src, dst)):
        r = draw(key, idx)
        hit = (r & U64(0xFFFFFFFF)) < U64(wlist.thr)
        u = r >> U64(32)
        pick = _mulhi32((u * u) >> U64(32), wlist.n).astype(np.int64)
        out.append(np.where(hit, wlist.addrs[pick], np.asarray(col, np.uint32)).astype(np.uint32))
    return out[0], out[1]


# ----------------------------------------------------------------------------
# Prefix tables
# ----------------------------------------------------------------------------
class _Disjoint:
    """Sorted set of disjoint half-open address ranges."""

    def __init__(self):
        self.starts: List[int] = []
        self.ends: List[int] = []

    def try_add(self, s: int, e: int) -> bool:
        i = bisect.bisect_right(self.starts, s)
        if i > 0 and self.ends[i - 1] > s:
            return False
        if i < len(self.starts) and self.starts[i] < e:
            return False
        self.starts.insert(i, s)
        self.ends.insert(i, e)
        return True


def _aligned(rng, L: int) -> int:
    """Uniform address aligned to a /L block."""
    if L == 0:
        return 0
    return int(rng.integers(0, 1 << L)) << (32 - L)


def _nested(rng, bases, lens, n_nested, max_len, max_extra=None):
    """Append n_nested prefixes, each strictly longer than and inside a random
    existing one (existing at the time of drawing)."""
    bases = list(bases)
    lens = list(lens)
    for _ in range(n_nested):
        while True:
            q = int(rng.integers(0, len(bases)))
            if lens[q] < max_len:
                break
        hi = max_len if max_extra is None else min(max_len, lens[q] + max_extra)
        L = int(rng.integers(lens[q] + 1, hi + 1))
        off = int(rng.integers(0, 1 << (L - lens[q]))) << (32 - L)
        bases.append(bases[q] + off)
        lens.append(L)
    return bases, lens


def _finish(rng, bases, lens, shuffle=True):
    b = np.asarray(bases, dtype=np.uint64).astype(np.uint32)
    l = np.asarray(lens, dtype=np.uint8)
    if shuffle:
        perm = rng.permutation(len(b))
        b, l = b[perm], l[perm]
    return b, l


def disjoint_table(rng, n: int, lmin: int, lmax: int):
    occ = _Disjoint()
    bases, lens = [], []
    while len(bases) < n:
        L = int(rng.integers(lmin, lmax + 1))
        for _ in range(64):
            s = _aligned(rng, L)
            if occ.try_add(s, s + (1 << (32 - L))):
                bases.append(s)
                lens.append(L)
                break
    return bases, lens


def table_tiny(seed: int):
    """64 disjoint prefixes, lengths 16..24, random canonical bases."""
    rng = np.random.Generator(np.random.PCG64(seed * 7919 + 1))
    b, l = disjoint_table(rng, 64, 16, 24)
    return _finish(rng, b, l)


def table_nested(seed: int, n: int, lmin: int, lmax: int, nested_frac: float):
    """n prefixes of lengths lmin..lmax; a share nested_frac of them lies
    strictly inside an earlier one (so longest-prefix match matters)."""
    rng = np.random.Generator(np.random.PCG64(seed * 7919 + 2))
    n_nest = int(round(n * nested_frac))
    b, l = disjoint_table(rng, n - n_nest, lmin, lmax)
    b, l = _nested(rng, b, l, n_nest, lmax)
    return _finish(rng, b, l)


def _block_length_weights():
    Ls = np.arange(8, 33)
    w = np.where(Ls <= 24, np.exp(-(24 - Ls) / 2.0), np.exp(-(Ls - 24) / 2.0))
    return Ls, w / w.sum()


def table_clustered(seed: int, n: int = 200_000, nested_frac: float = 0.3):
    """Large clustered table: top-level prefixes packed as consecutive aligned
    sub-prefixes of one length inside allocation blocks whose prefix count is
    lognormal(ln 20, 1); blocks sit at random aligned addresses without
    overlap.  Lengths 8..32 peak at /24, so coverage stays well below half of
    the address space.  A share nested_frac is nested (strictly longer, inside
    an existing prefix, at most 8 bits longer)."""
    rng = np.random.Generator(np.random.PCG64(seed * 7919 + 4))
    n_nest = int(round(n * nested_frac))
    n_top = n - n_nest
    Ls, w = _block_length_weights()
    occ = _Disjoint()
    bases, lens = [], []
    while len(bases) < n_top:
        L = int(rng.choice(Ls, p=w))
        c = int(np.clip(round(math.exp(rng.normal(math.log(20.0), 1.0))), 1, 4096))
        if L < 16:
            c = 1
        c = min(c, n_top - len(bases))
        kbits = 0 if c <= 1 else int(math.ceil(math.log2(c)))
        kbits = min(kbits, L)
        c = min(c, 1 << kbits)
        Lb = L - kbits
        for _ in range(64):
            s = _aligned(rng, Lb)
            if occ.try_add(s, s + (1 << (32 - Lb))):
                for slot in range(c):
                    bases.append(s + (slot << (32 - L)))
                    lens.append(L)
                break
    bases, lens = _nested(rng, bases, lens, n_nest, 32, max_extra=8)
    return _finish(rng, bases, lens)


def coverage(pbase: np.ndarray, plen: np.ndarray) -> float:
    """Share of the IPv4 space covered by the union of the prefixes."""
    s = pbase.astype(np.int64)
    e = s + (np.int64(1) << (32 - plen.astype(np.int64)))
    o = np.argsort(s, kind="stable")
    s, e = s[o], e[o]
    tot, cur_s, cur_e = 0, -1, -1
    for a, b in zip(s.tolist(), e.tolist()):
        if a >= cur_e:
            if cur_e > cur_s:
                tot += cur_e - cur_s
            cur_s, cur_e = a, b
        else:
            cur_e = max(cur_e, b)
    if cur_e > cur_s:
        tot += cur_e - cur_s
    return tot / float(1 << 32)


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------
_TABLE_CACHE = {}


def _cached(key, fn):
    if key not in _TABLE_CACHE:
        _TABLE_CACHE[key] = fn()
    return _TABLE_CACHE[key]


def config(k: int, n: Optional[int] = None, seed: Optional[int] = None):
    """Workload of configuration k (1..5); n overrides the session count.

    1 tiny: 1e6 sessions, ts uniform over one minute, 64 disjoint /16-/24.
    2 day: 1e8 sessions, diurnal nearly sorted day (+-5 s), 1,024 prefixes
      /12-/28, 20% nested.
    3 batch: see ``batch_streams``.
    4 learned: 5e8 sessions, config-2 time shape, 200,000 clustered prefixes.
    5 full day: 1.6e9 sessions, config-2 time shape, config-4 table.
    """
    seed = k if seed is None else seed
    if k == 1:
        b, l = _cached(("tiny", seed), lambda: table_tiny(seed))
        return Workload("tiny-1e6-64pfx-60k1ms", n or 1_000_000, seed, TS_UNIFORM,
                        60_000, pbase=b, plen=l, window=Window(0, 1, 60_000))
    if k == 2:
        b, l = _cached(("nested", seed), lambda: table_nested(seed, 1024, 12, 28, 0.2))
        return Workload("day-1e8-1024pfx-86.4M1ms", n or 100_000_000, seed, TS_DIURNAL,
                        DAY_MS, jitter=5000, pbase=b, plen=l,
                        window=Window(0, 1, DAY_MS))
    if k in (4, 5):
        b, l = _cached(("clustered", 4), lambda: table_clustered(4))
        nn = 500_000_000 if k == 4 else 1_600_000_000
        name = ("learned-5e8-200kpfx-86.4M1ms" if k == 4
                else "fullday-1.6e9-200kpfx-86.4M1ms")
        return Workload(name, n or nn, seed, TS_DIURNAL, DAY_MS, jitter=5000,
                        pbase=b, plen=l, window=Window(0, 1, DAY_MS))
    raise ValueError("config 3 is a batch: use batch_streams()")


def batch_streams(seed: int = 3, n_streams: int = 64, total: int = 300_000_000,
                  hist_cap: int = 32 << 30) -> List[Workload]:
    """Config 3: many independent uneven streams.

    Sizes lognormal(ln 2.5e6, 1.2) clipped to [1e4, 2e7] and rescaled to sum to
    about ``total``; window log-uniform over [1 min, 24 h]; bin width uniform
    over {1, 10, 1000} ms; each stream has its own table (64-4,096 prefixes,
    lengths 8-28, 20% nested), its own origin and +-min(5 s, W/20) jitter.
    Windows are redrawn while the summed histogram exceeds ``hist_cap`` bytes.
    """
    rng = np.random.Generator(np.random.PCG64(seed * 7919 + 3))
    sz = np.exp(rng.normal(math.log(2.5e6), 1.2, n_streams))
    for _ in range(8):
        sz = np.clip(sz * (total / sz.sum()), 1e4, 2e7)
    sizes = [int(round(x)) for x in sz]
    wins, widths = [], []
    for _ in range(n_streams):
        wins.append(int(round(math.exp(rng.uniform(math.log(6e4), math.log(8.64e7))))))
        widths.append(int(rng.choice([1, 10, 1000])))

    def hist_total():
        return sum(4 * 16 * -(-W // w) for W, w in zip(wins, widths))

    while hist_total() > hist_cap:
        s = int(np.argmax([-(-W // w) for W, w in zip(wins, widths)]))
        wins[s] = int(round(math.exp(rng.uniform(math.log(6e4), math.log(8.64e7)))))
    out = []
    for s in range(n_streams):
        W, w = wins[s], widths[s]
        npfx = int(round(math.exp(rng.uniform(math.log(64), math.log(4096)))))
        sseed = seed * 1000 + s
        b, l = _cached(("stream", sseed, npfx),
                       lambda: table_nested(sseed, npfx, 8, 28, 0.2))
        origin = int(rng.integers(0, DAY_MS - W + 1))
        out.append(Workload(f"stream{s}", sizes[s], sseed, TS_STRATIFIED, W,
                            jitter=min(5000, W // 20), t_origin=origin,
                            pbase=b, plen=l,
                            window=Window(origin, w, -(-W // w))))
    return out
