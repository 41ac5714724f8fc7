"""Synthetic session log text shaped like the paper's PA-7080 records.

Each session becomes one line of the 24 fields of Table 1 ("PA-7080 data
description") in that order, separated by commas and ended by a newline:

  1 capture_time      YYYY/MM/DD HH:MM:SS.mmm  (the session's ts, from the
                                                 origin day's midnight)
  2 generated_time    YYYY/MM/DD HH:MM:SS
  3 start_time        YYYY/MM/DD HH:MM:SS      (capture time minus elapsed)
  4 elapsed_time      seconds
  5 source_ip         dotted quad
  6 source_port
  7 src_country_code  two letters
  8 destination_ip    dotted quad
  9 destination_port
 10 dest_country_code
 11 protocol, 12 application, 13 subtype, 14 action, 15 session_end_reason
 16 repeat_count, 17 category
 18 packets, 19 packets_sent, 20 packets_received
 21 bytes             the session's byte total
 22 bytes_sent, 23 bytes_received
 24 device_name

Fields 1, 5, 8 and 21 carry the session columns; the others are filled from
their own SplitMix64 streams so that lines have realistic, varying lengths
(about 200 bytes).  Formatting is vectorised numpy integer arithmetic; the
calendar conversion is the days-to-civil algorithm of H. Hinnant ("chrono-
Compatible Low-Level Date Algorithms").  This module holds no part of the
parsing or of the method; it only produces inputs.
"""
from __future__ import annotations

import numpy as np

from . import U64, Workload, draw, sessions, stream_key

COL_TEXT = 9  # stream of the filler fields
ORIGIN_DAYS = 18_677  # 2021-02-19, the SINET day of Table 2, as days since 1970-01-01

_COUNTRIES = [b"JP", b"US", b"CN", b"KR", b"DE", b"GB", b"FR", b"NL", b"SG", b"NA"]
_PROTOS = [b"tcp", b"udp", b"icmp"]
_APPS = [b"ssl", b"web-browsing", b"dns", b"ntp", b"quic", b"ssh", b"smtp", b"incomplete"]
_SUBTYPES = [b"end", b"start", b"drop", b"deny"]
_ACTIONS = [b"allow", b"deny", b"drop", b"reset-both"]
_REASONS = [b"tcp-fin", b"aged-out", b"tcp-rst-from-client", b"tcp-rst-from-server", b"policy-deny"]
_CATEGORIES = [b"any", b"computer-and-internet-info", b"search-engines", b"educational-institutions"]


def civil_from_days(z: np.ndarray):
    """(year, month, day) of days since 1970-01-01 (proleptic Gregorian)."""
    z = np.asarray(z, dtype=np.int64) + 719_468
    era = np.floor_divide(z, 146_097)
    doe = z - era * 146_097
    yoe = (doe - doe // 1460 + doe // 36_524 - doe // 146_096) // 365
    y = yoe + era * 400
    doy = doe - (365 * yoe + yoe // 4 - yoe // 100)
    mp = (5 * doy + 2) // 153
    d = doy - (153 * mp + 2) // 5 + 1
    m = np.where(mp < 10, mp + 3, mp - 9)
    y = np.where(m <= 2, y + 1, y)
    return y, m, d


def _digits(x: np.ndarray, width: int = 0):
    """Decimal digits of non-negative integers: (chars[n, w] uint8 right
    aligned in w columns, length[n]); width > 0 zero-pads to that width."""
    x = np.asarray(x, dtype=U64)
    n = x.shape[0]
    w = max(width, 20)
    out = np.zeros((n, w), np.uint8)
    v = x.copy()
    for c in range(w - 1, -1, -1):
        out[:, c] = (v % U64(10)).astype(np.uint8) + ord("0")
        v //= U64(10)
    length = np.ones(n, np.int64)
    p = U64(10)
    for k in range(1, 20):
        length += (x >= p).astype(np.int64)
        if k < 19:
            p = p * U64(10)
    if width:
        length = np.maximum(length, width)
    return out, length


def _pick(choices, r: np.ndarray):
    """Strings from a list, chosen by the high words of draws r."""
    w = max(len(c) for c in choices)
    table = np.zeros((len(choices), w), np.uint8)
    lens = np.array([len(c) for c in choices], np.int64)
    for i, c in enumerate(choices):
        table[i, w - len(c):] = np.frombuffer(c, np.uint8)
    k = ((r >> U64(32)) * U64(len(choices)) >> U64(32)).astype(np.int64)
    return table[k], lens[k]


def _fixed(text: bytes, n: int):
    a = np.frombuffer(text, np.uint8)
    return np.broadcast_to(a, (n, a.shape[0])), np.full(n, a.shape[0], np.int64)


def _join(parts):
    """Right-aligned (chars, length) pieces concatenated row by row into one
    byte string per row, rows concatenated: (buffer, row offsets[n + 1])."""
    n = parts[0][1].shape[0]
    row_len = np.zeros(n, np.int64)
    for _, ln in parts:
        row_len += ln
    offs = np.zeros(n + 1, np.int64)
    np.cumsum(row_len, out=offs[1:])
    buf = np.empty(int(offs[-1]), np.uint8)
    pos = offs[:-1].copy()
    for chars, ln in parts:
        w = chars.shape[1]
        for c in range(w):
            # column c of a right-aligned piece holds character c - (w - ln)
            j = c - (w - ln)
            m = j >= 0
            if m.any():
                buf[pos[m] + j[m]] = chars[m, c]
        pos += ln
    return buf, offs


def _datetime(days, ms_of_day, with_ms: bool):
    y, mo, d = civil_from_days(days)
    h = ms_of_day // 3_600_000
    mi = (ms_of_day // 60_000) % 60
    s = (ms_of_day // 1000) % 60
    parts = [_digits(y, 4), _fixed(b"/", len(y)), _digits(mo, 2), _fixed(b"/", len(y)),
             _digits(d, 2), _fixed(b" ", len(y)), _digits(h, 2), _fixed(b":", len(y)),
             _digits(mi, 2), _fixed(b":", len(y)), _digits(s, 2)]
    if with_ms:
        parts += [_fixed(b".", len(y)), _digits(ms_of_day % 1000, 3)]
    return parts


def _ip(a: np.ndarray):
    a = np.asarray(a, dtype=np.uint32).astype(np.int64)
    n = a.shape[0]
    out = []
    for k, sh in enumerate((24, 16, 8, 0)):
        out.append(_digits((a >> sh) & 255))
        if k < 3:
            out.append(_fixed(b".", n))
    return out


def session_lines(wl: Workload, start: int = 0, stop=None, origin_days: int = ORIGIN_DAYS,
                  watch=None, cols=None):
    """Text of sessions [start, stop) of ``wl`` (or of the given columns
    ts/src/dst/bytes): (bytes buffer uint8, line offsets int64[n + 1])."""
    if cols is None:
        stop = wl.n if stop is None else stop
        cols = sessions(wl, start=start, stop=stop, watch=watch)
    n = cols["ts"].shape[0]
    idx = np.arange(start, start + n, dtype=np.int64)
    key = stream_key(wl.seed, COL_TEXT)
    r = [draw(key ^ (k * 0x9E3779B97F4A7C15 & ((1 << 64) - 1)), idx) for k in range(12)]
    ts = cols["ts"].astype(np.int64)
    days = origin_days + ts // 86_400_000
    msd = ts % 86_400_000
    elapsed = ((r[0] >> U64(32)) % U64(600)).astype(np.int64)
    start_ms = np.maximum(msd - elapsed * 1000, 0)
    nb = cols["bytes"].astype(U64)
    packets = nb // U64(900) + U64(1)
    sent = nb * ((r[1] >> U64(40)) % U64(100)) // U64(100)
    psent = packets * ((r[1] >> U64(48)) % U64(100)) // U64(100)
    comma = _fixed(b",", n)
    fields = [
        _datetime(days, msd, True),
        _datetime(days, msd - msd % 1000, False),
        _datetime(days, start_ms - start_ms % 1000, False),
        [_digits(elapsed)],
        _ip(cols["src"]),
        [_digits((r[2] >> U64(48)).astype(np.int64))],
        [_pick(_COUNTRIES, r[3])],
        _ip(cols["dst"]),
        [_digits((r[4] >> U64(48)).astype(np.int64))],
        [_pick(_COUNTRIES, r[5])],
        [_pick(_PROTOS, r[6])],
        [_pick(_APPS, r[7])],
        [_pick(_SUBTYPES, r[8])],
        [_pick(_ACTIONS, r[9])],
        [_pick(_REASONS, r[10])],
        [_digits((r[11] >> U64(62)).astype(np.int64))],
        [_pick(_CATEGORIES, r[11])],
        [_digits(packets)],
        [_digits(psent)],
        [_digits(packets - psent)],
        [_digits(nb)],
        [_digits(sent)],
        [_digits(nb - sent)],
        [_fixed(b"PA-7080", n)],
    ]
    parts = []
    for i, f in enumerate(fields):
        parts += f
        parts.append(comma if i < len(fields) - 1 else _fixed(b"\n", n))
    return _join(parts)
