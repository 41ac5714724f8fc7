"""Pins of the oracle's session-text parser (section "Dataset Description",
Table 1): hand-worked lines, the calendar against Python's datetime, the
generator's text round trip, and the line rules (empty lines, a last line
without a newline)."""
import datetime
import os

import numpy as np

import oracle
import sinetgen
from sinetgen import text

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "parse_examples.txt")


def _golden():
    out = []
    with open(GOLDEN) as f:
        for line in f:
            if not line.startswith("pline\t"):
                continue
            _, origin, expect, body = line.rstrip("\n").split("\t")
            out.append((int(origin), expect, body))
    return out


def test_parse_hand_examples():
    cases = _golden()
    assert len(cases) >= 25
    for origin, expect, body in cases:
        cols, bad = oracle.parse((body + "\n").encode(), origin)
        assert all(v.shape[0] == 1 for v in cols.values()), body
        got = (int(cols["ts"][0]), int(cols["src"][0]), int(cols["dst"][0]), int(cols["bytes"][0]))
        if expect == "BAD":
            assert bad == 1 and got == (0xFFFFFFFF, 0, 0, 0), body
        else:
            t, s, d, b = expect.split(",")
            assert bad == 0, body
            assert got == (int(t), int(s, 16), int(d, 16), int(b)), body


def test_parse_calendar_against_datetime():
    """Random capture times from 1970 to 2200: the parsed offset from the
    origin day equals datetime's difference in milliseconds."""
    rng = np.random.default_rng(8)
    epoch = datetime.datetime(1970, 1, 1)
    lines, exp, origins = [], [], []
    for _ in range(3000):
        day = int(rng.integers(0, 84_000))
        dt = epoch + datetime.timedelta(days=day, milliseconds=int(rng.integers(0, 86_400_000)))
        origin = day - int(rng.integers(0, 45))
        ms = (dt - (epoch + datetime.timedelta(days=origin))) // datetime.timedelta(milliseconds=1)
        cap = dt.strftime("%Y/%m/%d %H:%M:%S.") + f"{dt.microsecond // 1000:03d}"
        lines.append(f"{cap},a,b,c,1.2.3.4,p,q,5.6.7.8,x,x,x,x,x,x,x,x,x,x,x,x,9")
        exp.append(ms)
        origins.append(origin)
    for line, e, o in zip(lines, exp, origins):
        cols, bad = oracle.parse((line + "\n").encode(), o)
        assert bad == 0 and int(cols["ts"][0]) == e, line


def test_parse_round_trip_of_generated_text():
    """The generator's lines (formatted by numpy, separately from the
    parser) parse back to the columns they were made from, including byte
    counts up to 2^64 - 1 and the watch-list overlay's addresses."""
    wl = sinetgen.config(2, n=50_000)
    s = sinetgen.sessions(wl, start=1_000, stop=31_000, watch=sinetgen.watch_lists(frac=0.05))
    s["bytes"] = s["bytes"].copy()
    s["bytes"][:3] = [0, 1 << 63, (1 << 64) - 1]
    buf, offs = text.session_lines(wl, start=1_000, cols=s)
    assert offs.shape[0] == 30_001 and buf[-1] == 10
    cols, bad = oracle.parse(buf, text.ORIGIN_DAYS)
    assert bad == 0
    for k in ("ts", "src", "dst", "bytes"):
        assert np.array_equal(cols[k], s[k]), k
    assert 150 < buf.shape[0] / 30_000 < 260   # about 200 bytes per line, as in the paper


def test_parse_line_rules():
    good = "2021/02/19 00:00:01.000,a,b,c,1.2.3.4,p,q,5.6.7.8,x,x,x,x,x,x,x,x,x,x,x,x,9"
    # an empty line counts (bad); a last line without newline counts; a final
    # newline does not start another line
    t = (good + "\n\n" + good).encode()
    cols, bad = oracle.parse(t, text.ORIGIN_DAYS)
    assert cols["ts"].tolist() == [1000, 0xFFFFFFFF, 1000] and bad == 1
    cols, bad = oracle.parse((good + "\n").encode(), text.ORIGIN_DAYS)
    assert cols["ts"].shape[0] == 1 and bad == 0
    cols, bad = oracle.parse(b"", text.ORIGIN_DAYS)
    assert cols["ts"].shape[0] == 0 and bad == 0
    # a carriage return belongs to the last field, which is not parsed
    cols, bad = oracle.parse((good + ",x,x,PA\r\n").encode(), text.ORIGIN_DAYS)
    assert bad == 0 and int(cols["bytes"][0]) == 9


def test_civil_from_days_of_the_generator():
    """The generator's date conversion agrees with datetime (it formats the
    capture times the parser reads)."""
    days = np.array([0, 59, 60, 365, 11_016, 18_321, 18_677, 47_541, 84_000])
    y, m, d = text.civil_from_days(days)
    for k, z in enumerate(days):
        dt = datetime.date(1970, 1, 1) + datetime.timedelta(days=int(z))
        assert (int(y[k]), int(m[k]), int(d[k])) == (dt.year, dt.month, dt.day)


def test_parse_day_validity_against_datetime():
    """Random year/month/day triples, impossible ones included: a line parses
    exactly when datetime accepts the date, at (day - 1) days past the first
    of its month."""
    rng = np.random.default_rng(9)
    epoch = datetime.date(1970, 1, 1)
    n_bad = 0
    for _ in range(4000):
        y, m, d = int(rng.integers(1970, 2300)), int(rng.integers(1, 13)), int(rng.integers(1, 32))
        origin = (datetime.date(y, m, 1) - epoch).days
        line = f"{y:04d}/{m:02d}/{d:02d} 00:00:00.000,a,b,c,1.2.3.4,p,q,5.6.7.8,x,x,x,x,x,x,x,x,x,x,x,x,9"
        cols, bad = oracle.parse((line + "\n").encode(), origin)
        try:
            datetime.date(y, m, d)
            assert bad == 0 and int(cols["ts"][0]) == (d - 1) * 86_400_000, line
        except ValueError:
            n_bad += 1
            assert bad == 1, line
    assert n_bad > 30
