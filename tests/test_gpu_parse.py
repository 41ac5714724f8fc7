"""GPU parity of session-text parsing (sinet_parse_sessions) against the CPU
oracle: generated Table 1 lines, the hand-worked lines, ragged and
misaligned text, lines too long for the LDS staging, random bytes, and the
parsed columns through the pipeline."""
import os
import sys

import numpy as np
import pytest

import oracle
import sinetgen
from sinetgen import text as stext

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "parse_examples.txt")


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


def _dev_text(torch, buf):
    return torch.from_numpy(np.array(buf, dtype=np.uint8)).cuda()  # a writable host copy


def _check(sinet, torch, buf, origin, off=0):
    """Parse buf on the device (placed off bytes into its allocation, so the
    text's address is misaligned for off % 16 != 0) and compare with the
    oracle."""
    pad = np.concatenate([np.zeros(off, np.uint8), np.ascontiguousarray(buf, dtype=np.uint8)])
    cols, bad = sinet.parse_sessions(_dev_text(torch, pad)[off:], origin)
    torch.cuda.synchronize()
    exp, ebad = oracle.parse(np.ascontiguousarray(buf, dtype=np.uint8), origin)
    assert bad == ebad
    assert cols["ts"].shape[0] == exp["ts"].shape[0]
    for k in ("ts", "src", "dst"):
        assert np.array_equal(sinet.to_host_u32(cols[k]), exp[k]), k
    assert np.array_equal(sinet.to_host_u64(cols["bytes"]), exp["bytes"])
    return cols, exp, bad


def test_parse_generated_day_sample(sinet, torch):
    wl = sinetgen.config(2, n=2_000_000)
    _say("parse generated")
    buf, offs = stext.session_lines(wl, start=700_000, stop=1_000_000,
                                    watch=sinetgen.watch_lists(frac=0.01))
    cols, exp, bad = _check(sinet, torch, buf, stext.ORIGIN_DAYS)
    assert bad == 0 and cols["ts"].shape[0] == 300_000
    s = sinetgen.sessions(wl, start=700_000, stop=1_000_000, watch=sinetgen.watch_lists(frac=0.01))
    assert np.array_equal(exp["src"], s["src"]) and np.array_equal(exp["bytes"], s["bytes"])
    # the parsed columns through the pipeline equal the generated columns' result
    tab = sinet.Table(wl.pbase, wl.plen)
    w = wl.window
    lab1, h1 = sinet.pipeline(tab, cols["ts"], cols["src"], cols["dst"], cols["bytes"], w.t0,
                              w.width, w.n_bins)
    d = (sinet.to_device_u32(s["ts"]), sinet.to_device_u32(s["src"]), sinet.to_device_u32(s["dst"]),
         sinet.to_device_u64(s["bytes"]))
    lab2, h2 = sinet.pipeline(tab, *d, w.t0, w.width, w.n_bins)
    torch.cuda.synchronize()
    assert torch.equal(lab1, lab2) and all(torch.equal(x, y) for x, y in zip(h1, h2))


def test_parse_full_4gb_chunk(sinet, torch):
    """The benchmark's chunk and launch: 500,000 lines generated from the
    middle of the full synthetic day, repeated 40 times on the device
    (3.97 GB, 20 M lines); every output equals the oracle's parse of the
    500,000 lines."""
    wl = sinetgen.config(5)
    i0, unit, reps = wl.n // 2, 500_000, 40
    _say("parse 4 GB chunk")
    buf, _ = stext.session_lines(wl, start=i0, stop=i0 + unit)
    exp, ebad = oracle.parse(buf, stext.ORIGIN_DAYS)
    assert ebad == 0
    dev = torch.from_numpy(buf).cuda().repeat(reps)
    cols, bad = sinet.parse_sessions(dev, stext.ORIGIN_DAYS, capacity=unit * reps)
    torch.cuda.synchronize()
    assert bad == 0 and cols["ts"].shape[0] == unit * reps
    for k in ("ts", "src", "dst"):
        got = sinet.to_host_u32(cols[k]).reshape(reps, unit)
        assert (got == exp[k][None, :]).all(), k
    got = sinet.to_host_u64(cols["bytes"]).reshape(reps, unit)
    assert (got == exp["bytes"][None, :]).all()


def test_parse_hand_examples(sinet, torch):
    by_origin = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("pline\t"):
                _, origin, _, body = line.rstrip("\n").split("\t")
                by_origin.setdefault(int(origin), []).append(body)
    for origin, bodies in by_origin.items():
        buf = np.frombuffer(("\n".join(bodies) + "\n").encode(), np.uint8)
        _check(sinet, torch, buf, origin)


def test_parse_ragged_misaligned_and_long_lines(sinet, torch):
    wl = sinetgen.config(1, n=20_000)
    buf, _ = stext.session_lines(wl, start=0, stop=5_000)
    # misaligned text, no final newline, empty lines and a carriage return
    extra = b"\n\n" + bytes(buf[:500]).replace(b"\n", b"\r\n") + b"2021/02/19 00:00:01.000,x"
    for t, off in ((buf[1:], 3), (buf[:-1], 0), (np.concatenate([buf, np.frombuffer(extra, np.uint8)]), 5),
                   (buf[7:12_345], 9)):
        _check(sinet, torch, t, stext.ORIGIN_DAYS, off)
    # lines too long for the LDS staging of a group (a long last field)
    rows = bytes(buf).split(b"\n")[:600]
    long_lines = b"".join(r + b"," + (b"y" * (100 + 7 * (i % 90))) + b"\n" for i, r in enumerate(rows))
    cols, exp, bad = _check(sinet, torch, np.frombuffer(long_lines, np.uint8), stext.ORIGIN_DAYS)
    assert bad == 0 and cols["ts"].shape[0] == 600
    # single lines longer than the whole staging (parsed from device memory):
    # good ones with a long 24th field, a bad one with a long 21st field, between
    # ordinary lines and as the last line without newline
    giant = [rows[1] + b"," + b"z" * 70_001, b",".join(rows[2].split(b",")[:20]) + b"," + b"7" * 66_000]
    mixed = b"\n".join(rows[:300] + giant[:1] + rows[300:500] + giant[1:] + rows[500:] + giant[:1])
    cols, exp, bad = _check(sinet, torch, np.frombuffer(mixed, np.uint8), stext.ORIGIN_DAYS, 1)
    assert cols["ts"].shape[0] == 603 and bad == 1


def test_parse_random_bytes_and_capacity(sinet, torch):
    rng = np.random.default_rng(12)
    alphabet = np.frombuffer(b"0123456789/:., \nab", np.uint8)
    for n in (1, 17, 4_097, 200_003):
        buf = alphabet[rng.integers(0, alphabet.shape[0], n)]
        _check(sinet, torch, buf, 0)
    good = b"2021/02/19 00:00:01.000,a,b,c,1.2.3.4,p,q,5.6.7.8,x,x,x,x,x,x,x,x,x,x,x,x,9\n"
    t = _dev_text(torch, np.frombuffer(good * 10, np.uint8))
    with pytest.raises(sinet.SinetError):
        sinet.parse_sessions(t, stext.ORIGIN_DAYS, capacity=9)
    cols, bad = sinet.parse_sessions(t, stext.ORIGIN_DAYS, capacity=10)
    torch.cuda.synchronize()
    assert bad == 0 and cols["ts"].shape[0] == 10 and int(cols["ts"][9]) == 1000
    empty, bad = sinet.parse_sessions(t[:0], stext.ORIGIN_DAYS)
    assert empty["ts"].shape[0] == 0 and bad == 0
