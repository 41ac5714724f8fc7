"""CPU oracle for discrimination and millisecond histogramming, and for the
watch-list histograms, coarser time frames and session-text parsing beside
them.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the GPU library never does, and this
package never imports the GPU library.  The arithmetic lives in plain C
(``sinet_oracle.c``, single-threaded, built with gcc) and, for the learned
index, in float64 numpy (``learned.py``).  See the C file's header for the
definitions and the passages of the paper they follow.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sinet_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
NO_INST = 0xFFFFFFFF

EXTERNAL, EGRESS, INGRESS, INTERNAL = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no vectorisation tricks)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.or_bitmask.argtypes = [u32, i32]
        L.or_bitmask.restype = u32
        L.or_match.argtypes = [u32, u32, i32]
        L.or_match.restype = i32
        L.or_lookup_scan.argtypes = [P, P, u64, u32, P]
        L.or_lookup_scan.restype = i32
        L.or_classify.argtypes = [P, P, P, u64, i32, P, P, u64, P, P, P]
        L.or_classify.restype = i32
        L.or_histogram.argtypes = [P, P, P, u64, u32, u32, u32, P, P, P, i32]
        L.or_histogram.restype = i32
        L.or_pipeline.argtypes = [P, P, P, u64, i32, P, P, P, P, u64, u32, u32, u32,
                                  P, P, P, P, i32]
        L.or_pipeline.restype = i32
        L.or_watch.argtypes = [P, P, P, u64, i32, P, P, P, P, u64, u32, u32, u32, u32,
                               P, P, P, i32]
        L.or_watch.restype = i32
        L.or_rebin.argtypes = [P, u64, u64, u64, P]
        L.or_rebin.restype = i32
        L.or_parse.argtypes = [P, u64, ctypes.c_int64, P, P, P, P, u64, P, P]
        L.or_parse.restype = i32
        L.or_label_runs.argtypes = [P, u64, P, P]
        L.or_label_runs.restype = i32
        L.or_endpoints.argtypes = [P, P, u64, P, P]
        L.or_endpoints.restype = ctypes.c_int64
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _table(base, plen, inst=None):
    base = np.ascontiguousarray(base, dtype=np.uint32)
    plen = np.ascontiguousarray(plen, dtype=np.uint8)
    if inst is not None:
        inst = np.ascontiguousarray(inst, dtype=np.uint32)
    return base, plen, inst


def bitmask(x: int, z: int) -> int:
    return int(lib().or_bitmask(x & 0xFFFFFFFF, z))


def match(a: int, base: int, z: int) -> bool:
    return bool(lib().or_match(a & 0xFFFFFFFF, base & 0xFFFFFFFF, z))


def lookup_scan(base, plen, a: int):
    """(in, row) of one address by the linear Algorithm-1 scan."""
    base, plen, _ = _table(base, plen)
    row = ctypes.c_int64(-1)
    hit = lib().or_lookup_scan(_p(base), _p(plen), base.shape[0], a & 0xFFFFFFFF,
                               ctypes.byref(row))
    return bool(hit), int(row.value)


def classify(base, plen, src, dst, inst=None, mode: str = "hash", want_inst: bool = True):
    """label[n] (uint8) and, if asked, src_inst/dst_inst[n] (uint32)."""
    base, plen, inst = _table(base, plen, inst)
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    n = src.shape[0]
    label = np.empty(n, np.uint8)
    si = np.empty(n, np.uint32) if want_inst else None
    di = np.empty(n, np.uint32) if want_inst else None
    rc = lib().or_classify(_p(base), _p(plen), _p(inst), base.shape[0],
                           0 if mode == "scan" else 1, _p(src), _p(dst), n,
                           _p(label), _p(si), _p(di))
    assert rc == 0
    return (label, si, di) if want_inst else label


def histogram(ts, nbytes, label, t0: int, width: int, n_bins: int, out=None):
    """(count[4, n_bins], bytes[4, n_bins], dropped[4, 2]) as uint64.
    With ``out`` given, adds into it (the accumulate mode)."""
    ts = np.ascontiguousarray(ts, dtype=np.uint32)
    nbytes = np.ascontiguousarray(nbytes, dtype=np.uint64)
    label = np.ascontiguousarray(label, dtype=np.uint8)
    if out is None:
        cnt = np.empty((4, n_bins), np.uint64)
        byt = np.empty((4, n_bins), np.uint64)
        drp = np.empty((4, 2), np.uint64)
        acc = 0
    else:
        cnt, byt, drp = out
        acc = 1
    rc = lib().or_histogram(_p(ts), _p(nbytes), _p(label), ts.shape[0], t0, width, n_bins,
                            _p(cnt), _p(byt), _p(drp), acc)
    assert rc == 0
    return cnt, byt, drp


def pipeline(base, plen, ts, src, dst, nbytes, t0, width, n_bins, inst=None,
             mode: str = "hash"):
    """(label, count, bytes, dropped) of the fused definition."""
    base, plen, inst = _table(base, plen, inst)
    ts = np.ascontiguousarray(ts, dtype=np.uint32)
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    nbytes = np.ascontiguousarray(nbytes, dtype=np.uint64)
    n = ts.shape[0]
    label = np.empty(n, np.uint8)
    cnt = np.empty((4, n_bins), np.uint64)
    byt = np.empty((4, n_bins), np.uint64)
    drp = np.empty((4, 2), np.uint64)
    rc = lib().or_pipeline(_p(base), _p(plen), _p(inst), base.shape[0],
                           0 if mode == "scan" else 1, _p(ts), _p(src), _p(dst), _p(nbytes),
                           n, t0, width, n_bins, _p(label), _p(cnt), _p(byt), _p(drp), 0)
    assert rc == 0
    return label, cnt, byt, drp


def watch(base, plen, ts, src, dst, nbytes, t0, width, n_bins, n_keys, inst=None,
          mode: str = "hash", out=None):
    """Watch-list histograms: (count[2, n_keys, n_bins], bytes[2, n_keys,
    n_bins], dropped[2, 2]) as uint64.  Direction 0 counts sessions whose
    source matches the list (key of its longest match), direction 1 those
    whose destination does.  With ``out`` given, adds into it."""
    base, plen, inst = _table(base, plen, inst)
    ts = np.ascontiguousarray(ts, dtype=np.uint32)
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    nbytes = np.ascontiguousarray(nbytes, dtype=np.uint64)
    if out is None:
        cnt = np.empty((2, n_keys, n_bins), np.uint64)
        byt = np.empty((2, n_keys, n_bins), np.uint64)
        drp = np.empty((2, 2), np.uint64)
        acc = 0
    else:
        cnt, byt, drp = out
        acc = 1
    rc = lib().or_watch(_p(base), _p(plen), _p(inst), base.shape[0],
                        0 if mode == "scan" else 1, _p(ts), _p(src), _p(dst), _p(nbytes),
                        ts.shape[0], t0, width, n_bins, n_keys, _p(cnt), _p(byt), _p(drp), acc)
    if rc == 2:
        raise ValueError("a key is not below n_keys")
    assert rc == 0
    return cnt, byt, drp


def label_runs(label):
    """Session indices partitioned by label, stably (uint32 [n]), and the
    number of sessions with each label (uint64 [4])."""
    label = np.ascontiguousarray(label, dtype=np.uint8)
    n = label.shape[0]
    idx = np.empty(n, np.uint32)
    totals = np.zeros(4, np.uint64)
    rc = lib().or_label_runs(_p(label), n, _p(idx), _p(totals))
    if rc == 1:
        raise ValueError("2^32 sessions or more")
    assert rc == 0
    return idx, totals


def rebin(a, factor: int):
    """Coarser frames of a [..., n_bins] uint64 histogram: every group of
    ``factor`` consecutive bins summed (the last group may be shorter)."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    n_bins = a.shape[-1]
    rows = int(np.prod(a.shape[:-1], dtype=np.int64)) if a.ndim > 1 else 1
    n_out = -(-n_bins // factor)
    out = np.empty(a.shape[:-1] + (n_out,), np.uint64)
    rc = lib().or_rebin(_p(a), rows, n_bins, factor, _p(out))
    assert rc == 0
    return out


def parse(text, origin_days: int):
    """Session text (bytes or a uint8 array) to columns: dict of ts, src,
    dst (uint32) and bytes (uint64), plus the number of bad lines."""
    buf = np.frombuffer(text, np.uint8) if isinstance(text, (bytes, bytearray)) else \
        np.ascontiguousarray(text, dtype=np.uint8)
    cap = int(np.count_nonzero(buf == 10)) + 1
    cols = {"ts": np.empty(cap, np.uint32), "src": np.empty(cap, np.uint32),
            "dst": np.empty(cap, np.uint32), "bytes": np.empty(cap, np.uint64)}
    n = ctypes.c_uint64(0)
    bad = ctypes.c_uint64(0)
    rc = lib().or_parse(_p(buf), buf.shape[0], origin_days, _p(cols["ts"]), _p(cols["src"]),
                        _p(cols["dst"]), _p(cols["bytes"]), cap, ctypes.byref(n), ctypes.byref(bad))
    assert rc == 0
    return {k: v[:n.value].copy() for k, v in cols.items()}, int(bad.value)


def endpoints(base, plen):
    """Sorted elementary-interval boundaries B[m] and owner[m] (LPM row + 1,
    or 0 where no prefix covers the interval)."""
    base, plen, _ = _table(base, plen)
    P = base.shape[0]
    B = np.empty(2 * P + 1, np.uint32)
    own = np.empty(2 * P + 1, np.uint32)
    m = lib().or_endpoints(_p(base), _p(plen), P, _p(B), _p(own))
    assert m > 0
    return B[:m].copy(), own[:m].copy()
