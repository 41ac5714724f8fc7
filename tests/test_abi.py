"""The C-ABI library loads, exports every entry point its header declares,
and rejects bad arguments on the host before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sinet.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sinet_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("sinet_discriminate", "sinet_histogram", "sinet_pipeline", "sinet_table_create",
                 "sinet_table_train", "sinet_batch_plan_create", "sinet_batch_run",
                 "sinet_autotune", "sinet_mlp_loss_grad", "sinet_watch_histogram", "sinet_rebin",
                 "sinet_parse_sessions", "sinet_streamer_pipeline"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2106_12863_amd as sinet
    lib = sinet.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert "gfx950" in sinet.version()


def test_host_side_argument_errors():
    import paper_2106_12863_amd as sinet
    lib = sinet.lib()
    P = ctypes.c_void_p
    out = P()
    base = np.array([0x0A000000], np.uint32)
    plen = np.array([8], np.uint8)
    bad_len = np.array([33], np.uint8)
    inst_bad = np.array([0xFFFFFFFF], np.uint32)
    bp, lp = base.ctypes.data_as(P), plen.ctypes.data_as(P)
    assert lib.sinet_table_create(None, lp, None, 1, 0, None, ctypes.byref(out)) == sinet.ERR_INVALID_ARG
    assert lib.sinet_table_create(bp, lp, None, 0, 0, None, ctypes.byref(out)) == sinet.ERR_INVALID_ARG
    assert lib.sinet_table_create(bp, bad_len.ctypes.data_as(P), None, 1, 0, None,
                                  ctypes.byref(out)) == sinet.ERR_INVALID_ARG
    assert b"above 32" in lib.sinet_last_error()
    assert lib.sinet_table_create(bp, lp, inst_bad.ctypes.data_as(P), 1, 0, None,
                                  ctypes.byref(out)) == sinet.ERR_INVALID_ARG
    assert lib.sinet_table_create(bp, lp, None, 1, 9, None, ctypes.byref(out)) == sinet.ERR_INVALID_ARG
    big = np.zeros(1025, np.uint32)
    bigl = np.zeros(1025, np.uint8)
    assert lib.sinet_table_create(big.ctypes.data_as(P), bigl.ctypes.data_as(P), None, 1025, 1, None,
                                  ctypes.byref(out)) == sinet.ERR_INVALID_ARG
    assert lib.sinet_table_create(bp, lp, None, (1 << 22) + 1, 2, None,
                                  ctypes.byref(out)) == sinet.ERR_INVALID_ARG
    w0 = sinet.Window(0, 0, 10)
    nb0 = sinet.Window(0, 1, 0)
    h = sinet.Hist(P(16), P(16), None)
    for w in (w0, nb0):
        assert lib.sinet_histogram(P(16), P(16), P(16), 4, ctypes.byref(w), ctypes.byref(h), 0,
                                   None) == sinet.ERR_INVALID_ARG
    assert lib.sinet_histogram(P(16), P(16), P(16), 4, None, ctypes.byref(h), 0,
                               None) == sinet.ERR_INVALID_ARG
    cols = sinet.Columns(P(16), P(16), P(16), P(16), 4)
    w = sinet.Window(0, 1, 10)
    assert lib.sinet_pipeline(None, ctypes.byref(cols), ctypes.byref(w), None, ctypes.byref(h), 0,
                              None) == sinet.ERR_INVALID_ARG
    assert lib.sinet_discriminate(None, P(16), P(16), 4, P(16), None, None, None) == sinet.ERR_INVALID_ARG
    assert lib.sinet_label_runs(P(16), 4, P(16), None, None) == sinet.ERR_INVALID_ARG
    assert lib.sinet_label_runs(None, 4, P(16), P(16), None) == sinet.ERR_INVALID_ARG
    assert lib.sinet_label_runs(P(16), 1 << 32, P(16), P(16), None) == sinet.ERR_UNSUPPORTED
    assert lib.sinet_watch_histogram(None, ctypes.byref(cols), ctypes.byref(w), 3, ctypes.byref(h), 0,
                                     None) == sinet.ERR_INVALID_ARG
    assert lib.sinet_rebin(None, 4, 10, 2, P(16), None) == sinet.ERR_INVALID_ARG
    assert lib.sinet_rebin(P(16), 4, 10, 0, P(16), None) == sinet.ERR_INVALID_ARG
    n_lines, n_bad = ctypes.c_uint64(0), ctypes.c_uint64(0)
    assert lib.sinet_parse_sessions(P(16), 10, 0, None, ctypes.byref(n_lines), ctypes.byref(n_bad),
                                    None) == sinet.ERR_INVALID_ARG
    empty_cols = sinet.Columns(None, None, None, None, 4)
    assert lib.sinet_parse_sessions(P(16), 10, 0, ctypes.byref(empty_cols), ctypes.byref(n_lines),
                                    ctypes.byref(n_bad), None) == sinet.ERR_INVALID_ARG
    assert lib.sinet_streamer_create(0, ctypes.byref(out)) == sinet.ERR_INVALID_ARG
    assert lib.sinet_streamer_create((1 << 31) + 1, ctypes.byref(out)) == sinet.ERR_INVALID_ARG
    assert lib.sinet_streamer_pipeline(None, None, None, None, None, None, 0, None) == sinet.ERR_INVALID_ARG
    assert lib.sinet_mlp_loss_grad(None, P(16), P(16), 4, P(16), P(16), None) == sinet.ERR_INVALID_ARG
    assert lib.sinet_batch_plan_create(None, 0, None, None, ctypes.byref(out)) != sinet.OK
    assert lib.sinet_status_string(2) == b"out of device memory"
