"""Python binding of libsinet (session discrimination + millisecond histogram
on MI355X).  Argument marshalling only: every step runs in the HIP library.

Device buffers are torch tensors used purely as memory: uint32 columns live
in int32 tensors, uint64 in int64 tensors, labels in uint8; the library
reinterprets them as unsigned.  Calls are enqueued on torch's current stream.
The library must be built (``__graft_entry__.build()``); importing this
package without it raises ImportError.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsinet.so")

OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_UNSUPPORTED = 0, 1, 2, 3, 4
EXTERNAL, EGRESS, INGRESS, INTERNAL = 0, 1, 2, 3
NO_INST = 0xFFFFFFFF
MLP_PARAMS = 49
KINDS = {"auto": 0, "scan": 1, "bsearch": 2, "trie": 3, "pla": 4, "mlp": 5}
KIND_NAMES = {v: k for k, v in KINDS.items()}
NO_INOUT_INDEX = 0x100
GLOBAL_BSEARCH = 0x200

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libsinet is not built ({LIB_PATH} missing): run __graft_entry__.build()")
_lib = ctypes.CDLL(LIB_PATH)

P = ctypes.c_void_p
U32, U64, I32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int


class Columns(ctypes.Structure):
    _fields_ = [("ts", P), ("src", P), ("dst", P), ("bytes", P), ("n", U64)]


class Window(ctypes.Structure):
    _fields_ = [("t0_ms", U32), ("width_ms", U32), ("n_bins", U32)]


class Hist(ctypes.Structure):
    _fields_ = [("count", P), ("bytes", P), ("dropped", P)]


class TableInfo(ctypes.Structure):
    _fields_ = [("kind", U32), ("inout_index", U32), ("n_prefix", U64), ("m", U64),
                ("device_bytes", U64),
                ("trained", U32), ("max_err", U32), ("segments", U32), ("pla_window", U32),
                ("fallbacks", U64)]


class TrainParams(ctypes.Structure):
    _fields_ = [("steps", U32), ("lr", ctypes.c_float), ("init", P), ("segments", U32),
                ("target_err", U32)]


class TrainReport(ctypes.Structure):
    _fields_ = [("loss_first", ctypes.c_float), ("loss_last", ctypes.c_float),
                ("max_err_untrained", U32), ("max_err", U32), ("train_ms", ctypes.c_double)]


class Tune(ctypes.Structure):
    _fields_ = [("block", U32), ("chunk", U32), ("grid", U32), ("reserved", U32)]


class Stream(ctypes.Structure):
    _fields_ = [("cols", Columns), ("table", P), ("win", Window), ("label", P), ("hist", Hist)]


class Timing(ctypes.Structure):
    _fields_ = [("lookup_ms", ctypes.c_double), ("stage1_ms", ctypes.c_double),
                ("index_ms", ctypes.c_double), ("stage2_ms", ctypes.c_double),
                ("far_ms", ctypes.c_double), ("calls", U64), ("stage1_launches", U64),
                ("window_calls", U64)]


def _sig(name, args, res=I32):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("sinet_status_string", [I32], ctypes.c_char_p)
_sig("sinet_last_error", [], ctypes.c_char_p)
_sig("sinet_version", [], ctypes.c_char_p)
_sig("sinet_table_create", [P, P, P, U64, I32, P, ctypes.POINTER(P)])
_sig("sinet_table_train", [P, ctypes.POINTER(TrainParams), P, ctypes.POINTER(TrainReport)])
_sig("sinet_table_info", [P, ctypes.POINTER(TableInfo)])
_sig("sinet_table_intervals", [P, P, P, U64])
_sig("sinet_table_get_model", [P, P, P, P, P, U32, P])
_sig("sinet_table_set_model", [P, P, P, P, P, U32, U32])
_sig("sinet_table_destroy", [P])
_sig("sinet_table_position", [P, P, U64, P, P])
_sig("sinet_discriminate", [P, P, P, U64, P, P, P, P])
_sig("sinet_label_runs", [P, U64, P, P, P])
_sig("sinet_histogram", [P, P, P, U64, ctypes.POINTER(Window), ctypes.POINTER(Hist), I32, P])
_sig("sinet_pipeline", [P, ctypes.POINTER(Columns), ctypes.POINTER(Window), P,
                        ctypes.POINTER(Hist), I32, P])
_sig("sinet_pipeline_noalloc", [P, ctypes.POINTER(Columns), ctypes.POINTER(Window), P,
                                ctypes.POINTER(Hist), I32, P])
_sig("sinet_watch_histogram", [P, ctypes.POINTER(Columns), ctypes.POINTER(Window), U32,
                               ctypes.POINTER(Hist), I32, P])
_sig("sinet_rebin", [P, U32, U32, U32, P, P])
_sig("sinet_parse_sessions", [P, U64, ctypes.c_int32, ctypes.POINTER(Columns), ctypes.POINTER(U64),
                              ctypes.POINTER(U64), P])
_sig("sinet_streamer_create", [U64, ctypes.POINTER(P)])
_sig("sinet_streamer_pipeline", [P, P, ctypes.POINTER(Columns), ctypes.POINTER(Window), P,
                                 ctypes.POINTER(Hist), I32, P])
_sig("sinet_streamer_destroy", [P])
_sig("sinet_mlp_loss_grad", [P, P, P, U64, P, P, P])
_sig("sinet_autotune", [P, U32, ctypes.c_char_p, P, ctypes.POINTER(Tune)])
_sig("sinet_batch_plan_create", [P, U32, ctypes.POINTER(Tune), P, ctypes.POINTER(P)])
_sig("sinet_batch_run", [P, P])
_sig("sinet_batch_plan_destroy", [P])
_sig("sinet_timing_enable", [I32])
_sig("sinet_timing_read", [ctypes.POINTER(Timing)])
_sig("sinet_set_reduce", [I32])


class SinetError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.sinet_last_error().decode()
        super().__init__(f"{where}: {_lib.sinet_status_string(status).decode()} ({msg})")


def _check(rc: int, where: str):
    if rc != OK:
        raise SinetError(rc, where)


def version() -> str:
    return _lib.sinet_version().decode()


def lib():
    return _lib


def _stream(device=None):
    import torch
    return P(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return None if t is None else P(t.data_ptr())


def _dev_check(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("device tensors must be CUDA (HIP) and contiguous")


def _sized(t, esize: int, numel: int, name: str):
    """A device buffer of at least numel elements of esize bytes (the kernels
    read or write exactly that many)."""
    if t is None:
        return
    _dev_check(t)
    if t.element_size() != esize:
        raise ValueError(f"{name}: elements of {esize} bytes expected, got {t.dtype}")
    if t.numel() < numel:
        raise ValueError(f"{name}: {numel} elements needed, {t.numel()} given")


def _check_hist(out, n_bins: int):
    if len(out) < 2:
        raise ValueError("out: (count, bytes[, dropped]) expected")
    _sized(out[0], 8, 4 * n_bins, "count")
    _sized(out[1], 8, 4 * n_bins, "bytes")
    if len(out) > 2:
        _sized(out[2], 8, 8, "dropped")


def _check_columns(n: int, ts=None, src=None, dst=None, nbytes=None):
    for t, es, name in ((ts, 4, "ts"), (src, 4, "src"), (dst, 4, "dst"), (nbytes, 8, "bytes")):
        if t is not None:
            _sized(t, es, n, name)
            if t.numel() != n:
                raise ValueError(f"{name}: {t.numel()} elements, the other columns have {n}")


class Table:
    """Device-resident prefix table (library-owned)."""

    def __init__(self, base, plen, inst=None, kind: str = "auto", inout_index: bool = True,
                 global_bsearch: bool = False):
        base = np.ascontiguousarray(base, dtype=np.uint32)
        plen = np.ascontiguousarray(plen, dtype=np.uint8)
        self._inst = None if inst is None else np.ascontiguousarray(inst, dtype=np.uint32)
        out = P()
        rc = _lib.sinet_table_create(base.ctypes.data_as(P), plen.ctypes.data_as(P),
                                     None if self._inst is None else self._inst.ctypes.data_as(P),
                                     base.shape[0],
                                     KINDS[kind] | (0 if inout_index else NO_INOUT_INDEX)
                                     | (GLOBAL_BSEARCH if global_bsearch else 0),
                                     _stream(), ctypes.byref(out))
        _check(rc, "sinet_table_create")
        self.handle = out
        self.n_prefix = base.shape[0]

    def train(self, steps: int = 0, lr: float = 0.0, init: Optional[Sequence[float]] = None,
              segments: int = 0, target_err: int = 0) -> TrainReport:
        prm = TrainParams()
        prm.steps, prm.lr, prm.segments, prm.target_err = steps, lr, segments, target_err
        buf = None
        if init is not None:
            buf = np.ascontiguousarray(init, dtype=np.float32)
            prm.init = buf.ctypes.data_as(P)
        rep = TrainReport()
        _check(_lib.sinet_table_train(self.handle, ctypes.byref(prm), _stream(), ctypes.byref(rep)),
               "sinet_table_train")
        return rep

    def get_model(self):
        """Saved model: ("mlp", params[49], max_err) or ("pla", (knot, c, g), max_err)."""
        inf = self.info()
        err = ctypes.c_uint32()
        if KIND_NAMES[inf.kind] == "mlp":
            prm = np.empty(MLP_PARAMS, np.float32)
            _check(_lib.sinet_table_get_model(self.handle, prm.ctypes.data_as(P), None, None, None,
                                              0, ctypes.byref(err)), "sinet_table_get_model")
            return "mlp", prm, err.value
        S = inf.segments
        knot, c, g = np.empty(S, np.uint32), np.empty(S, np.float32), np.empty(S, np.float32)
        _check(_lib.sinet_table_get_model(self.handle, None, knot.ctypes.data_as(P),
                                          c.ctypes.data_as(P), g.ctypes.data_as(P), S,
                                          ctypes.byref(err)), "sinet_table_get_model")
        return "pla", (knot, c, g), err.value

    def set_model(self, params=None, pla=None, max_err: Optional[int] = None):
        """Load a model; max_err None measures the bound on the GPU."""
        e = 0xFFFFFFFF if max_err is None else int(max_err)
        if params is not None:
            prm = np.ascontiguousarray(params, dtype=np.float32)
            _check(_lib.sinet_table_set_model(self.handle, prm.ctypes.data_as(P), None, None, None,
                                              0, e), "sinet_table_set_model")
        else:
            knot = np.ascontiguousarray(pla[0], dtype=np.uint32)
            c = np.ascontiguousarray(pla[1], dtype=np.float32)
            g = np.ascontiguousarray(pla[2], dtype=np.float32)
            _check(_lib.sinet_table_set_model(self.handle, None, knot.ctypes.data_as(P),
                                              c.ctypes.data_as(P), g.ctypes.data_as(P),
                                              knot.shape[0], e), "sinet_table_set_model")

    def info(self) -> TableInfo:
        inf = TableInfo()
        _check(_lib.sinet_table_info(self.handle, ctypes.byref(inf)), "sinet_table_info")
        return inf

    @property
    def kind(self) -> str:
        return KIND_NAMES[self.info().kind]

    def intervals(self):
        m = self.info().m
        B = np.empty(m, np.uint32)
        own = np.empty(m, np.uint32)
        _check(_lib.sinet_table_intervals(self.handle, B.ctypes.data_as(P), own.ctypes.data_as(P), m),
               "sinet_table_intervals")
        return B, own

    def position(self, addr, out=None):
        import torch
        _dev_check(addr)
        _sized(addr, 4, addr.numel(), "addr")
        if out is None:
            out = torch.empty_like(addr, dtype=torch.int32)
        _sized(out, 4, addr.numel(), "out")
        _check(_lib.sinet_table_position(self.handle, _ptr(addr), addr.shape[0], _ptr(out),
                                         _stream(addr.device)), "sinet_table_position")
        return out

    def close(self):
        if getattr(self, "handle", None):
            _lib.sinet_table_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _opt_out(arg, n, dtype, device):
    """True: allocate; False/None: not stored; a tensor: written in place."""
    import torch
    if arg is True:
        return torch.empty(n, dtype=dtype, device=device)
    if arg is None or arg is False:
        return None
    _dev_check(arg)
    return arg


def discriminate(table: Table, src, dst, label=True, src_inst=False, dst_inst=False):
    """Labels (uint8) and optional institution ids (int32 storage of uint32)."""
    import torch
    _dev_check(src, dst)
    n = src.numel()
    _check_columns(n, src=src, dst=dst)
    dev = src.device
    lab = _opt_out(label, n, torch.uint8, dev)
    si = _opt_out(src_inst, n, torch.int32, dev)
    di = _opt_out(dst_inst, n, torch.int32, dev)
    _sized(lab, 1, n, "label")
    _sized(si, 4, n, "src_inst")
    _sized(di, 4, n, "dst_inst")
    _check(_lib.sinet_discriminate(table.handle, _ptr(src), _ptr(dst), n, _ptr(lab), _ptr(si),
                                   _ptr(di), _stream(dev)), "sinet_discriminate")
    return lab, si, di


def label_runs(label, idx=None, totals=None):
    """Session indices partitioned by label, stably: (idx int32 storage of
    uint32 [n], totals int64 storage of uint64 [4]).  label: device uint8."""
    import torch
    _dev_check(label)
    n = label.numel()
    _sized(label, 1, n, "label")
    dev = label.device
    if idx is None:
        idx = torch.empty(n, dtype=torch.int32, device=dev)
    if totals is None:
        totals = torch.empty(4, dtype=torch.int64, device=dev)
    _sized(idx, 4, n, "idx")
    _sized(totals, 8, 4, "totals")
    _check(_lib.sinet_label_runs(_ptr(label), n, _ptr(idx), _ptr(totals), _stream(dev)),
           "sinet_label_runs")
    return idx, totals


def new_hist(n_bins: int, device="cuda"):
    import torch
    return (torch.empty((4, n_bins), dtype=torch.int64, device=device),
            torch.empty((4, n_bins), dtype=torch.int64, device=device),
            torch.empty((4, 2), dtype=torch.int64, device=device))


def _hist_struct(out):
    h = Hist()
    h.count, h.bytes = _ptr(out[0]), _ptr(out[1])
    h.dropped = _ptr(out[2]) if len(out) > 2 and out[2] is not None else None
    return h


def histogram(ts, nbytes, label, t0: int, width: int, n_bins: int, out=None,
              accumulate: bool = False):
    _dev_check(ts, nbytes, label)
    n = ts.numel()
    _check_columns(n, ts=ts, nbytes=nbytes)
    _sized(label, 1, n, "label")
    out = new_hist(n_bins, ts.device) if out is None else out
    _check_hist(out, n_bins)
    w = Window(t0, width, n_bins)
    h = _hist_struct(out)
    _check(_lib.sinet_histogram(_ptr(ts), _ptr(nbytes), _ptr(label), n, ctypes.byref(w),
                                ctypes.byref(h), int(accumulate), _stream(ts.device)),
           "sinet_histogram")
    return out


def pipeline(table: Table, ts, src, dst, nbytes, t0: int, width: int, n_bins: int, label=True,
             out=None, accumulate: bool = False):
    """Fused discrimination + histogram.  Returns (label or None, (count, bytes, dropped))."""
    import torch
    _dev_check(ts, src, dst, nbytes)
    n = ts.numel()
    _check_columns(n, ts, src, dst, nbytes)
    lab = _opt_out(label, n, torch.uint8, ts.device)
    _sized(lab, 1, n, "label")
    out = new_hist(n_bins, ts.device) if out is None else out
    _check_hist(out, n_bins)
    c = Columns(_ptr(ts), _ptr(src), _ptr(dst), _ptr(nbytes), n)
    w = Window(t0, width, n_bins)
    h = _hist_struct(out)
    _check(_lib.sinet_pipeline(table.handle, ctypes.byref(c), ctypes.byref(w), _ptr(lab),
                               ctypes.byref(h), int(accumulate), _stream(ts.device)),
           "sinet_pipeline")
    return lab, out


def pipeline_noalloc(table: Table, ts, src, dst, nbytes, t0: int, width: int, n_bins: int, label,
                     out, accumulate: bool = False):
    """sinet_pipeline_noalloc: the pipeline with the library's static device
    workspace (at most 2^25 sessions per call).  The outputs are the
    caller's: `label` a uint8 tensor of n or None, `out` (count, bytes,
    dropped); nothing is allocated here either."""
    _dev_check(ts, src, dst, nbytes)
    n = ts.numel()
    _check_columns(n, ts, src, dst, nbytes)
    if label is not None:
        _sized(label, 1, n, "label")
    _check_hist(out, n_bins)
    c = Columns(_ptr(ts), _ptr(src), _ptr(dst), _ptr(nbytes), n)
    w = Window(t0, width, n_bins)
    h = _hist_struct(out)
    _check(_lib.sinet_pipeline_noalloc(table.handle, ctypes.byref(c), ctypes.byref(w),
                                       _ptr(label) if label is not None else None, ctypes.byref(h),
                                       int(accumulate), _stream(ts.device)),
           "sinet_pipeline_noalloc")
    return label, out


WATCH_SRC, WATCH_DST = 0, 1


def new_watch_hist(n_keys: int, n_bins: int, device="cuda"):
    import torch
    return (torch.empty((2, n_keys, n_bins), dtype=torch.int64, device=device),
            torch.empty((2, n_keys, n_bins), dtype=torch.int64, device=device),
            torch.empty((2, 2), dtype=torch.int64, device=device))


def watch_histogram(wlist: Table, ts, src, dst, nbytes, t0: int, width: int, n_bins: int,
                    n_keys: int, out=None, accumulate: bool = False):
    """Watch-list histograms: (count[2, n_keys, n_bins], bytes[2, n_keys, n_bins],
    dropped[2, 2]); direction WATCH_SRC counts sessions whose source matches
    the list, WATCH_DST those whose destination does, keyed by the list
    table's inst ids."""
    _dev_check(ts, src, dst, nbytes)
    n = ts.numel()
    _check_columns(n, ts, src, dst, nbytes)
    out = new_watch_hist(n_keys, n_bins, ts.device) if out is None else out
    if len(out) < 2:
        raise ValueError("out: (count, bytes[, dropped]) expected")
    _sized(out[0], 8, 2 * n_keys * n_bins, "count")
    _sized(out[1], 8, 2 * n_keys * n_bins, "bytes")
    if len(out) > 2:
        _sized(out[2], 8, 4, "dropped")
    c = Columns(_ptr(ts), _ptr(src), _ptr(dst), _ptr(nbytes), n)
    w = Window(t0, width, n_bins)
    h = _hist_struct(out)
    _check(_lib.sinet_watch_histogram(wlist.handle, ctypes.byref(c), ctypes.byref(w), n_keys,
                                      ctypes.byref(h), int(accumulate), _stream(ts.device)),
           "sinet_watch_histogram")
    return out


def rebin(h, factor: int, out=None):
    """Coarser frames of a [..., n_bins] int64 (uint64) device histogram:
    every group of ``factor`` consecutive bins summed; returns [..., n_out]."""
    import torch
    _dev_check(h)
    if h.element_size() != 8 or h.dim() < 1:
        raise ValueError("h: a [..., n_bins] tensor of 8-byte elements expected")
    n_bins = h.shape[-1]
    rows = h.numel() // n_bins if n_bins else 0
    n_out = -(-n_bins // factor) if factor > 0 else 0
    if out is None:
        out = torch.empty(tuple(h.shape[:-1]) + (n_out,), dtype=h.dtype, device=h.device)
    _dev_check(out)
    _sized(out, 8, rows * n_out, "out")
    _check(_lib.sinet_rebin(_ptr(h), rows, n_bins, factor, _ptr(out), _stream(h.device)),
           "sinet_rebin")
    return out


def parse_sessions(text, origin_days: int, capacity: Optional[int] = None):
    """Session text (a uint8 device tensor, one Table 1 record per line) to
    columns: (dict of ts/src/dst int32 and bytes int64 device tensors of the
    lines' count, number of bad lines)."""
    import torch
    _dev_check(text)
    if text.element_size() != 1:
        raise ValueError("text: a uint8 (or int8) device tensor expected")
    n_bytes = text.numel()
    cap = n_bytes // 64 + 16 if capacity is None else capacity
    for _ in range(2):
        cols = {"ts": torch.empty(cap, dtype=torch.int32, device=text.device),
                "src": torch.empty(cap, dtype=torch.int32, device=text.device),
                "dst": torch.empty(cap, dtype=torch.int32, device=text.device),
                "bytes": torch.empty(cap, dtype=torch.int64, device=text.device)}
        c = Columns(_ptr(cols["ts"]), _ptr(cols["src"]), _ptr(cols["dst"]), _ptr(cols["bytes"]), cap)
        n_lines, n_bad = U64(0), U64(0)
        st = _lib.sinet_parse_sessions(_ptr(text), n_bytes, origin_days, ctypes.byref(c),
                                       ctypes.byref(n_lines), ctypes.byref(n_bad),
                                       _stream(text.device))
        if st == ERR_INVALID_ARG and n_lines.value > cap and capacity is None:
            cap = n_lines.value  # every line counted: the second call fits
            continue
        _check(st, "sinet_parse_sessions")
        n = n_lines.value
        return {k: v[:n] for k, v in cols.items()}, n_bad.value
    raise SinetError(ERR_INVALID_ARG, "sinet_parse_sessions")


def _host_ptr(a, esize: int, n: int, name: str):
    """Address of a contiguous host array (numpy, or a CPU torch tensor,
    pinned or not) of at least n elements of esize bytes."""
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"] or a.itemsize != esize or a.size < n:
            raise ValueError(f"{name}: contiguous array of {n} {esize}-byte elements expected")
        return P(a.ctypes.data)
    if getattr(a, "is_cuda", True) or not a.is_contiguous() or a.element_size() != esize \
            or a.numel() < n:
        raise ValueError(f"{name}: contiguous host tensor of {n} {esize}-byte elements expected")
    return P(a.data_ptr())


class Streamer:
    """Out-of-core pipeline: columns in host memory streamed through two
    device staging slots of `chunk` sessions each (see sinet_streamer_*)."""

    def __init__(self, chunk: int = 64 << 20):
        out = P()
        _check(_lib.sinet_streamer_create(chunk, ctypes.byref(out)), "sinet_streamer_create")
        self.handle = out
        self.chunk = chunk

    def pipeline(self, table: Table, ts, src, dst, nbytes, t0: int, width: int, n_bins: int,
                 label=True, out=None, accumulate: bool = False, device="cuda"):
        """Host columns (numpy or CPU tensors) -> (host labels or None, device histogram)."""
        n = len(ts)
        c = Columns(_host_ptr(ts, 4, n, "ts"), _host_ptr(src, 4, n, "src"),
                    _host_ptr(dst, 4, n, "dst"), _host_ptr(nbytes, 8, n, "bytes"), n)
        for a, name in ((src, "src"), (dst, "dst"), (nbytes, "bytes")):
            if len(a) != n:
                raise ValueError(f"{name}: {len(a)} elements, ts has {n}")
        if label is True:
            lab = np.empty(n, np.uint8)
        elif label is None or label is False:
            lab = None
        else:
            lab = label
        lp = None if lab is None else _host_ptr(lab, 1, n, "label")
        out = new_hist(n_bins, device) if out is None else out
        _check_hist(out, n_bins)
        w = Window(t0, width, n_bins)
        h = _hist_struct(out)
        _check(_lib.sinet_streamer_pipeline(self.handle, table.handle, ctypes.byref(c),
                                            ctypes.byref(w), lp, ctypes.byref(h), int(accumulate),
                                            _stream(out[0].device)), "sinet_streamer_pipeline")
        return lab, out

    def close(self):
        if getattr(self, "handle", None):
            _lib.sinet_streamer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_loss_grad(params, x, y):
    """(loss[1], grad[49]) float32 device tensors."""
    import torch
    _dev_check(params, x, y)
    _sized(params, 4, MLP_PARAMS, "params")
    if x.element_size() != 4 or y.element_size() != 4 or y.numel() != x.numel():
        raise ValueError("x and y: float32 of the same length expected")
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
    _check(_lib.sinet_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(y), x.shape[0], _ptr(loss),
                                    _ptr(grad), _stream(x.device)), "sinet_mlp_loss_grad")
    return loss, grad


class BatchStream:
    """One stream of a batch: columns, table, window, outputs (device tensors)."""

    def __init__(self, table: Table, ts, src, dst, nbytes, t0, width, n_bins, label=None, out=None):
        _dev_check(ts, src, dst, nbytes, label)
        n = ts.numel()
        _check_columns(n, ts, src, dst, nbytes)
        _sized(label, 1, n, "label")
        if out is None:
            raise ValueError("out: a (count, bytes[, dropped]) histogram is required")
        _check_hist(out, n_bins)
        self.table, self.ts, self.src, self.dst, self.nbytes = table, ts, src, dst, nbytes
        self.t0, self.width, self.n_bins = t0, width, n_bins
        self.label = label
        self.out = out

    def struct(self) -> Stream:
        s = Stream()
        s.cols = Columns(_ptr(self.ts), _ptr(self.src), _ptr(self.dst), _ptr(self.nbytes),
                         self.ts.shape[0])
        s.table = self.table.handle
        s.win = Window(self.t0, self.width, self.n_bins)
        s.label = _ptr(self.label)
        s.hist = _hist_struct(self.out)
        return s


def _streams_array(streams):
    arr = (Stream * len(streams))()
    for i, s in enumerate(streams):
        arr[i] = s.struct()
    return arr


def autotune(streams, cache_path: Optional[str] = None) -> Tune:
    arr = _streams_array(streams)
    t = Tune()
    _check(_lib.sinet_autotune(arr, len(streams), None if cache_path is None else cache_path.encode(),
                               _stream(), ctypes.byref(t)), "sinet_autotune")
    return t


class BatchPlan:
    def __init__(self, streams, tune: Optional[Tune] = None):
        self.streams = list(streams)   # keeps the buffers alive
        arr = _streams_array(self.streams)
        out = P()
        _check(_lib.sinet_batch_plan_create(arr, len(self.streams),
                                            None if tune is None else ctypes.byref(tune),
                                            _stream(), ctypes.byref(out)),
               "sinet_batch_plan_create")
        self.handle = out

    def run(self):
        _check(_lib.sinet_batch_run(self.handle, _stream()), "sinet_batch_run")

    def close(self):
        if getattr(self, "handle", None):
            _lib.sinet_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def timing_enable(on: bool = True):
    """Start (clearing earlier figures) or stop phase timing of histogram and
    pipeline calls."""
    _check(_lib.sinet_timing_enable(int(bool(on))), "sinet_timing_enable")


def timing_read() -> dict:
    """Device ms per phase summed over the calls timed since timing_enable."""
    t = Timing()
    _check(_lib.sinet_timing_read(ctypes.byref(t)), "sinet_timing_read")
    return {name: getattr(t, name) for name, _ in Timing._fields_}


REDUCES = {"auto": 0, "records": 1, "window": 2}


def set_reduce(mode: str = "auto"):
    """Reduce of later histogram / pipeline calls: "records" (two-stage
    partition into 4-byte records), "window" (sliding window of bins in LDS
    over labelled sessions) or "auto" (window from 2^28 sessions on)."""
    if mode not in REDUCES:
        raise ValueError(f"reduce must be one of {sorted(REDUCES)}")
    _check(_lib.sinet_set_reduce(REDUCES[mode]), "sinet_set_reduce")


# host <-> device helpers for uint32/uint64 data held in signed tensors
def to_device_u32(a, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(device)


def to_device_u64(a, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to(device)


def to_host_u32(t):
    return t.cpu().numpy().view(np.uint32)


def to_host_u64(t):
    return t.cpu().numpy().view(np.uint64)
