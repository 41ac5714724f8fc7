"""Device-side fill of session columns (same values as ``sinetgen.sessions``).

Only the benchmark and the GPU tests use this, to materialise multi-billion
session days directly in HBM; any index can be regenerated on the host with
``sinetgen.sessions(wl, idx=...)`` for checking.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import (TS_DIURNAL, Workload, diurnal_table, lognormal_table)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.hip")
_LIB = os.path.join(_HERE, "libsinetgen.so")


class _Params(ctypes.Structure):
    _fields_ = [("n_total", ctypes.c_uint64), ("key", ctypes.c_uint64 * 6),
                ("ts_mode", ctypes.c_uint32), ("ts_span", ctypes.c_uint32),
                ("jitter", ctypes.c_uint32), ("t_origin", ctypes.c_uint32),
                ("in_thr", ctypes.c_uint32), ("n_prefix", ctypes.c_uint32)]


def build() -> str:
    tmp = _LIB + ".tmp"
    subprocess.check_call([
        os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "-O3", "-std=c++17", "-fPIC", "-shared",
        f"--offload-arch={os.environ.get('SINET_OFFLOAD_ARCH', 'gfx950')}",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None
_tables = {}


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise ImportError(f"{_LIB} is not built; run __graft_entry__.build()")
        _lib = ctypes.CDLL(_LIB)
        _lib.sinetgen_fill.argtypes = [ctypes.POINTER(_Params)] + [ctypes.c_void_p] * 4 + [
            ctypes.c_uint64, ctypes.c_uint64] + [ctypes.c_void_p] * 5
        _lib.sinetgen_fill.restype = ctypes.c_int
        _lib.sinetgen_watch.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]
        _lib.sinetgen_watch.restype = ctypes.c_int
    return _lib


def _dev_tables(wl: Workload, device):
    import torch
    key = (id(wl.pbase), wl.n_prefix, str(device), wl.ts_span if wl.ts_mode == TS_DIURNAL else 0)
    if key not in _tables:
        lt = torch.from_numpy(lognormal_table().view(np.int64)).to(device)
        qt = (torch.from_numpy(diurnal_table(wl.ts_span).view(np.int64)).to(device)
              if wl.ts_mode == TS_DIURNAL else None)
        pb = torch.from_numpy(wl.pbase.view(np.int32)).to(device) if wl.n_prefix else None
        pl = torch.from_numpy(wl.plen).to(device) if wl.n_prefix else None
        _tables[key] = (lt, qt, pb, pl, wl.pbase)  # keep pbase alive so id() stays unique
    return _tables[key]


def fill(wl: Workload, ts=None, src=None, dst=None, nbytes=None, i0: int = 0, n=None):
    """Write sessions [i0, i0 + n) of ``wl`` into device tensors (int32/int64
    storage reinterpreted as uint32/uint64); None skips a column."""
    import torch
    lib = _load()
    ref = next(t for t in (ts, src, dst, nbytes) if t is not None)
    n = ref.shape[0] if n is None else n
    lt, qt, pb, pl, _ = _dev_tables(wl, ref.device)
    p = _Params()
    p.n_total = wl.n
    for i, k in enumerate(wl.keys()):
        p.key[i] = k
    p.ts_mode, p.ts_span, p.jitter, p.t_origin = wl.ts_mode, wl.ts_span, wl.jitter, wl.t_origin
    p.in_thr, p.n_prefix = wl.in_thr, wl.n_prefix
    ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    stream = torch.cuda.current_stream(ref.device).cuda_stream
    rc = lib.sinetgen_fill(ctypes.byref(p), ptr(pb), ptr(pl), ptr(qt), ptr(lt), i0, n,
                           ptr(ts), ptr(src), ptr(dst), ptr(nbytes), ctypes.c_void_p(stream))
    if rc != 0:
        raise RuntimeError(f"sinetgen_fill failed ({rc})")


def watch_fill(wlist, src, dst, i0: int = 0):
    """Place the list's hosts into device columns holding sessions
    [i0, i0 + len) (the same values as ``sinetgen.watch_overlay``)."""
    import torch
    lib = _load()
    n = src.shape[0]
    addrs = torch.from_numpy(wlist.addrs.view(np.int32)).to(src.device)
    ks, kd = wlist.keys()
    stream = torch.cuda.current_stream(src.device).cuda_stream
    rc = lib.sinetgen_watch(ctypes.c_void_p(addrs.data_ptr()), wlist.n, ks, kd, wlist.thr, i0, n,
                            ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                            ctypes.c_void_p(stream))
    if rc != 0:
        raise RuntimeError(f"sinetgen_watch failed ({rc})")
    torch.cuda.current_stream(src.device).synchronize()  # addrs is freed on return


def alloc_and_fill(wl: Workload, device="cuda", columns=("ts", "src", "dst", "bytes")):
    """Fresh device columns for the whole workload."""
    import torch
    out = {}
    for c in columns:
        dt = torch.int64 if c == "bytes" else torch.int32
        out[c] = torch.empty(wl.n, dtype=dt, device=device)
    fill(wl, out.get("ts"), out.get("src"), out.get("dst"), out.get("bytes"))
    return out
