"""CPU oracle (test infrastructure only): ctypes binding of ewah_oracle.c.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  The GPU library never uses it.

Functions follow the paper's definitions:
  decode     -- EWAH stream -> uncompressed words (Section 3.1; layout of the
                marker word as adopted in ewah_oracle.c)
  encode     -- uncompressed words -> canonical EWAH stream (rules C1-C4)
  threshold  -- ScanCount T-of-N threshold (Section 2 definition, Section 5.1
                method), returns the canonical EWAH result and the count
                histogram
  symmetric  -- the same counting with any function of the count (Sections 2,
                3.2 and 5.1), returns the canonical EWAH result
  opt_threshold -- largest T whose result has at least K rows (Section 3.3),
                read off the count histogram, and that result
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libewah_oracle.so")
SRC_PATH = os.path.join(_HERE, "ewah_oracle.c")

OK, EINVAL, EFORMAT, ENOMEM, ENOSPC = 0, -1, -2, -3, -4

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, -O2, no vector intrinsics)."""
    if force or not os.path.exists(LIB_PATH):
        import subprocess
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-Wall", "-o", tmp, SRC_PATH])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
        L.orc_decode.restype = ctypes.c_int
        L.orc_decode.argtypes = [vp, u64, u64, vp]
        L.orc_encode.restype = ctypes.c_int
        L.orc_encode.argtypes = [vp, u64, vp, u64, vp]
        L.orc_threshold.restype = ctypes.c_int
        L.orc_threshold.argtypes = [vp, vp, u32, u64, u32, vp, u64, vp, vp]
        L.orc_symmetric.restype = ctypes.c_int
        L.orc_symmetric.argtypes = [vp, vp, u32, u64, vp, vp, u64, vp]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def decode(words, n_bits: int) -> np.ndarray:
    w = _u64(words)
    U = (n_bits + 63) // 64
    dense = np.zeros(max(U, 1), dtype=np.uint64)
    rc = _load().orc_decode(w.ctypes.data if len(w) else None, len(w), n_bits, dense.ctypes.data)
    if rc != OK:
        raise OracleError(rc, "decode")
    return dense[:U]


def encode(dense, n_bits: int) -> np.ndarray:
    d = _u64(dense)
    U = (n_bits + 63) // 64
    assert len(d) == U
    cap = U + 1
    out = np.zeros(max(cap, 1), dtype=np.uint64)
    n = ctypes.c_uint64(0)
    rc = _load().orc_encode(d.ctypes.data if U else None, n_bits, out.ctypes.data, cap, ctypes.byref(n))
    if rc != OK:
        raise OracleError(rc, "encode")
    return out[: n.value].copy()


def threshold(streams, n_bits: int, T: int, want_hist: bool = True):
    """Returns (canonical EWAH words of the result, count histogram or None)."""
    arrs = [_u64(s) for s in streams]
    N = len(arrs)
    ptrs = (ctypes.c_void_p * max(N, 1))(*[a.ctypes.data for a in arrs])
    nws = np.array([len(a) for a in arrs] or [0], dtype=np.uint64)
    U = (n_bits + 63) // 64
    cap = U + 1
    out = np.zeros(max(cap, 1), dtype=np.uint64)
    n = ctypes.c_uint64(0)
    hist = np.zeros(N + 1, dtype=np.uint64) if want_hist else None
    rc = _load().orc_threshold(ptrs, nws.ctypes.data, N, n_bits, T, out.ctypes.data, cap, ctypes.byref(n),
                               hist.ctypes.data if want_hist else None)
    if rc != OK:
        raise OracleError(rc, "threshold")
    return out[: n.value].copy(), hist


def symmetric(streams, n_bits: int, f):
    """Canonical EWAH words of the rows whose count c (inputs with the row set) has f[c] true;
    f has len(streams) + 1 entries."""
    arrs = [_u64(s) for s in streams]
    N = len(arrs)
    if len(f) != N + 1:
        raise ValueError("f needs N + 1 entries")
    ptrs = (ctypes.c_void_p * max(N, 1))(*[a.ctypes.data for a in arrs])
    nws = np.array([len(a) for a in arrs] or [0], dtype=np.uint64)
    tab = np.array([1 if v else 0 for v in f], dtype=np.uint8)
    U = (n_bits + 63) // 64
    cap = U + 1
    out = np.zeros(max(cap, 1), dtype=np.uint64)
    n = ctypes.c_uint64(0)
    rc = _load().orc_symmetric(ptrs, nws.ctypes.data, N, n_bits, tab.ctypes.data, out.ctypes.data, cap,
                               ctypes.byref(n))
    if rc != OK:
        raise OracleError(rc, "symmetric")
    return out[: n.value].copy()


def opt_threshold(streams, n_bits: int, K: int):
    """(T, canonical EWAH words of the T-of-N result) for the largest T in [0, N] whose result has at
    least K rows (Section 3.3; K = 1 is the largest row count, as ScanCount reads it off its
    counters, Section 5.1).  The row counts come from the count histogram h: |result(T)| is the sum
    of h[c] over c >= T."""
    N = len(streams)
    if not 1 <= K <= n_bits:
        raise ValueError("K must be in [1, n_bits]")
    _, hist = threshold(streams, n_bits, N + 1, want_hist=True)
    best, above = 0, 0
    for T in range(N, -1, -1):
        above += int(hist[T])
        if above >= K:
            best = T
            break
    out, _ = threshold(streams, n_bits, best, want_hist=False)
    return best, out
