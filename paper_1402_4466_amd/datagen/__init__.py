"""Seeded synthetic EWAH bitmaps and query sets.

Input generation only: nothing here computes a threshold, decodes a stream or
encodes a result.  The generators are shared by the CPU oracle tests and the
GPU path so that both sides read identical bytes.

The configurations stand in for the paper's real datasets (Section 7.2, Table
real-data-char), which are not available: they reproduce the workload shapes
(log-uniform N, skewed densities, clustered runs, long empty stretches) with
synthetic bitmaps.  The recipe of each configuration is written out in the
function that builds it.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libewahgen.so")
_lib = None

SEED_BASE = 14024466  # configuration k uses SEED_BASE + k


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"generator library not built: {_LIB_PATH} (run __graft_entry__.build())")
        L = ctypes.CDLL(_LIB_PATH)
        u64, i32, dbl = ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        vp = ctypes.c_void_p
        L.ewahgen_key.restype = u64
        L.ewahgen_key.argtypes = [u64, u64]
        L.ewahgen_bitmap.restype = u64
        L.ewahgen_bitmap.argtypes = [i32, dbl, dbl, u64, u64, i32, vp, u64]
        L.ewahgen_batch.restype = None
        L.ewahgen_batch.argtypes = [i32, vp, vp, vp, u64, vp, i32, vp, u64, vp]
        L.ewahgen_queries.restype = None
        L.ewahgen_queries.argtypes = [u64, i32, i32, i32, i32, vp, vp, vp]
        L.ewahgen_uniform.restype = None
        L.ewahgen_uniform.argtypes = [u64, i32, vp]
        _lib = L
    return _lib


def key(seed: int, stream_id: int) -> int:
    return int(lib().ewahgen_key(seed & (2**64 - 1), stream_id & (2**64 - 1)))


def uniform(key_: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    lib().ewahgen_uniform(key_, count, out.ctypes.data)
    return out


IID, MARKOV = 0, 1


def _cap(n_bits: int, noncanon: bool) -> int:
    u = (n_bits + 63) // 64
    return 2 * u + 64 if noncanon else u + 1


def bitmap(model: int, a: float, b: float, n_bits: int, key_: int, noncanon: bool = False) -> np.ndarray:
    """One EWAH stream (np.uint64)."""
    cap = _cap(n_bits, noncanon)
    buf = np.empty(max(cap, 1), dtype=np.uint64)
    n = lib().ewahgen_bitmap(model, a, b, n_bits, key_, 1 if noncanon else 0, buf.ctypes.data, cap)
    if n == 2**64 - 1:
        raise RuntimeError("generator buffer too small")
    return buf[:n].copy()


def bitmaps(models, a, b, n_bits: int, keys, noncanon: bool = False, chunk: int = 256) -> list[np.ndarray]:
    """Many EWAH streams generated in parallel (OpenMP inside the library)."""
    count = len(keys)
    models = np.ascontiguousarray(np.broadcast_to(np.asarray(models, dtype=np.int32), (count,)))
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (count,)))
    b = np.ascontiguousarray(np.broadcast_to(np.asarray(b, dtype=np.float64), (count,)))
    keys = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64))
    cap = _cap(n_bits, noncanon)
    out: list[np.ndarray] = []
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        m = e - s
        buf = np.empty((m, cap), dtype=np.uint64)
        nout = np.empty(m, dtype=np.uint64)
        lib().ewahgen_batch(m, models[s:e].ctypes.data, a[s:e].ctypes.data, b[s:e].ctypes.data, n_bits,
                            keys[s:e].ctypes.data, 1 if noncanon else 0, buf.ctypes.data, cap, nout.ctypes.data)
        for i in range(m):
            n = int(nout[i])
            if n == 2**64 - 1:
                raise RuntimeError("generator buffer too small")
            out.append(buf[i, :n].copy())
        del buf
    return out


@dataclass
class Query:
    idx: np.ndarray   # indices into a bitmap list / pool (uint32)
    T: int


@dataclass
class Workload:
    """A set of bitmaps over n_bits rows plus threshold queries over them."""
    name: str
    n_bits: int
    streams: list          # list[np.ndarray uint64]
    queries: list          # list[Query]
    meta: dict = field(default_factory=dict)

    @property
    def n_words(self) -> np.ndarray:
        return np.array([len(s) for s in self.streams], dtype=np.int64)

    def input_words(self, q: Query) -> int:
        nw = self.n_words
        return int(nw[q.idx].sum())


def queries(seed: int, n_queries: int, n_pool: int, nmin: int, nmax: int) -> list[Query]:
    nout = np.empty(n_queries, dtype=np.uint32)
    tout = np.empty(n_queries, dtype=np.uint32)
    idx = np.empty((n_queries, nmax), dtype=np.uint32)
    lib().ewahgen_queries(seed, n_queries, n_pool, nmin, nmax, nout.ctypes.data, tout.ctypes.data, idx.ctypes.data)
    return [Query(idx[q, : nout[q]].copy(), int(tout[q])) for q in range(n_queries)]


# ------------------------------------------------------------------ configs

def config1() -> Workload:
    """N=8 bitmaps over 2^16 rows, each bit iid Bernoulli(0.1); one query, T=4."""
    seed = SEED_BASE + 1
    n_bits = 1 << 16
    keys = [key(seed, k) for k in range(8)]
    streams = bitmaps(IID, 0.1, 0.0, n_bits, keys)
    return Workload("c1_n8_r2^16_iid0.1", n_bits, streams, [Query(np.arange(8, dtype=np.uint32), 4)])


def config2(n_bits: int = 1 << 24, n: int = 64) -> Workload:
    """N=64 bitmaps over 2^24 rows, two-state Markov bits: 1-runs geometric with
    mean 32 bits, 0-runs geometric with mean 512 bits, first state from the
    stationary law; queries T in {2, 32, 63}."""
    seed = SEED_BASE + 2
    keys = [key(seed, k) for k in range(n)]
    streams = bitmaps(MARKOV, 32.0, 512.0, n_bits, keys)
    idx = np.arange(n, dtype=np.uint32)
    ts = [t for t in (2, 32, 63) if t <= n]
    return Workload(f"c2_n{n}_r{n_bits}_markov32_512", n_bits, streams, [Query(idx, t) for t in ts])


def config3(n_bits: int = 1 << 26, n: int = 1024) -> Workload:
    """N=1024 bitmaps over 2^26 rows; bitmap k (k = 1..N) has density d_k = 0.3/k,
    produced by the two-state Markov model with mean 1-run 32 bits and mean
    0-run 32 (1 - d_k) / d_k bits (so the stationary density is d_k);
    queries T in {8, 128, 512}."""
    seed = SEED_BASE + 3
    keys = [key(seed, k) for k in range(n)]
    d = 0.3 / np.arange(1, n + 1, dtype=np.float64)
    m1 = np.full(n, 32.0)
    m0 = 32.0 * (1.0 - d) / d
    streams = bitmaps(MARKOV, m1, m0, n_bits, keys)
    idx = np.arange(n, dtype=np.uint32)
    ts = [t for t in (8, 128, 512) if t <= n]
    return Workload(f"c3_n{n}_r{n_bits}_zipf0.3", n_bits, streams, [Query(idx, t) for t in ts])


def pool_densities(n_pool: int, seed: int | None = None) -> np.ndarray:
    """Densities log-uniform in [1e-4, 0.3]."""
    seed = SEED_BASE + 4 if seed is None else seed
    u = uniform(key(seed, 0xFFFF_FFFF), n_pool)
    lo, hi = np.log(1e-4), np.log(0.3)
    return np.exp(lo + (hi - lo) * (1.0 - u))


def config4_pool(n_pool: int = 10_000, n_bits: int = 1 << 22) -> tuple[list, np.ndarray]:
    """Pool of EWAH bitmaps over 2^22 rows, each bit iid Bernoulli(d) with d
    log-uniform in [1e-4, 0.3] per bitmap."""
    seed = SEED_BASE + 4
    d = pool_densities(n_pool, seed)
    keys = [key(seed, k) for k in range(n_pool)]
    return bitmaps(IID, d, 0.0, n_bits, keys), d


def config4(n_pool: int = 10_000, n_queries: int = 4096, n_bits: int = 1 << 22, nmax: int = 256,
            pool=None) -> Workload:
    """4,096 queries over the pool: N uniform in [2, 256] distinct bitmaps,
    T uniform in [1, N]."""
    seed = SEED_BASE + 4
    if pool is None:
        pool, d = config4_pool(n_pool, n_bits)
    else:
        d = pool_densities(n_pool, seed)
    qs = queries(seed, n_queries, n_pool, 2, min(nmax, n_pool))
    return Workload(f"c4_pool{n_pool}_q{n_queries}_r{n_bits}", n_bits, pool, qs, {"density": d})


def config5_queries(n_pool: int = 10_000, n_train: int = 50_000, n_test: int = 10_000, nmax: int = 256):
    """Training and held-out query sets drawn as in config 4 (disjoint seeds)."""
    tr = queries(SEED_BASE + 5, n_train, n_pool, 2, min(nmax, n_pool))
    te = queries(SEED_BASE + 6, n_test, n_pool, 2, min(nmax, n_pool))
    return tr, te
