"""Opt-threshold on the GPU path (needs an MI355X): the largest T whose result has
at least K rows (Section 3.3), and that result, against the oracle.

Covers several tiles with a ragged tail, word and 4-word bounds (N up to 1000),
K from 1 to n_bits, all-zero inputs (T = 0: every row), a single row, the
full-size config-2 inputs, and the argument checks.  The count histogram that
K > 1 reads (ewah_count_histogram) is compared with the oracle's directly.
"""
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_1402_4466_amd import datagen as D

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TW = int(re.search(r"#define EWT_TILE_WORDS (\d+)",
                   open(os.path.join(ROOT, "paper_1402_4466_amd", "csrc", "thr_device.h")).read()).group(1))
TW_ROWS = TW * 64   # rows per tile


@pytest.fixture(scope="module")
def G():
    from tests import gpu_util
    gpu_util.lib()
    return gpu_util


def _gpu_opt(G, bms, K):
    E = G.lib()
    n_bits = bms[0].n_bits
    out, out_n, cap = G.alloc_out(n_bits, sum(b.n_words for b in bms))
    T = E.opt_threshold(bms, K, out.data_ptr(), cap, out_n.data_ptr())
    return T, G.fetch(out, out_n)


@pytest.mark.parametrize("case", range(5))
def test_opt_against_oracle(G, case):
    E = G.lib()
    rng = np.random.default_rng(900 + case)
    n = [1, 5, 64, 64, 300][case]
    n_bits = [1, 777, TW_ROWS, 3 * TW_ROWS + 4321, 2 * TW_ROWS + 99][case]
    if case % 2:
        streams = D.bitmaps(D.MARKOV, 200.0, np.full(n, 2000.0), n_bits, [D.key(910 + case, k) for k in range(n)])
    else:
        streams = D.bitmaps(D.IID, rng.uniform(0.001, 0.3, n), 0.0, n_bits, [D.key(910 + case, k) for k in range(n)])
    bms = G.register(streams, n_bits)
    try:
        for K in sorted({1, 2, 37, max(1, n_bits // 3), n_bits}):
            if K > n_bits:
                continue
            want_T, want = O.opt_threshold(streams, n_bits, K)
            T, got = _gpu_opt(G, bms, K)
            assert T == want_T, (n, n_bits, K)
            assert np.array_equal(got, want), (n, n_bits, K)
    finally:
        for b in bms:
            b.release()
    assert E.device_errors() == 0


def test_all_zero_inputs_and_errors(G):
    E = G.lib()
    n_bits = 2 * TW_ROWS + 5
    U = (n_bits + 63) // 64
    streams = [O.encode(np.zeros(U, dtype=np.uint64), n_bits) for _ in range(4)]
    bms = G.register(streams, n_bits)
    try:
        for K in (1, 1000, n_bits):
            want_T, want = O.opt_threshold(streams, n_bits, K)
            T, got = _gpu_opt(G, bms, K)
            assert T == want_T == 0 and np.array_equal(got, want), K
        out, out_n, cap = G.alloc_out(n_bits, sum(b.n_words for b in bms))
        for K in (0, n_bits + 1):
            with pytest.raises(E.EwahError) as e:
                E.opt_threshold(bms, K, out.data_ptr(), cap, out_n.data_ptr())
            assert e.value.code == E.EINVAL
    finally:
        for b in bms:
            b.release()
    assert E.device_errors() == 0


def test_config2_full(G):
    E = G.lib()
    w = D.config2()
    bms = G.register(w.streams, w.n_bits)
    try:
        for K in (1, 1000, 2_000_000):
            want_T, want = O.opt_threshold(w.streams, w.n_bits, K)
            T, got = _gpu_opt(G, bms, K)
            print(f"config 2 K={K}: T={T} ({len(got)} words)", flush=True)
            assert T == want_T and np.array_equal(got, want), K
    finally:
        for b in bms:
            b.release()
    assert E.device_errors() == 0


@pytest.mark.parametrize("case", range(6))
def test_count_histogram_against_oracle(G, case):
    """ewah_count_histogram against the oracle's ScanCount histogram: word (N <= 256) and
    4-word (N > 256) bounds, tiles settled as uniform, one-fills, a ragged tail, one row."""
    E = G.lib()
    n = [1, 7, 64, 300, 1000, 40][case]
    n_bits = [1, 3 * TW_ROWS + 77, 2 * TW_ROWS, TW_ROWS + 5, 3000, 5 * TW_ROWS + 1][case]
    if case == 5:   # long one-fills and zero-fills: tiles where every count is equal
        streams = D.bitmaps(D.MARKOV, float(TW_ROWS), float(TW_ROWS), n_bits, [D.key(950, k) for k in range(n)])
    elif case % 2:
        streams = D.bitmaps(D.MARKOV, 100.0, np.full(n, 1500.0), n_bits, [D.key(940 + case, k) for k in range(n)])
    else:
        rng = np.random.default_rng(930 + case)
        streams = D.bitmaps(D.IID, rng.uniform(0.001, 0.5, n), 0.0, n_bits, [D.key(940 + case, k) for k in range(n)])
    bms = G.register(streams, n_bits)
    try:
        _, want = O.threshold(streams, n_bits, n + 1)
        got = E.count_histogram(bms)
        assert np.array_equal(got, want), (n, n_bits)
        # repeated inputs count once per occurrence
        twice = bms + bms[: max(1, n // 3)]
        _, want2 = O.threshold(streams + streams[: max(1, n // 3)], n_bits, len(twice) + 1)
        assert np.array_equal(E.count_histogram(twice), want2), (n, n_bits, "repeats")
    finally:
        for b in bms:
            b.release()
    assert E.device_errors() == 0


def test_count_histogram_full_config2_and_errors(G):
    E = G.lib()
    w = D.config2()
    bms = G.register(w.streams, w.n_bits)
    try:
        _, want = O.threshold(w.streams, w.n_bits, len(w.streams) + 1)
        got = E.count_histogram(bms)
        print(f"config 2 histogram: rows of count >= 1: {int(got[1:].sum())}", flush=True)
        assert np.array_equal(got, want)
        with pytest.raises(E.EwahError) as e:
            E.count_histogram([])
        assert e.value.code == E.EINVAL
    finally:
        for b in bms:
            b.release()
    assert E.device_errors() == 0


def test_largest_count_many_tiles(G):
    """The largest-count pass reads the running maximum once per workgroup, so every
    wavefront of a tile takes the same early exit while other tiles raise the maximum;
    many tiles of uneven counts (word and 4-word bounds) make the maximum move during the
    launch."""
    E = G.lib()
    for n, seed in ((48, 951), (300, 952)):
        n_bits = 40 * TW_ROWS + 17
        rng = np.random.default_rng(seed)
        dens = rng.uniform(0.0005, 0.05, n)
        streams = D.bitmaps(D.MARKOV, 32.0, 32.0 * (1.0 - dens) / dens, n_bits, [D.key(seed, k) for k in range(n)])
        bms = G.register(streams, n_bits)
        try:
            want_T, want = O.opt_threshold(streams, n_bits, 1)
            for rep in range(3):
                T, got = _gpu_opt(G, bms, 1)
                print(f"largest count N={n} rep {rep}: T={T}", flush=True)
                assert T == want_T and np.array_equal(got, want), (n, rep)
        finally:
            for b in bms:
                b.release()
    assert E.device_errors() == 0
