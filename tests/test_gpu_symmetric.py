"""Symmetric functions of the row count on the GPU path (needs an MI355X).

Output row i is f[c_i] (c_i = inputs with row i set), f a table over 0..N
(Section 2: at most T, a range [T1, T2]; Section 3.2: parity).  Every case is
compared word for word with the oracle on the same seeded inputs: several
tiles and a ragged tail, word-level (N <= 256) and 4-word-group (N > 256)
bounds, tables whose first value is 1 (groups settled as ones), parity, constant
tables, eight runs of ones (the largest that goes through run ends), and general
tables of many runs (looked up per row) at N = 20, 64, 300 and 4095.
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


def _gpu_symmetric(G, bms, f):
    E = G.lib()
    n_bits = bms[0].n_bits
    out, out_n, cap = G.alloc_out(n_bits, sum(b.n_words for b in bms))
    E.symmetric(bms, f, out.data_ptr(), cap, out_n.data_ptr())
    return G.fetch(out, out_n)


def _tables(n, rng):
    t1 = int(rng.integers(0, n + 1))
    t2 = int(rng.integers(t1, n + 1))
    tabs = {
        "at_least": [1 if c >= max(t1, 1) else 0 for c in range(n + 1)],
        "at_most": [1 if c <= t1 else 0 for c in range(n + 1)],
        "exactly": [1 if c == t1 else 0 for c in range(n + 1)],
        "range": [1 if t1 <= c <= t2 else 0 for c in range(n + 1)],
        "outside": [0 if t1 <= c <= t2 else 1 for c in range(n + 1)],
        "odd": [c % 2 for c in range(n + 1)],
        "even": [1 - c % 2 for c in range(n + 1)],
        "none": [0] * (n + 1),
        "all": [1] * (n + 1),
    }
    if n >= 16:   # eight runs of ones: counts 1, 3, ..., 15
        tabs["eight_runs"] = [1 if c < 16 and c % 2 == 1 else 0 for c in range(n + 1)]
    if n >= 18:   # nine runs: looked up per row
        tabs["nine_runs"] = [1 if c < 18 and c % 2 == 1 else 0 for c in range(n + 1)]
    tabs["mod3"] = [1 if c % 3 == 0 else 0 for c in range(n + 1)]
    tabs["random"] = [int(v) for v in rng.integers(0, 2, n + 1)]
    return tabs


@pytest.mark.parametrize("case", range(6))
def test_tables_against_oracle(G, case):
    E = G.lib()
    rng = np.random.default_rng(500 + case)
    n = [1, 3, 8, 64, 200, 300][case]
    n_bits = int(rng.choice([1, 65, TW_ROWS - 3, 3 * TW_ROWS + 901]))
    if case % 2:
        streams = D.bitmaps(D.IID, rng.uniform(0.001, 0.4, n), 0.0, n_bits, [D.key(600 + case, k) for k in range(n)])
    else:   # runs far apart: some words touched by few inputs (groups settled), others by many
        streams = D.bitmaps(D.MARKOV, 300.0, np.full(n, 3000.0), n_bits, [D.key(600 + case, k) for k in range(n)])
    bms = G.register(streams, n_bits)
    try:
        for name, f in _tables(n, rng).items():
            want = O.symmetric(streams, n_bits, f)
            got = _gpu_symmetric(G, bms, f)
            assert np.array_equal(got, want), (n, n_bits, name)
            if name == "at_least":
                T = f.index(1) if 1 in f else n + 1
                assert np.array_equal(got, G.gpu_threshold(bms, T)), (n, n_bits, "threshold path")
    finally:
        for b in bms:
            b.release()
    assert E.device_errors() == 0


def test_at_most_and_ranges_with_settled_groups(G):
    """Tables with f(0) = 1 over inputs whose runs leave most words touched by few inputs."""
    E = G.lib()
    n_bits = 4 * TW_ROWS + 333
    n = 120
    streams = D.bitmaps(D.MARKOV, 400.0, np.full(n, 4000.0), n_bits, [D.key(7070, k) for k in range(n)])
    bms = G.register(streams, n_bits)
    try:
        for T in (0, 1, 3, 8, 15, 30):
            f = [1 if c <= T else 0 for c in range(n + 1)]
            assert np.array_equal(_gpu_symmetric(G, bms, f), O.symmetric(streams, n_bits, f)), ("at_most", T)
        for t1, t2 in ((0, 2), (5, 9), (12, 40), (1, 1)):
            f = [0 if t1 <= c <= t2 else 1 for c in range(n + 1)]
            assert np.array_equal(_gpu_symmetric(G, bms, f), O.symmetric(streams, n_bits, f)), ("outside", t1, t2)
    finally:
        for b in bms:
            b.release()
    assert E.device_errors() == 0


def test_general_tables_and_table_length(G):
    E = G.lib()
    n_bits = 1000
    n = 20
    streams = D.bitmaps(D.IID, np.full(n, 0.3), 0.0, n_bits, [D.key(8080, k) for k in range(n)])
    bms = G.register(streams, n_bits)
    try:
        out, out_n, cap = G.alloc_out(n_bits, sum(b.n_words for b in bms))
        with pytest.raises(E.EwahError) as e:
            E.symmetric(bms, [1] * n, out.data_ptr(), cap, out_n.data_ptr())   # one entry short
        assert e.value.code == E.EINVAL
        eight, nine = [0] * (n + 1), [0] * (n + 1)
        for j in range(8):
            eight[2 * j] = 1
        for j in range(9):
            nine[2 * j] = 1   # nine runs of ones, not parity
        for f in (eight, nine):
            assert np.array_equal(_gpu_symmetric(G, bms, f), O.symmetric(streams, n_bits, f))
    finally:
        for b in bms:
            b.release()
    assert E.device_errors() == 0


@pytest.mark.parametrize("n,n_bits,seed", [(64, 3 * TW_ROWS + 5001, 71), (300, 2 * TW_ROWS + 99, 72),
                                           (4095, TW_ROWS + 777, 73)])
def test_many_run_tables_against_oracle(G, n, n_bits, seed):
    """Tables with many runs of counts giving 1 (random, counts divisible by 3, every
    count but one), including f(0) = 1, against the oracle."""
    E = G.lib()
    rng = np.random.default_rng(seed)
    dens = rng.uniform(0.01, 0.5, n)
    streams = D.bitmaps(D.MARKOV, 16.0, 16.0 * (1.0 - dens) / dens, n_bits, [D.key(seed, k) for k in range(n)])
    bms = G.register(streams, n_bits)
    try:
        tabs = [[int(v) for v in rng.integers(0, 2, n + 1)] for _ in range(2)]
        tabs.append([1 if c % 3 == 0 else 0 for c in range(n + 1)])
        k = int(rng.integers(1, n))
        tabs.append([0 if c == k else 1 for c in range(n + 1)])
        for f in tabs:
            want = O.symmetric(streams, n_bits, f)
            got = _gpu_symmetric(G, bms, f)
            assert np.array_equal(got, want), (n, n_bits, f[:20])
    finally:
        for b in bms:
            b.release()
    assert E.device_errors() == 0
