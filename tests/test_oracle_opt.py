"""Pins of the oracle's opt-threshold query (CPU only).

* brute force (row by row) on tiny inputs: T is the largest value whose result
  holds at least K rows;
* K = 1: the result is exactly the set of rows whose count equals the largest
  count (the ScanCount reading of Section 5.1);
* the count histogram against row membership counted in decoded row sets;
* at larger sizes, the defining property |result(T)| >= K > |result(T + 1)|, with
  row counts taken as popcounts of decoded threshold results.
"""
import numpy as np

from oracle import brute as Bf
from oracle import oracle as O
from paper_1402_4466_amd import datagen as D


def _rows(stream, n_bits):
    return Bf.rows_from_words(O.decode(stream, n_bits), n_bits)


def _popcount(stream, n_bits):
    w = O.decode(stream, n_bits)
    return int(sum(bin(int(x)).count("1") for x in w))


def test_brute_force_tiny():
    rng = np.random.default_rng(17)
    for case in range(25):
        n = int(rng.integers(1, 6))
        n_bits = int(rng.integers(1, 300))
        dens = rng.uniform(0.05, 0.7, n)
        streams = D.bitmaps(D.IID, dens, 0.0, n_bits, [D.key(7000 + case, k) for k in range(n)])
        sets = [_rows(s, n_bits) for s in streams]
        counts = [sum(1 for s in sets if row in s) for row in range(n_bits)]
        for K in sorted({1, 2, int(rng.integers(1, n_bits + 1)), n_bits}):
            want_T = max(T for T in range(n + 1) if sum(1 for c in counts if c >= T) >= K)
            T, out = O.opt_threshold(streams, n_bits, K)
            assert T == want_T, (case, K)
            assert _rows(out, n_bits) == Bf.threshold_sets(sets, n_bits, T), (case, K)


def test_k1_rows_with_the_largest_count():
    rng = np.random.default_rng(23)
    for case in range(10):
        n = int(rng.integers(2, 9))
        n_bits = int(rng.integers(64, 700))
        streams = D.bitmaps(D.MARKOV, 20.0, 60.0, n_bits, [D.key(7100 + case, k) for k in range(n)])
        sets = [_rows(s, n_bits) for s in streams]
        counts = [sum(1 for s in sets if row in s) for row in range(n_bits)]
        m = max(counts)
        T, out = O.opt_threshold(streams, n_bits, 1)
        assert T == m
        assert _rows(out, n_bits) == {r for r in range(n_bits) if counts[r] == m}


def test_defining_property():
    n_bits = 64 * 900 + 31
    for n, seed in ((12, 1), (40, 2)):
        streams = D.bitmaps(D.IID, np.linspace(0.01, 0.3, n), 0.0, n_bits, [D.key(7200 + seed, k) for k in range(n)])
        for K in (1, 5, 100, 10_000, n_bits):
            T, out = O.opt_threshold(streams, n_bits, K)
            assert _popcount(out, n_bits) >= K, (n, K)
            if T < n:
                nxt, _ = O.threshold(streams, n_bits, T + 1, want_hist=False)
                assert _popcount(nxt, n_bits) < K, (n, K)


def test_count_histogram_brute_force():
    """The oracle's count histogram (hist[c] = rows set in exactly c inputs) against
    counting row membership in decoded row sets, including non-canonical streams."""
    rng = np.random.default_rng(23)
    for case in range(20):
        n = int(rng.integers(1, 7))
        n_bits = int(rng.integers(1, 400))
        dens = rng.uniform(0.02, 0.8, n)
        streams = D.bitmaps(D.IID, dens, 0.0, n_bits, [D.key(7100 + case, k) for k in range(n)],
                            noncanon=bool(case % 2))
        sets = [_rows(s, n_bits) for s in streams]
        counts = [sum(1 for s in sets if row in s) for row in range(n_bits)]
        _, hist = O.threshold(streams, n_bits, n + 1)
        assert [int(h) for h in hist] == [counts.count(c) for c in range(n + 1)], case
