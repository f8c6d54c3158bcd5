"""Pins of the oracle's symmetric-function query (CPU only).

The oracle computes output row i = f[c_i] from ScanCount counters.  It is
checked against things that do not share that computation:

* brute force (row by row, sets of rows) on tiny inputs, for every table f when
  N <= 3 and random tables above;
* the identity of Section 2: "at most T of the N bits are set" equals the
  threshold N - T over the complemented inputs (complements taken on decoded
  words, the threshold oracle pinned separately);
* Section 3.2: odd parity of the count is the XOR of the inputs (numpy XOR of
  the decoded words);
* a range [T1, T2] is the threshold T1 AND NOT the threshold T2 + 1;
* constant tables give all zeros / all ones over r rows.
"""
import itertools

import numpy as np

from oracle import brute as Bf
from oracle import oracle as O
from paper_1402_4466_amd import datagen as D


def _inputs(seed, n, n_bits, noncanon=False):
    rng = np.random.default_rng(seed)
    dens = rng.uniform(0.02, 0.6, n)
    return D.bitmaps(D.IID, dens, 0.0, n_bits, [D.key(seed, k) for k in range(n)], noncanon=noncanon)


def _rows(stream, n_bits):
    return Bf.rows_from_words(O.decode(stream, n_bits), n_bits)


def _mask(n_bits):
    U = (n_bits + 63) // 64
    m = np.full(U, np.uint64(2**64 - 1), dtype=np.uint64)
    if n_bits % 64:
        m[-1] = np.uint64((1 << (n_bits % 64)) - 1)
    return m


def test_brute_force_every_table_small_n():
    for n, n_bits, seed in ((1, 70, 1), (2, 130, 2), (3, 200, 3), (3, 64, 4)):
        streams = _inputs(seed, n, n_bits, noncanon=bool(seed % 2))
        sets = [_rows(s, n_bits) for s in streams]
        for f in itertools.product([0, 1], repeat=n + 1):
            got = _rows(O.symmetric(streams, n_bits, f), n_bits)
            assert got == Bf.symmetric_sets(sets, n_bits, f), (n, f)


def test_brute_force_random_tables():
    rng = np.random.default_rng(9)
    for case in range(12):
        n = int(rng.integers(4, 7))
        n_bits = int(rng.integers(1, 400))
        streams = _inputs(100 + case, n, n_bits)
        sets = [_rows(s, n_bits) for s in streams]
        f = rng.integers(0, 2, n + 1)
        got = _rows(O.symmetric(streams, n_bits, f), n_bits)
        assert got == Bf.symmetric_sets(sets, n_bits, f), case


def test_at_most_is_threshold_of_complements():
    n_bits = 3 * 64 * 50 + 17
    n = 9
    streams = _inputs(21, n, n_bits)
    m = _mask(n_bits)
    comp = [O.encode(~O.decode(s, n_bits) & m, n_bits) for s in streams]
    for T in range(0, n + 1):
        f = [1 if c <= T else 0 for c in range(n + 1)]
        want, _ = O.threshold(comp, n_bits, n - T, want_hist=False)
        assert np.array_equal(O.symmetric(streams, n_bits, f), want), T


def test_odd_parity_is_xor():
    n_bits = 5000
    for n in (1, 2, 5, 8):
        streams = _inputs(30 + n, n, n_bits)
        x = np.zeros((n_bits + 63) // 64, dtype=np.uint64)
        for s in streams:
            x ^= O.decode(s, n_bits)
        f_odd = [c % 2 for c in range(n + 1)]
        f_even = [1 - c % 2 for c in range(n + 1)]
        assert np.array_equal(O.symmetric(streams, n_bits, f_odd), O.encode(x, n_bits)), n
        assert np.array_equal(O.symmetric(streams, n_bits, f_even), O.encode(~x & _mask(n_bits), n_bits)), n


def test_range_is_threshold_and_not_threshold():
    n_bits = 64 * 77 + 5
    n = 7
    streams = _inputs(44, n, n_bits)
    for t1, t2 in ((0, 0), (1, 3), (2, 2), (3, 7), (5, 6)):
        f = [1 if t1 <= c <= t2 else 0 for c in range(n + 1)]
        lo = O.decode(O.threshold(streams, n_bits, t1, want_hist=False)[0], n_bits)
        hi = O.decode(O.threshold(streams, n_bits, t2 + 1, want_hist=False)[0], n_bits)
        assert np.array_equal(O.symmetric(streams, n_bits, f), O.encode(lo & ~hi, n_bits)), (t1, t2)


def test_constant_tables():
    for n_bits in (1, 64, 65, 1000):
        streams = _inputs(55, 3, n_bits)
        U = (n_bits + 63) // 64
        assert np.array_equal(O.symmetric(streams, n_bits, [0, 0, 0, 0]), O.encode(np.zeros(U, dtype=np.uint64), n_bits))
        assert np.array_equal(O.symmetric(streams, n_bits, [1, 1, 1, 1]), O.encode(_mask(n_bits), n_bits))
