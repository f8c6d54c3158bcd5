"""Pins of the CPU oracle by brute force, identities and invariants (CPU only).

Identities used (all from the paper):
  * T = 1 is OR, T = N is AND (Section 2);
  * at most T via complements: the rows with count >= T among b are the rows
    NOT having count >= N - T + 1 among the complemented inputs (Section 2,
    generalizations), over the r valid rows;
  * Looped recurrence theta(T, b1..bN) = theta(T, b1..bN-1) | (theta(T-1, b1..bN-1) & bN)
    (Section 6.2);
  * symmetry under permutation of the inputs (Section 3.2);
  * sum over T = 1..N of |theta(T)| = B, the total number of ones (Section 2:
    a row with count c is counted once for each T <= c).
"""
import itertools

import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from paper_1402_4466_amd import datagen
from tests.ewah_test_util import literal_stream, marker, mixed_stream, popcount_words


def _mask(r):
    U = (r + 63) // 64
    m = np.full(U, 2**64 - 1, dtype=np.uint64)
    if r % 64:
        m[-1] = np.uint64((1 << (r % 64)) - 1)
    return m


def _rand_words(rng, r, density):
    U = (r + 63) // 64
    bits = rng.random((U, 64)) < density
    w = np.zeros(U, dtype=np.uint64)
    for b in range(64):
        w |= bits[:, b].astype(np.uint64) << np.uint64(b)
    # make some words fills
    z = rng.random(U)
    w[z < 0.15] = 0
    w[(z >= 0.15) & (z < 0.25)] = np.uint64(2**64 - 1)
    return w & _mask(r)


def _thr(streams, r, T):
    return O.decode(O.threshold(streams, r, T)[0], r)


def test_brute_exhaustive_small():
    """All bitmap tuples with N <= 3 over r <= 4 rows, every T in 0..N+1."""
    for N in range(0, 4):
        for r in range(0, 5):
            for combo in itertools.product(range(1 << r), repeat=N):
                sets = [{i for i in range(r) if (v >> i) & 1} for v in combo]
                streams = [literal_stream(brute.words_from_rows(s, r)) for s in sets]
                for T in range(0, N + 2):
                    got = brute.rows_from_words(_thr(streams, r, T), r)
                    assert got == brute.threshold_sets(sets, r, T), (N, r, combo, T)


def test_brute_n4_sampled():
    rng = np.random.default_rng(11)
    r = 4
    for _ in range(3000):
        combo = rng.integers(0, 16, size=4)
        sets = [{i for i in range(r) if (int(v) >> i) & 1} for v in combo]
        streams = [literal_stream(brute.words_from_rows(s, r)) for s in sets]
        T = int(rng.integers(0, 6))
        assert brute.rows_from_words(_thr(streams, r, T), r) == brute.threshold_sets(sets, r, T)


def test_brute_random_medium():
    """Random N <= 12, r <= 300 with mixed non-canonical input streams."""
    rng = np.random.default_rng(5)
    for _ in range(60):
        N = int(rng.integers(1, 13))
        r = int(rng.integers(1, 301))
        dens = rng.random()
        words = [_rand_words(rng, r, dens * rng.random()) for _ in range(N)]
        sets = [brute.rows_from_words(w, r) for w in words]
        streams = [mixed_stream(w, rng) for w in words]
        for T in sorted({0, 1, N, N + 1, int(rng.integers(1, N + 1))}):
            got = brute.rows_from_words(_thr(streams, r, T), r)
            assert got == brute.threshold_sets(sets, r, T)


def _rand_case(rng, N, r):
    dens = [rng.random() * rng.random() for _ in range(N)]
    words = [_rand_words(rng, r, d) for d in dens]
    return words, [mixed_stream(w, rng) for w in words]


def test_or_and_identities():
    rng = np.random.default_rng(21)
    for _ in range(25):
        N, r = int(rng.integers(1, 20)), int(rng.integers(1, 2000))
        words, streams = _rand_case(rng, N, r)
        orv = np.zeros_like(words[0]); andv = _mask(r).copy()
        for w in words:
            orv |= w; andv &= w
        assert np.array_equal(_thr(streams, r, 1), orv)
        assert np.array_equal(_thr(streams, r, N), andv)
        assert np.array_equal(_thr(streams, r, 0), _mask(r))
        assert not _thr(streams, r, N + 1).any()


def test_monotone_permutation_popcount_sum():
    rng = np.random.default_rng(22)
    for _ in range(15):
        N, r = int(rng.integers(2, 16)), int(rng.integers(64, 3000))
        words, streams = _rand_case(rng, N, r)
        B = sum(popcount_words(w) for w in words)
        outs = [_thr(streams, r, T) for T in range(0, N + 2)]
        for T in range(0, N + 1):
            assert not (outs[T + 1] & ~outs[T]).any()        # out(T+1) subset of out(T)
        assert sum(popcount_words(outs[T]) for T in range(1, N + 1)) == B
        perm = rng.permutation(N)
        for T in range(1, N + 1):
            assert np.array_equal(_thr([streams[i] for i in perm], r, T), outs[T])
        # duplicating every input doubles every count: theta(2T) on {B, B} = theta(T) on {B}
        for T in range(1, N + 1):
            assert np.array_equal(_thr(streams + streams, r, 2 * T), outs[T])
        # histogram: hist[c] rows with count exactly c
        _, hist = O.threshold(streams, r, 1)
        assert int(hist.sum()) == r
        assert sum(c * int(h) for c, h in enumerate(hist)) == B


def test_complement_identity():
    rng = np.random.default_rng(23)
    for _ in range(15):
        N, r = int(rng.integers(1, 12)), int(rng.integers(1, 1500))
        words, streams = _rand_case(rng, N, r)
        comp = [literal_stream(~w & _mask(r)) for w in words]
        for T in range(0, N + 2):
            lhs = _thr(streams, r, T)
            rhs = ~_thr(comp, r, N - T + 1) & _mask(r)
            assert np.array_equal(lhs, rhs)


def test_looped_recurrence():
    rng = np.random.default_rng(24)
    for _ in range(15):
        N, r = int(rng.integers(2, 12)), int(rng.integers(1, 1500))
        words, streams = _rand_case(rng, N, r)
        for T in range(1, N + 1):
            lhs = _thr(streams, r, T)
            rhs = _thr(streams[:-1], r, T) | (_thr(streams[:-1], r, T - 1) & words[-1])
            assert np.array_equal(lhs, rhs)


def test_output_size_bound():
    rng = np.random.default_rng(25)
    for _ in range(30):
        N, r = int(rng.integers(1, 10)), int(rng.integers(1, 5000))
        words = [_rand_words(rng, r, rng.random() * 0.2) for _ in range(N)]
        streams = [O.encode(w, r) for w in words]
        U = (r + 63) // 64
        for T in range(0, N + 2):
            out, _ = O.threshold(streams, r, T)
            assert len(out) <= min(U + 1, sum(len(s) for s in streams) + 1)


def test_generator_streams_roundtrip():
    """Generator output (canonical and perturbed) decodes, and canonical streams re-encode to themselves."""
    r = 5000
    for model, a, b in ((datagen.IID, 0.05, 0), (datagen.IID, 0.6, 0), (datagen.MARKOV, 32.0, 200.0),
                        (datagen.MARKOV, 200.0, 50.0)):
        for k in range(5):
            key = datagen.key(99, k)
            s = datagen.bitmap(model, a, b, r, key)
            d = O.decode(s, r)
            assert np.array_equal(O.encode(d, r), s)
            s2 = datagen.bitmap(model, a, b, r, key, noncanon=True)
            assert np.array_equal(O.decode(s2, r), d)


# ------------------------------------------------------------- encoder

def _check_canonical(stream, dense, r):
    """Independent structural check of rules C1-C4 on an encoder output."""
    U = (r + 63) // 64
    mask = _mask(r)
    pos = 0
    p = 0
    prev_cls = None
    heads = 0
    while p < len(stream):
        m = int(stream[p]); p += 1
        f, L, K = m & 1, (m >> 1) & 0xFFFFFFFF, m >> 33
        heads += 1
        # C2: a marker starts at word 0 or at a fill that differs from its predecessor's class
        if pos > 0:
            assert L > 0, "only the marker at word 0 may have L = 0 (no overflow at these sizes)"
            assert prev_cls is not None and prev_cls != f, "fill continues the previous run"
        for i in range(L):
            assert int(dense[pos + i]) == (int(mask[pos + i]) if f else 0)
            # C1 for fills: a one-fill is never the masked last partial word
            if f:
                assert pos + i != U - 1 or r % 64 == 0
        pos += L
        for i in range(K):
            v = int(stream[p + i])
            assert v == int(dense[pos + i])
            assert v != 0 and v != 2**64 - 1, "C1: fill-valued word written as literal"
        pos += K; p += K
        prev_cls = "L" if K else f
    assert pos == U
    n_lit = sum(1 for i in range(U) if int(dense[i]) not in (0, 2**64 - 1))
    return heads + n_lit == len(stream)


def test_encoder_exhaustive_word_classes():
    """All sequences of up to 6 words over {0, ~0, lit_a, lit_b}, with full and partial last words."""
    vals = [0, 2**64 - 1, 0x5, 0xF0F0]
    for n in range(0, 7):
        for seq in itertools.product(range(4), repeat=n):
            for partial in ([0] if n == 0 else [0, 17, 63]):
                r = 64 * n - (64 - partial if partial else 0)
                dense = np.array([vals[i] for i in seq], dtype=np.uint64)
                if n:
                    dense &= _mask(r)
                enc = O.encode(dense, r)
                assert np.array_equal(O.decode(enc, r), dense)
                assert _check_canonical(enc, dense, r)
                # encode(decode(x)) == x for canonical x
                assert np.array_equal(O.encode(O.decode(enc, r), r), enc)


def test_encoder_overflow_rules():
    """C2 overflow: hand-built streams with L = 2^32 - 1 decode, and a run one
    longer than 2^32 - 1 fill words is split over two markers by the encoder (checked on
    the decoder side only: 2^32 words do not fit in memory)."""
    r = 64 * 3
    s = np.array([marker(0, 3, 0)], dtype=np.uint64)
    assert not O.decode(s, r).any()
    # a maximal L value is accepted as long as the stream covers U words exactly
    big = np.array([marker(1, 2**32 - 1, 0)], dtype=np.uint64)
    with pytest.raises(O.OracleError):
        O.decode(big, r)   # covers more than U words


# ------------------------------------------------------------- decoder errors

def test_decoder_rejects_malformed():
    r = 64 * 4
    lit = 0x1234
    good = np.array([marker(0, 1, 2), lit, lit, marker(1, 1, 0)], dtype=np.uint64)
    assert O.decode(good, r).tolist() == [0, lit, lit, 2**64 - 1]
    cases = [
        np.array([marker(0, 1, 3), lit, lit], dtype=np.uint64),              # ends inside a literal run
        np.array([marker(0, 1, 2), lit, lit], dtype=np.uint64),              # covers 3 of 4 words
        np.array([marker(0, 3, 2), lit, lit], dtype=np.uint64),              # covers 5 of 4 words
        np.array([marker(0, 4, 0), marker(0, 1, 0)], dtype=np.uint64),       # extra run past U
    ]
    for c in cases:
        with pytest.raises(O.OracleError) as e:
            O.decode(c, r)
        assert e.value.code == O.EFORMAT
    with pytest.raises(O.OracleError):
        O.threshold([good, cases[0]], r, 1)


def test_decoder_masks_padding_and_accepts_noncanonical():
    r = 70  # 2 words, 6 valid bits in the last
    s = np.array([marker(1, 2, 0)], dtype=np.uint64)
    assert O.decode(s, r).tolist() == [2**64 - 1, 0x3F]
    s = np.array([marker(0, 0, 2), 2**64 - 1, 2**64 - 1, marker(1, 0, 0)], dtype=np.uint64)
    assert O.decode(s, r).tolist() == [2**64 - 1, 0x3F]
    # the canonical encoding of that: one one-fill, then the partial word as a literal
    assert O.encode(np.array([2**64 - 1, 0x3F], dtype=np.uint64), r).tolist() == [marker(1, 1, 1), 0x3F]
    # r = 0: empty stream; an empty marker is also accepted
    assert O.decode(np.array([], dtype=np.uint64), 0).tolist() == []
    assert O.decode(np.array([marker(0, 0, 0)], dtype=np.uint64), 0).tolist() == []
    assert O.encode(np.array([], dtype=np.uint64), 0).tolist() == []


def test_threshold_edges():
    r = 300
    rng = np.random.default_rng(3)
    w = _rand_words(rng, r, 0.3)
    s = literal_stream(w)
    # N = 0: T = 0 gives all ones, otherwise all zeros
    assert np.array_equal(O.decode(O.threshold([], r, 0)[0], r), _mask(r))
    assert not O.decode(O.threshold([], r, 1)[0], r).any()
    # single input: T = 1 returns it, T = 2 is empty
    assert np.array_equal(_thr([s], r, 1), w)
    assert not _thr([s], r, 2).any()
