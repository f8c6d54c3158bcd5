"""Pins of the CPU oracle against values the paper prints (tests/golden/*.json).

Each fixture names the passage it comes from.  These tests run on the CPU.
"""
import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from tests.ewah_test_util import (bits_lr, golden, literal_stream, marker, popcount_words,
                                  words_of_columns)


def _oracle_rows(streams, r, T):
    out, hist = O.threshold(streams, r, T)
    return brute.rows_from_words(O.decode(out, r), r), out, hist


def test_formulation_example():
    g = golden("formulation_example.json")
    r = g["r"]
    # the printed bit strings are most-significant bit first
    for s, bits in zip(g["sets"], g["bitstrings_msb_first"]):
        assert int(bits, 2) == sum(1 << x for x in s)
    streams = [literal_stream(brute.words_from_rows(s, r)) for s in g["sets"]]
    for T, want in g["expected"].items():
        rows, _, hist = _oracle_rows(streams, r, int(T))
        assert rows == set(want)
    # B = total number of ones = sum over c of c * hist[c]
    _, _, hist = _oracle_rows(streams, r, 1)
    assert sum(c * int(h) for c, h in enumerate(hist)) == g["B"]


def test_fig_basicexample():
    g = golden("fig_basicexample.json")
    r, T = g["r"], g["T"]
    words = words_of_columns(g["columns"], r)
    rows, _, _ = _oracle_rows([literal_stream(w) for w in words], r, T)
    want = {i for i, b in enumerate(g["expected"]) if b}
    assert rows == want


def test_uncompressed_layout():
    g = golden("uncompressed_layout.json")
    # W = 8 words, printed most-significant bit first
    w8 = [int(s, 2) for s in g["w8_words_msb_first"]]
    rows8 = {i * 8 + b for i, w in enumerate(w8) for b in range(8) if (w >> b) & 1}
    assert rows8 == set(g["set"])
    # W = 64: the oracle's decoder places row i at bit i mod 64 of word i // 64
    r = g["r"]
    dense = O.decode(literal_stream([int(g["w64_word0"], 16)]), r)
    assert brute.rows_from_words(dense, r) == set(g["set"])
    # and the threshold of the single bitmap at T=1 returns it unchanged
    rows, _, _ = _oracle_rows([literal_stream([int(g["w64_word0"], 16)])], r, 1)
    assert rows == set(g["set"])


def _bitmaps_with_counts(counts):
    """N = max(counts) bitmaps whose per-row Hamming weight is counts[row]."""
    N = max(counts)
    cols = [[1 if c > k else 0 for c in counts] for k in range(N)]
    return cols


def test_bitsliced_index_counts():
    g = golden("bitsliced_index.json")
    counts = g["counts"]
    for c, a1, a2 in zip(counts, g["A1"], g["A2"]):
        assert c == a1 + 2 * a2
    r = len(counts)
    cols = _bitmaps_with_counts(counts)
    streams = [literal_stream(w) for w in words_of_columns(cols, r)]
    N = len(cols)
    _, _, hist = _oracle_rows(streams, r, 1)
    assert [int(h) for h in hist] == [counts.count(c) for c in range(N + 1)]
    for T in range(0, N + 2):
        rows, _, _ = _oracle_rows(streams, r, T)
        assert rows == {i for i, c in enumerate(counts) if c >= T}


def test_hamming_weight_fig():
    g = golden("hamming_weight.json")
    rows = g["rows"]
    r = len(rows)
    cols = [[row[k] for row in rows] for k in range(3)]
    streams = [literal_stream(w) for w in words_of_columns(cols, r)]
    for T in range(0, 5):
        got, _, _ = _oracle_rows(streams, r, T)
        assert got == {i for i, wgt in enumerate(g["weight"]) if wgt >= T}
    for wgt, a1, a2 in zip(g["weight"], g["A1"], g["A2"]):
        assert wgt == a1 + 2 * a2


def test_bstm_walkthrough():
    g = golden("bstm_walkthrough.json")
    r = g["r"]
    cols = [bits_lr(s) for s in g["bitmaps"]]
    streams = [literal_stream(w) for w in words_of_columns(cols, r)]
    # A1 / A2 are the bit slices of the per-row counts
    counts = [sum(c[i] for c in cols) for i in range(r)]
    assert [c & 1 for c in counts] == bits_lr(g["A1"])
    assert [(c >> 1) & 1 for c in counts] == bits_lr(g["A2"])
    got, _, _ = _oracle_rows(streams, r, g["T"])
    assert got == {i for i, b in enumerate(bits_lr(g["expected"])) if b}


def test_looped_walkthrough():
    g = golden("looped_walkthrough.json")
    r = g["r"]
    cols = [bits_lr(s) for s in g["bitmaps"]]
    streams = [literal_stream(w) for w in words_of_columns(cols, r)]
    for T, key in ((1, "C1"), (2, "C2")):
        got, _, _ = _oracle_rows(streams, r, T)
        assert got == {i for i, b in enumerate(bits_lr(g[key])) if b}


def test_rbmrg_ewah_example():
    g = golden("rbmrg_ewah_example.json")
    r, T = g["r"], g["T"]
    words = [[int(x, 16) for x in b] for b in g["words"]]
    ewah = [np.array([int(x, 16) for x in e], dtype=np.uint64) for e in g["ewah"]]
    # the encodings decode to the printed words ...
    for e, w in zip(ewah, words):
        assert [int(x) for x in O.decode(e, r)] == w
        # ... and are the canonical encodings of them
        assert [int(x) for x in O.encode(np.array(w, dtype=np.uint64), r)] == [int(x) for x in e]
    # run structure stated in the text: number of fill runs and dirty runs
    for w, nf, nd in zip(words, g["runs"]["fill_runs"], g["runs"]["dirty_runs"]):
        cls = ["f" if x in (0, 2**64 - 1) else "d" for x in w]
        runs = [c for i, c in enumerate(cls) if i == 0 or cls[i - 1] != c]
        assert runs.count("f") == nf and runs.count("d") == nd
    # the threshold result at T=3, as words and as its canonical encoding
    out, hist = O.threshold(ewah, r, T)
    assert [int(x) for x in O.decode(out, r)] == [int(x, 16) for x in g["expected_words"]]
    assert [int(x) for x in out] == [int(x, 16) for x in g["expected_ewah"]]
    # the text's T=2 slip: at T=2 word 0 would be all ones (two one-fills), not 0x0
    out2, _ = O.threshold(ewah, r, 2)
    assert int(O.decode(out2, r)[0]) == 2**64 - 1


def test_marker_layout_values():
    # M(f, L, K) = f | L << 1 | K << 33; the fixture values are this formula
    assert marker(0, 1, 1) == 0x0000000200000002
    assert marker(0, 3, 2) == 0x0000000400000006
    assert marker(1, 2, 3) == 0x0000000600000005
    assert marker(1, 4, 3) == 0x0000000600000009


def test_n3_closed_forms_exhaustive():
    """Section 5.3: for N=3, theta(2) = (b1 & b2) | (b2 & b3) | (b1 & b3) = (b2 & (b1 | b3)) | (b1 & b3),
    theta(1) = b1 | b2 | b3, theta(3) = b1 & b2 & b3 (the paper's "(T=3) theta(2, ...)" is a typo for theta(3, ...))."""
    rng = np.random.default_rng(7)
    r = 200
    for _ in range(20):
        w = [rng.integers(0, 2**63, size=(r + 63) // 64, dtype=np.uint64) * np.uint64(2)
             + rng.integers(0, 2, size=(r + 63) // 64, dtype=np.uint64) for _ in range(3)]
        mask = np.array([2**64 - 1] * ((r + 63) // 64), dtype=np.uint64)
        mask[-1] = np.uint64((1 << (r % 64)) - 1)
        b1, b2, b3 = [x & mask for x in w]
        streams = [literal_stream(x) for x in (b1, b2, b3)]
        got = {T: O.decode(O.threshold(streams, r, T)[0], r) for T in (1, 2, 3)}
        assert np.array_equal(got[1], b1 | b2 | b3)
        assert np.array_equal(got[2], (b1 & b2) | (b2 & b3) | (b1 & b3))
        assert np.array_equal(got[2], (b2 & (b1 | b3)) | (b1 & b3))
        assert np.array_equal(got[3], b1 & b2 & b3)
