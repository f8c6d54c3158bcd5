"""Brute-force threshold and symmetric functions (test infrastructure only): pure
Python, bit by bit.

Used on tiny inputs to pin the C oracle.  Bitmaps are Python sets of row
numbers; the threshold result is the set of rows present in at least T of
the N sets (Section 2, Formulation).
"""
from __future__ import annotations


def threshold_sets(sets, r: int, T: int) -> set:
    out = set()
    for row in range(r):
        count = 0
        for s in sets:
            if row in s:
                count += 1
        if count >= T:
            out.add(row)
    return out


def symmetric_sets(sets, r: int, f) -> set:
    """Rows whose count c (sets holding the row) has f[c] true (Section 2, Section 3.2)."""
    out = set()
    for row in range(r):
        count = 0
        for s in sets:
            if row in s:
                count += 1
        if f[count]:
            out.add(row)
    return out


def words_from_rows(rows, r: int) -> list:
    """Uncompressed layout (Section 3.1, W = 64): row i is bit i mod 64 of word i // 64."""
    U = (r + 63) // 64
    words = [0] * U
    for row in rows:
        words[row // 64] |= 1 << (row % 64)
    return words


def rows_from_words(words, r: int) -> set:
    out = set()
    for i, w in enumerate(words):
        w = int(w)
        for b in range(64):
            if (w >> b) & 1 and i * 64 + b < r:
                out.add(i * 64 + b)
    return out
