"""Test-only helpers: hand-made EWAH streams and golden fixtures.

The stream writers here are deliberately simple and non-canonical (one marker
per word), so that inputs fed to the oracle do not come from any canonical
encoder under test.
"""
from __future__ import annotations

import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name: str) -> dict:
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def marker(f: int, L: int, K: int) -> int:
    """Marker word under the adopted layout: fill bit 0, L in bits 1..32, K in bits 33..63."""
    assert f in (0, 1) and 0 <= L < 2**32 and 0 <= K < 2**31
    return f | (L << 1) | (K << 33)


def literal_stream(words) -> np.ndarray:
    """Every word as its own literal: [M(0,0,1), w0, M(0,0,1), w1, ...]."""
    out = []
    for w in words:
        out.append(marker(0, 0, 1))
        out.append(int(w))
    return np.array(out, dtype=np.uint64)


def mixed_stream(words, rng) -> np.ndarray:
    """Random well-formed, usually non-canonical stream: each word either as a
    one-word fill (if it is 0 or ~0) or as a one-word literal, with random empty markers."""
    out = []
    for w in words:
        w = int(w)
        if rng.random() < 0.1:
            out.append(marker(int(rng.integers(2)), 0, 0))
        if w in (0, 2**64 - 1) and rng.random() < 0.7:
            out.append(marker(1 if w else 0, 1, 0))
        else:
            out.append(marker(int(rng.integers(2)), 0, 1))
            out.append(w)
    return np.array(out, dtype=np.uint64)


def bits_lr(s: str) -> list:
    """'0011' (rows left to right) -> [0,0,1,1]."""
    return [int(c) for c in s]


def words_of_columns(cols, r) -> list:
    U = (r + 63) // 64
    out = []
    for col in cols:
        w = [0] * U
        for i, b in enumerate(col):
            if b:
                w[i // 64] |= 1 << (i % 64)
        out.append(w)
    return out


def popcount_words(words) -> int:
    return int(sum(bin(int(w)).count("1") for w in words))
