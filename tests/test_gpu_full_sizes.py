"""Parity at the full workload sizes, in the launch configurations the benchmark times
(needs an MI355X).

* N=64 Markov bitmaps over 2^24 rows and N=1024 Zipf-density bitmaps over 2^26
  rows: every output word of every threshold compared with the oracle (the
  oracle finishes these in seconds);
* (the full-size batched workloads are compared output by output in
  test_gpu_headline.py);
* degenerate shapes and the input-count limit (N = 4095: threshold, the unary counter at its
  12 levels, the 4,096-bin count histogram, opt-threshold and a symmetric function).
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1402_4466_amd import datagen as D

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def G():
    from tests import gpu_util
    gpu_util.lib()
    return gpu_util


def _plain_all_T(G, w, variants):
    E = G.lib()
    bms = G.register(w.streams, w.n_bits)
    try:
        for q in w.queries:
            want, _ = O.threshold([w.streams[i] for i in q.idx], w.n_bits, q.T, want_hist=False)
            for v in variants:
                got = G.gpu_threshold([bms[i] for i in q.idx], q.T, variant=v)
                _say(f"{w.name} T={q.T} variant={v:#x}: {len(got)} words (oracle {len(want)})")
                assert np.array_equal(got, want), (w.name, q.T, v)
    finally:
        for b in bms:
            b.release()
    assert E.device_errors() == 0


def test_config2_full(G):
    E = G.lib()
    _plain_all_T(G, D.config2(), [0, E.variant_code(False, 0, 0), E.variant_code(False, 8, 8, looped=True)])


def test_config3_full(G):
    E = G.lib()
    _plain_all_T(G, D.config3(), [0, E.variant_code(False, 8, 8, looped=True)])


def test_degenerate_shapes(G):
    E = G.lib()
    rng = np.random.default_rng(77)
    for n_bits in (1, 63, 64, 65, 64 * 1024, 64 * 1024 + 1, 64 * 2048 - 1):
        U = (n_bits + 63) // 64
        zeros = np.zeros(U, dtype=np.uint64)
        ones = np.full(U, ~np.uint64(0), dtype=np.uint64)
        rnd = rng.integers(0, 2**63, U, dtype=np.uint64) | rng.integers(0, 2, U, dtype=np.uint64) << np.uint64(63)
        streams = [O.encode(x, n_bits) for x in (zeros, ones, rnd)]
        bms = G.register(streams, n_bits)
        try:
            for sub in ([0], [1], [2], [0, 1], [1, 2], [0, 1, 2], [1, 1, 2, 2]):
                ins = [bms[i] for i in sub]
                for T in range(0, len(sub) + 2):
                    want, _ = O.threshold([streams[i] for i in sub], n_bits, T, want_hist=False)
                    got = G.gpu_threshold(ins, T)
                    assert np.array_equal(got, want), (n_bits, sub, T)
        finally:
            for b in bms:
                b.release()
    assert E.device_errors() == 0


def test_input_count_limit(G):
    E = G.lib()
    n_bits = 2 * 64 * 1024 + 333
    n = 4095   # largest query the planes admit
    dens = np.full(n, 0.002)
    streams = D.bitmaps(D.IID, dens, 0.0, n_bits, [D.key(4095, k) for k in range(n)])
    bms = G.register(streams, n_bits)
    try:
        for T in (1, 2, 3, 4095):
            want, _ = O.threshold(streams, n_bits, T, want_hist=False)
            got = G.gpu_threshold(bms, T)
            assert np.array_equal(got, want), T
        # the unary counter at its largest level count (T = bit length of N = 12)
        want, hist = O.threshold(streams, n_bits, 12)
        assert np.array_equal(G.gpu_threshold(bms, 12, variant=E.variant_code(False, 8, 8, looped=True)), want)
        # count histogram (N + 1 = 4096 bins, the LDS bin capacity), opt-threshold, a symmetric function
        assert np.array_equal(E.count_histogram(bms), hist)
        out, out_n, cap = G.alloc_out(n_bits, sum(len(s) for s in streams))
        for K in (1, 50):
            want_T, want_words = O.opt_threshold(streams, n_bits, K)
            assert E.opt_threshold(bms, K, out.data_ptr(), cap, out_n.data_ptr()) == want_T, K
            assert np.array_equal(G.fetch(out, out_n), want_words), K
        f = [1 if 2 <= c <= 5 else 0 for c in range(n + 1)]
        E.symmetric(bms, f, out.data_ptr(), cap, out_n.data_ptr())
        assert np.array_equal(G.fetch(out, out_n), O.symmetric(streams, n_bits, f))
        out, out_n, cap = G.alloc_out(n_bits, sum(len(s) for s in streams) * 2)
        with pytest.raises(E.EwahError) as e:
            E.threshold(bms + bms[:1], 1, out.data_ptr(), cap, out_n.data_ptr())
        assert e.value.code == E.EINVAL
        with pytest.raises(E.EwahError) as e:
            E.count_histogram(bms + bms[:1])
        assert e.value.code == E.EINVAL
    finally:
        for b in bms:
            b.release()
    assert E.device_errors() == 0
