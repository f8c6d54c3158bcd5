"""Bit-exact parity of the HIP path against the CPU oracle (needs an MI355X).

Every case compares the canonical EWAH output words of the GPU path with the
oracle's, element by element, on the same seeded inputs.  Inputs cover several
tiles (TW uncompressed words each, read from the kernel header) and a ragged last
tile, canonical and non-canonical streams, every kernel variant, and the
degenerate cases.
"""
import itertools
import os
import re
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1402_4466_amd import datagen as D
from tests.ewah_test_util import golden, literal_stream, marker, mixed_stream

pytestmark = pytest.mark.gpu

TW = int(re.search(r"#define EWT_TILE_WORDS (\d+)",
                   open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                     "paper_1402_4466_amd", "csrc", "thr_device.h")).read()).group(1))
TW_ROWS = TW * 64   # rows per tile


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def G():
    from tests import gpu_util
    gpu_util.lib()
    return gpu_util


VARIANTS = None


def _variants(E):
    return [0,
            E.variant_code(False, 0, 0),      # everything cooperative, sparse counting
            E.variant_code(False, 255, 255),  # everything walked by single lanes
            E.variant_code(True, 0, 0),       # dense CSA + cooperative
            E.variant_code(True, 4, 16),
            E.variant_code(True, 32, 64),
            E.variant_code(False, 0, 0, looped=True),     # unary counter (T <= bit length of N), cooperative
            E.variant_code(False, 255, 255, looped=True),  # unary counter, walked by single lanes
            E.variant_code(True, 8, 8, looped=True)]       # dense flag ignored by the unary counter


def _check(G, streams, n_bits, Ts, variants=(0,), label=""):
    bms = G.register(streams, n_bits)
    try:
        for T in Ts:
            want, _ = O.threshold(streams, n_bits, T, want_hist=False)
            for v in variants:
                got = G.gpu_threshold(bms, T, variant=v)
                if not np.array_equal(got, want):
                    _say(f"MISMATCH {label} T={T} variant={v:#x} got {len(got)} words want {len(want)}")
                    k = next((i for i in range(min(len(got), len(want))) if got[i] != want[i]), None)
                    _say(f"  first diff at {k}: got {got[k] if k is not None else None} want {want[k] if k is not None else None}")
                assert np.array_equal(got, want), (label, T, v)
    finally:
        for b in bms:
            b.release()


def test_golden_rbmrg_example(G):
    g = golden("rbmrg_ewah_example.json")
    ewah = [np.array([int(x, 16) for x in e], dtype=np.uint64) for e in g["ewah"]]
    bms = G.register(ewah, g["r"])
    got = G.gpu_threshold(bms, g["T"])
    assert [int(x) for x in got] == [int(x, 16) for x in g["expected_ewah"]]
    for T in range(0, 6):
        want, _ = O.threshold(ewah, g["r"], T)
        assert np.array_equal(G.gpu_threshold(bms, T), want)
    for b in bms:
        b.release()


def test_golden_small_examples(G):
    for name in ("fig_basicexample.json",):
        g = golden(name)
        r = g["r"]
        cols = g["columns"]
        words = []
        for col in cols:
            w = 0
            for i, b in enumerate(col):
                w |= b << i
            words.append(literal_stream([w]))
        _check(G, words, r, range(0, len(cols) + 2), variants=_variants(G.lib()), label=name)


def test_random_small_all_variants(G):
    rng = np.random.default_rng(101)
    E = G.lib()
    for case in range(30):
        N = int(rng.integers(1, 13))
        r = int(rng.choice([1, 63, 64, 65, 1000, TW_ROWS - 1, TW_ROWS, TW_ROWS + 1,
                            3 * TW_ROWS + 4321, 5 * TW_ROWS]))
        model = int(rng.integers(0, 2))
        keys = [D.key(7000 + case, k) for k in range(N)]
        if model == D.IID:
            streams = D.bitmaps(D.IID, rng.choice([0.001, 0.05, 0.5]), 0.0, r, keys,
                                noncanon=bool(rng.integers(0, 2)))
        else:
            streams = D.bitmaps(D.MARKOV, float(rng.choice([32.0, 300.0, 5000.0])),
                                float(rng.choice([64.0, 512.0, 20000.0])), r, keys, noncanon=bool(rng.integers(0, 2)))
        Ts = sorted({0, 1, N, N + 1, int(rng.integers(1, N + 1))})
        _say(f"case {case}: N={N} r={r} model={model} Ts={Ts}")
        _check(G, streams, r, Ts, variants=_variants(E), label=f"case{case}")


def test_long_runs_across_tiles(G):
    """Fills and dirty runs spanning many tiles; markers closed several tiles later."""
    r = 7 * TW_ROWS + 100
    U = (r + 63) // 64
    E = G.lib()
    rng = np.random.default_rng(3)
    streams = []
    # one-fill of 3.5 tiles, zero-fill, dirty run of 1.5 tiles, one-fill to the end
    a, b = 7 * TW // 2, 39 * TW // 8 + 8
    c = b + 3 * TW // 2
    d = np.zeros(U, dtype=np.uint64)
    d[: a] = np.uint64(2**64 - 1)
    d[b: c] = rng.integers(1, 2**63, size=c - b, dtype=np.uint64)
    d[c:] = np.uint64(2**64 - 1)
    d[-1] &= np.uint64((1 << (r % 64)) - 1)
    streams.append(O.encode(d, r))
    # all ones
    d1 = np.full(U, 2**64 - 1, dtype=np.uint64); d1[-1] &= np.uint64((1 << (r % 64)) - 1)
    streams.append(O.encode(d1, r))
    # all zeros
    streams.append(O.encode(np.zeros(U, dtype=np.uint64), r))
    # the same bitmap as mixed non-canonical stream
    streams.append(mixed_stream(d, rng))
    # a single-marker dirty bitmap (every word a literal)
    dl = rng.integers(1, 2**63, size=U, dtype=np.uint64); dl[-1] &= np.uint64((1 << (r % 64)) - 1)
    streams.append(O.encode(dl, r))
    for subset in ([0], [1], [2], [0, 1], [0, 2], [0, 3], [4], [0, 4], [1, 4], [0, 1, 2, 3, 4], [2, 2, 2]):
        ss = [streams[i] for i in subset]
        _check(G, ss, r, range(0, len(ss) + 2), variants=_variants(E), label=f"subset{subset}")


def test_duplicates_and_permutation(G):
    r = 2 * TW_ROWS + 77
    keys = [D.key(4242, k) for k in range(6)]
    streams = D.bitmaps(D.MARKOV, 40.0, 200.0, r, keys)
    bms = G.register(streams, r)
    for T in range(1, 7):
        a = G.gpu_threshold(bms, T)
        b = G.gpu_threshold(bms[::-1], T)
        c = G.gpu_threshold(bms + bms, 2 * T)
        assert np.array_equal(a, b) and np.array_equal(a, c)
    for b_ in bms:
        b_.release()


def test_config1_full(G):
    w = D.config1()
    q = w.queries[0]
    _check(G, [w.streams[i] for i in q.idx], w.n_bits, [q.T, 1, 2, 8], variants=_variants(G.lib()), label="c1")


def test_config2_reduced(G):
    w = D.config2(n_bits=1 << 20, n=64)
    _check(G, w.streams, w.n_bits, [2, 32, 63, 1, 64], variants=_variants(G.lib())[:3], label="c2-2^20")


def test_errors_and_bounds(G):
    E = G.lib()
    r = 1000
    good = literal_stream([1] * 16)
    with pytest.raises(E.EwahError) as e:
        E.register_many([np.array([marker(0, 1, 5), 1, 2], dtype=np.uint64)], r)
    assert e.value.code == E.EFORMAT
    # many streams built in parallel: the lowest failing index is the one reported
    many = [good] * 40
    many[31] = np.array([marker(0, 1, 5), 1, 2], dtype=np.uint64)   # ends inside its literal run
    many[17] = np.array([marker(0, 3, 0)], dtype=np.uint64)          # covers 3 of 16 words
    with pytest.raises(E.EwahError) as e:
        E.register_many(many, r)
    assert e.value.code == E.EFORMAT and "bitmap 17:" in str(e.value), str(e.value)
    bms = G.register([good], r)
    out, out_n, cap = G.alloc_out(r, 10)
    with pytest.raises(E.EwahError) as e:
        E.threshold(bms, 1, out.data_ptr(), 0, out_n.data_ptr())
    assert e.value.code == E.ENOSPC
    other = G.register([literal_stream([1] * 2)], 100)
    with pytest.raises(E.EwahError) as e:
        E.threshold(bms + other, 1, out.data_ptr(), cap, out_n.data_ptr())
    assert e.value.code == E.EINVAL
    for b in bms + other:
        b.release()
    assert E.output_bound(0, 5) == 0
    assert E.output_bound(64 * 10, 3) == 4
    assert E.output_bound(64 * 10, 100) == 11


def test_batched_matches_plain_and_oracle(G):
    import torch
    E = G.lib()
    n_bits = 3 * TW_ROWS + 999
    pool_n = 120
    d = D.pool_densities(pool_n, seed=999)
    keys = [D.key(12345, k) for k in range(pool_n)]
    pool = D.bitmaps(D.IID, d, 0.0, n_bits, keys)
    bms = E.register_many(pool, n_bits)
    qs = D.queries(777, 40, pool_n, 2, 40)
    outs, ns, caps = [], [], []
    for q in qs:
        o, n, c = G.alloc_out(n_bits, int(sum(len(pool[i]) for i in q.idx)))
        outs.append(o); ns.append(n); caps.append(c)
    vs = _variants(E)
    variants = [vs[i % len(vs)] for i in range(len(qs))]
    batch = E.Batch(bms, [(q.idx, q.T) for q in qs], [o.data_ptr() for o in outs], caps,
                    [n.data_ptr() for n in ns], variants=variants, use_graph=True)
    wants = [O.threshold([pool[i] for i in q.idx], n_bits, q.T, want_hist=False)[0] for q in qs]
    for pre in (False, True):   # without and with the bounds pre-pass
        batch.set_prepass(pre)
        for rep in range(3):
            for o in outs:
                o.zero_()
            batch.run()
            torch.cuda.synchronize()
            x = torch.ones(1000, device="cuda").sum()   # eager work between replays
            torch.cuda.synchronize()
            assert E.device_errors() == 0
            for i, q in enumerate(qs):
                got = G.fetch(outs[i], ns[i])
                assert np.array_equal(got, wants[i]), (pre, rep, i)
    # eager (no graph) and grid change
    batch.set_grid(7)
    batch.run()
    for i in range(len(qs)):
        assert np.array_equal(G.fetch(outs[i], ns[i]), wants[i])
    batch.free()
    nb = E.Batch(bms, [(q.idx, q.T) for q in qs], [o.data_ptr() for o in outs], caps,
                 [n.data_ptr() for n in ns], use_graph=False)
    nb.run()
    for i in range(len(qs)):
        assert np.array_equal(G.fetch(outs[i], ns[i]), wants[i])
    nb.free()
    # plain path for a few of them
    for i in range(0, len(qs), 7):
        got = G.gpu_threshold([bms[j] for j in qs[i].idx], qs[i].T)
        assert np.array_equal(got, wants[i])
    assert E.device_errors() == 0
    for b in bms:
        b.release()


def test_single_query_many_tiles(G):
    """A single threshold query with more tiles than there are resident workgroups runs as a
    batch of one on the persistent kernel (staged tiles, scan, placement): every variant and
    T from 0 to N + 1, fills spanning tiles, a ragged tail, and repeated calls on one stream
    (device epochs of that path)."""
    E = G.lib()
    n_bits = 2100 * TW_ROWS + 777      # 2,101 tiles: above the resident workgroups of the kernel
    keys = [D.key(8800, k) for k in range(5)]
    streams = (D.bitmaps(D.IID, [0.002, 0.03], 0.0, n_bits, keys[:2]) +
               D.bitmaps(D.MARKOV, [3000.0, 64.0, 20000.0], [9000.0, 900.0, 40000.0], n_bits, keys[2:]))
    _check(G, streams, n_bits, range(0, len(streams) + 2), variants=_variants(E), label="many tiles")


def test_prepared_inputs_match_lists(G):
    """ewahthr.Inputs (handles marshalled once) gives the same results as a list of bitmaps
    in every query function."""
    E = G.lib()
    n_bits = 3 * TW_ROWS + 17
    streams = D.bitmaps(D.IID, [0.01, 0.2, 0.05, 0.3], 0.0, n_bits, [D.key(8900, k) for k in range(4)])
    bms = G.register(streams, n_bits)
    try:
        ins = E.Inputs(bms)
        for T in (1, 2, 4):
            assert np.array_equal(G.gpu_threshold(ins, T), G.gpu_threshold(bms, T)), T
        assert np.array_equal(E.count_histogram(ins), E.count_histogram(bms))
        out, out_n, cap = G.alloc_out(n_bits, sum(len(s) for s in streams))
        assert E.opt_threshold(ins, 5, out.data_ptr(), cap, out_n.data_ptr()) == \
            E.opt_threshold(bms, 5, out.data_ptr(), cap, out_n.data_ptr())
    finally:
        for b in bms:
            b.release()


def test_single_query_around_the_switch(G):
    """512 tiles (one per resident workgroup: look-back kernel) and 513 tiles (batch of one), on
    non-canonical input streams."""
    E = G.lib()
    for tiles in (512, 513):
        n_bits = (tiles - 1) * TW_ROWS + 4097
        # non-canonical but well-formed streams (split runs, empty markers, fill-valued literals)
        streams = D.bitmaps(D.MARKOV, 32.0, 512.0, n_bits, [D.key(8810 + tiles, k) for k in range(6)],
                            noncanon=True)
        _check(G, streams, n_bits, (0, 1, 2, 4, 7), variants=(0, E.variant_code(False, 0, 0),
                                                            E.variant_code(False, 8, 8, looped=True)),
               label=f"{tiles} tiles")


def test_slots_inline_and_uploaded(G):
    """Threshold queries of up to 256 inputs pass their slots in the kernel arguments, wider
    ones upload them: 255, 256 and 257 inputs, through the allocating and the allocation-free
    entry points, with the same inputs in reversed order (the slots differ, the result not)."""
    E = G.lib()
    n_bits = 3 * TW_ROWS + 129
    streams = D.bitmaps(D.MARKOV, 64.0, 30000.0, n_bits, [D.key(8830, k) for k in range(257)])
    bms = G.register(streams, n_bits)
    try:
        for n in (255, 256, 257):
            for T in (1, 2, 4):
                want, _ = O.threshold(streams[:n], n_bits, T, want_hist=False)
                assert np.array_equal(G.gpu_threshold(bms[:n], T), want), (n, T)
                assert np.array_equal(G.gpu_threshold(bms[:n][::-1], T), want), (n, T, "reversed")
                out, out_n, cap = G.alloc_out(n_bits, sum(len(s) for s in streams[:n]))
                E.threshold_noalloc(bms[:n], T, out.data_ptr(), cap, out_n.data_ptr())
                assert np.array_equal(G.fetch(out, out_n), want), (n, T, "noalloc")
        assert E.device_errors() == 0
    finally:
        for b in bms:
            b.release()


def _bits_to_stream(bits):
    """Row i = character / element i (the walk-throughs list rows left to right)."""
    w = 0
    for i, b in enumerate(bits):
        w |= int(b) << i
    return literal_stream([w])


def _stream_rows(words, r):
    d = O.decode(words, r)
    return [int((int(d[i // 64]) >> (i % 64)) & 1) for i in range(r)]


def test_golden_walkthroughs_on_the_gpu(G):
    """The paper's printed walk-throughs through the GPU path: Looped (Section 6.2) at T = 1
    and 2, BSTM (Section 5.3.1) at T = 2 and its slices A1 (odd count) and A2 (count in
    [2, 3]) as symmetric functions, the Hamming-weight figure's slices and histogram, and the
    Section 2 example as threshold and opt-threshold; every threshold under every variant."""
    E = G.lib()
    lp = golden("looped_walkthrough.json")
    bm = golden("bstm_walkthrough.json")
    hw = golden("hamming_weight.json")
    fx = golden("formulation_example.json")

    def run(bitmaps, r, check):
        bms = G.register([_bits_to_stream(b) for b in bitmaps], r)
        try:
            check(bms)
        finally:
            for b in bms:
                b.release()

    def thr(bms, T, v=0):
        return _stream_rows(G.gpu_threshold(bms, T, variant=v), bms[0].n_bits)

    def sym(bms, f):
        out, out_n, cap = G.alloc_out(bms[0].n_bits, sum(b.n_words for b in bms))
        E.symmetric(bms, f, out.data_ptr(), cap, out_n.data_ptr())
        return _stream_rows(G.fetch(out, out_n), bms[0].n_bits)

    as_list = lambda s: [int(c) for c in s]

    def looped(bms):
        for v in _variants(E):
            assert thr(bms, 1, v) == as_list(lp["C1"]) and thr(bms, 2, v) == as_list(lp["C2"]), v
    run(lp["bitmaps"], lp["r"], looped)

    def bstm(bms):
        for v in _variants(E):
            assert thr(bms, bm["T"], v) == as_list(bm["expected"]), v
        assert sym(bms, [0, 1, 0, 1]) == as_list(bm["A1"])
        assert sym(bms, [0, 0, 1, 1]) == as_list(bm["A2"])
    run(bm["bitmaps"], bm["r"], bstm)

    cols = [[row[k] for row in hw["rows"]] for k in range(3)]   # bitmap k = column k of the rows

    def hamming(bms):
        assert sym(bms, [0, 1, 0, 1]) == hw["A1"] and sym(bms, [0, 0, 1, 1]) == hw["A2"]
        want = [sum(1 for w in hw["weight"] if w == c) for c in range(4)]
        assert E.count_histogram(bms).tolist() == want
    run(cols, len(hw["rows"]), hamming)

    r = fx["r"]
    sets = [[1 if i in s else 0 for i in range(r)] for s in fx["sets"]]

    def formulation(bms):
        for T, rows in fx["expected"].items():
            want = [1 if i in rows else 0 for i in range(r)]
            for v in _variants(E):
                assert thr(bms, int(T), v) == want, (T, v)
        out, out_n, cap = G.alloc_out(r, sum(b.n_words for b in bms))
        assert E.opt_threshold(bms, 1, out.data_ptr(), cap, out_n.data_ptr()) == 2
        assert _stream_rows(G.fetch(out, out_n), r) == [1 if i in fx["expected"]["2"] else 0 for i in range(r)]
    run(sets, r, formulation)
