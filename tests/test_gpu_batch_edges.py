"""Batched path at the edges of the threshold's range and of the planner's limits (needs an
MI355X).

* T = 0 (every row), T = N + 1 and larger (no row) and N = 1 (the input itself) inside a
  batch whose other queries do real work, on every counter variant and every build of
  the persistent kernel (4..7 windows per wavefront batch), against the oracle;
* the planner sums (query, tile) items in 64 bits and rejects a batch of 2^31 or more
  items before it allocates anything (a 32-bit sum would wrap and size the tile states
  too small);
* inputs built so that the quarter-word bounds leave every word in play and the 8-row
  bounds settle whole tiles, with a hot spot where neither may prune;
* a batch whose items split into whole queries per XCD share, so that the bounds pre-pass
  takes them in blocks of tiles across queries, with a ragged last block.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1402_4466_amd import datagen as D
from tests.ewah_test_util import marker

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def G():
    from tests import gpu_util
    gpu_util.lib()
    return gpu_util


def test_batched_trivial_thresholds_and_single_inputs(G):
    import torch
    E = G.lib()
    n_bits = 2 * 512 * 64 + 321            # two full tiles and a ragged one
    pool_n = 24
    d = D.pool_densities(pool_n, seed=4242)
    pool = D.bitmaps(D.IID, d, 0.0, n_bits, [D.key(4242, k) for k in range(pool_n)])
    bms = E.register_many(pool, n_bits)
    rng = np.random.default_rng(4242)
    qs = []
    for i in range(48):
        n = 1 if i % 4 == 0 else int(rng.integers(2, 12))
        idx = rng.choice(pool_n, size=n, replace=False).astype(np.uint32)
        kind = i % 6
        T = {0: 0, 1: n + 1, 2: n + 7, 3: 1, 4: n, 5: int(rng.integers(1, n + 1))}[kind]
        qs.append((idx, T))
    codes = [0, E.variant_code(False, 0, 0), E.variant_code(True, 255, 255), E.variant_code(False, 8, 8, looped=True)]
    outs, ns, caps = [], [], []
    for idx, _ in qs:
        o, n, c = G.alloc_out(n_bits, int(sum(len(pool[i]) for i in idx)))
        outs.append(o); ns.append(n); caps.append(c)
    wants = [O.threshold([pool[i] for i in idx], n_bits, T, want_hist=False)[0] for idx, T in qs]
    batch = E.Batch(bms, qs, [o.data_ptr() for o in outs], caps, [n.data_ptr() for n in ns], use_graph=True)
    try:
        for v, wb, pre in [(c, w, p) for c in codes for w in (4, 5, 6, 7) for p in (False, True)]:
            batch.set_variants(np.full(len(qs), v, dtype=np.uint32))
            batch.set_win_batch(wb)
            batch.set_prepass(pre)
            for rep in range(2):
                _say(f"batched edges: variant {v:#x}, {wb} windows per batch, pre-pass {pre}, replay {rep}")
                for o in outs:
                    o.fill_(-1)
                batch.run()
                torch.cuda.synchronize()
                assert E.device_errors() == 0
                for i, (idx, T) in enumerate(qs):
                    got = G.fetch(outs[i], ns[i])
                    assert np.array_equal(got, wants[i]), (v, pre, rep, i, len(idx), T)
    finally:
        batch.free()
        for b in bms:
            b.release()


def test_batch_plan_rejects_item_overflow(G):
    import torch
    E = G.lib()
    # one all-zero bitmap of 2^30 words: 2^21 tiles per query; 2,048 such queries hold 2^32
    # items, 1,024 already reach 2^31
    U = 1 << 30
    n_bits = U * 64
    bms = E.register_many([np.array([marker(0, U, 0)], dtype=np.uint64)], n_bits)
    cap = E.output_bound(n_bits, 1)
    assert cap == 2
    nq = 2048
    out = torch.zeros(nq * cap, dtype=torch.int64, device="cuda")
    out_n = torch.zeros(nq, dtype=torch.int64, device="cuda")
    try:
        with pytest.raises(E.EwahError) as e:
            E.Batch(bms, [([0], 1)] * nq, [out.data_ptr() + 8 * cap * i for i in range(nq)], [cap] * nq,
                    [out_n.data_ptr() + 8 * i for i in range(nq)], use_graph=False)
        assert e.value.code == E.EINVAL and "too many tiles" in str(e.value), str(e.value)
        assert E.device_errors() == 0
    finally:
        for b in bms:
            b.release()


def test_eight_row_bounds_settle_what_quarters_cannot(G):
    """Inputs 0-1 hold ones only in rows 0-7 of every word, inputs 2-3 only in rows 8-15: at
    T = 3 each word's first quarter is touched by four inputs (the quarter bounds prune nothing)
    but each 8-row group by two (the 8-row bounds settle the tile). Input 4 adds rows 0-7 of
    some words of the second tile (counts reach 3 there: those words must not be pruned), and
    input 5 a few rows 48-63. Single queries and batches, every gate, against the oracle."""
    import torch
    E = G.lib()
    TWW = 512
    U = 3 * TWW + 5                             # three tiles and a ragged one
    n_bits = U * 64 - 17
    rng = np.random.default_rng(8080)
    def words(mask_fn):
        w = np.zeros(U, dtype=np.uint64)
        for i in range(U):
            w[i] = np.uint64(mask_fn(i))
        if n_bits % 64:
            w[-1] &= np.uint64((1 << (n_bits % 64)) - 1)
        return w
    lo = lambda: int(rng.integers(1, 256))
    dense = [words(lambda i: lo()), words(lambda i: lo()),
             words(lambda i: lo() << 8), words(lambda i: lo() << 8),
             words(lambda i: lo() if TWW + 100 <= i < TWW + 140 else 0),
             words(lambda i: (lo() << 48) if i % 97 == 0 else 0)]
    streams = [O.encode(d, n_bits) for d in dense]
    bms = G.register(streams, n_bits)
    codes = [0, E.variant_code(True, 8, 8, gate=1), E.variant_code(True, 8, 8, gate=2),
             E.variant_code(True, 128, 255, gate=1), E.variant_code(False, 0, 0)]
    try:
        for T in (2, 3, 4):
            want, _ = O.threshold(streams, n_bits, T, want_hist=False)
            for v in codes:
                assert np.array_equal(G.gpu_threshold(bms, T, variant=v), want), ("single", T, v)
            qs = [(np.arange(6, dtype=np.uint32), T), (np.array([0, 1, 2, 3], dtype=np.uint32), T),
                  (np.array([0, 2, 4], dtype=np.uint32), T)]
            wants = [O.threshold([streams[i] for i in idx], n_bits, t, want_hist=False)[0] for idx, t in qs]
            outs, ns, caps = [], [], []
            for idx, _ in qs:
                o, n, c = G.alloc_out(n_bits, int(sum(len(streams[i]) for i in idx)))
                outs.append(o); ns.append(n); caps.append(c)
            batch = E.Batch(bms, qs, [o.data_ptr() for o in outs], caps, [n.data_ptr() for n in ns], use_graph=True)
            try:
                for v, pre in [(c, p) for c in codes for p in (False, True)]:
                    batch.set_variants(np.full(len(qs), v, dtype=np.uint32))
                    batch.set_prepass(pre)
                    _say(f"8-row bounds: T={T}, variant {v:#x}, pre-pass {pre}")
                    for o in outs:
                        o.fill_(-1)
                    batch.run()
                    torch.cuda.synchronize()
                    assert E.device_errors() == 0
                    for i, (idx, t) in enumerate(qs):
                        assert np.array_equal(G.fetch(outs[i], ns[i]), wants[i]), ("batched", T, v, pre, i)
            finally:
                batch.free()
    finally:
        for b in bms:
            b.release()


def test_query_busy_times_with_and_without_prepass(G):
    """Per-query busy times (the selector's labels) of one batch with the bounds pre-pass off,
    on, and off again: every time is positive and of the order of the batch's own launch, so
    the pre-pass share is counted only when the pre-pass ran."""
    E = G.lib()
    n_bits = 4 * 512 * 64 + 77
    pool_n = 32
    d = D.pool_densities(pool_n, seed=5150)
    pool = D.bitmaps(D.IID, d, 0.0, n_bits, [D.key(5150, k) for k in range(pool_n)])
    bms = E.register_many(pool, n_bits)
    qs = [(q.idx, q.T) for q in D.queries(5151, 24, pool_n, 2, pool_n)]
    outs, ns, caps = [], [], []
    for idx, _ in qs:
        o, n, c = G.alloc_out(n_bits, int(sum(len(pool[i]) for i in idx)))
        outs.append(o); ns.append(n); caps.append(c)
    batch = E.Batch(bms, qs, [o.data_ptr() for o in outs], caps, [n.data_ptr() for n in ns], use_graph=False)
    try:
        for pre in (False, True, False):
            batch.set_prepass(pre)
            t = batch.time_queries(2)
            _say(f"busy times, pre-pass {pre}: max {t.max():.1f} us")
            assert np.all(np.isfinite(t)) and np.all(t > 0) and np.all(t < 1e5), (pre, t)
        assert E.device_errors() == 0
    finally:
        batch.free()
        for b in bms:
            b.release()


def test_prepass_block_order_with_ragged_last_block(G):
    """32 queries of 37 tiles: 1,184 items in 296 workgroups of the pre-pass, 148 items (4 whole
    queries) per XCD share, taken in blocks of 16, 16 and 5 tiles across the share's queries.
    Every output equals the oracle's with the pre-pass on and off."""
    import torch
    E = G.lib()
    n_bits = 36 * 512 * 64 + 5000          # 37 tiles, the last one ragged
    pool_n = 40
    d = D.pool_densities(pool_n, seed=6161)
    pool = D.bitmaps(D.IID, d, 0.0, n_bits, [D.key(6161, k) for k in range(pool_n)])
    bms = E.register_many(pool, n_bits)
    rng = np.random.default_rng(6161)
    qs = []
    for i in range(32):
        n = int(rng.integers(2, 16))
        idx = rng.choice(pool_n, size=n, replace=False).astype(np.uint32)
        qs.append((idx, int(rng.integers(1, n + 1))))
    outs, ns, caps = [], [], []
    for idx, _ in qs:
        o, n, c = G.alloc_out(n_bits, int(sum(len(pool[i]) for i in idx)))
        outs.append(o); ns.append(n); caps.append(c)
    wants = [O.threshold([pool[i] for i in idx], n_bits, T, want_hist=False)[0] for idx, T in qs]
    batch = E.Batch(bms, qs, [o.data_ptr() for o in outs], caps, [n.data_ptr() for n in ns], use_graph=True)
    try:
        for pre in (True, False, True):
            batch.set_prepass(pre)
            _say(f"pre-pass block order: 32 queries x 37 tiles, pre-pass {pre}")
            for o in outs:
                o.fill_(-1)
            batch.run()
            torch.cuda.synchronize()
            assert E.device_errors() == 0
            for i, (idx, T) in enumerate(qs):
                got = G.fetch(outs[i], ns[i])
                assert np.array_equal(got, wants[i]), (pre, i, len(idx), T)
    finally:
        batch.free()
        for b in bms:
            b.release()
